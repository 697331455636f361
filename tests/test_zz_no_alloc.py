"""mps_gram_block_noalloc: the allocation-free variant of mps_gram_block.

Called through the C ABI, it must give the same K as mps_gram_block bit for
bit (same kernels, same configuration) on two calls in a row, the second on
a smaller input (the static scratch keeps the first call's work queue, which
the second call overwrites), allocate no device memory (PyTorch's caching
allocator, the library's default, sees no new block), refuse a batch whose
packed planes are missing, and refuse a work queue larger than its scratch,
both before any launch.
"""
import ctypes

import numpy as np
import pytest

import synthdata as sd
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

FORMS = ("fp64", "fp32", "split_bf16", "split_i8")


def _sim(n, chi=16, seed_shift=0):
    import paper_2411_09336_amd as q
    torch = require_gpu()
    w = sd.WORKLOADS["fp32"]
    X = sd.workload_features(w, n + seed_shift)[seed_shift:]
    xt = torch.tensor(X, dtype=torch.float64, device="cuda")
    spec = q.CircuitSpec(w.n_qubits, w.distance, w.reps, w.coef_z, w.coef_xx, 1)
    return q.simulate(xt, spec, chi, w.cutoff)


def _noalloc(a, a0, na, b, b0, nb, upper, prec, out):
    """The entry point called directly through ctypes (no Python wrapper)."""
    import paper_2411_09336_amd as q
    from paper_2411_09336_amd import api
    lib = ctypes.CDLL(q.library_path())
    f = lib.mps_gram_block_noalloc
    I64 = ctypes.c_int64
    f.argtypes = [ctypes.c_void_p, I64, I64, ctypes.c_void_p, I64, I64, ctypes.c_int32, ctypes.c_int,
                  ctypes.c_void_p, I64, ctypes.c_void_p]
    f.restype = ctypes.c_int
    return f(a.handle, a0, na, b.handle, b0, nb, int(upper), api.Precision.of(prec), out.data_ptr(),
             out.stride(0), None)


def test_noalloc_matches_gram_block_twice():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    big = _sim(9, chi=32)
    small = _sim(4, chi=16, seed_shift=3)
    for f in FORMS:
        big.pack(f)
        small.pack(f)
    torch.cuda.synchronize()
    cases = [(big, 0, 9, 0, 9, True), (small, 1, 3, 0, 4, False)]
    for f in FORMS:
        for (bt, a0, na, b0, nb, upper) in cases:
            ref = torch.full((na, nb), -1.0, dtype=torch.float64, device="cuda")
            q.gram_block(bt, a0, na, bt, b0, nb, precision=f, upper_only=upper, out=ref)
            got = torch.full((na, nb), -1.0, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            before = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
            st = _noalloc(bt, a0, na, bt, b0, nb, upper, f, got)
            torch.cuda.synchronize()
            after = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
            assert st == 0, (f, q.api._load().qk_last_error())
            assert after == before, (f, "device allocation during the no-alloc call")
            # bit for bit, including entries neither call writes (left at -1)
            assert torch.equal(got, ref), (f, na, nb, (got - ref).abs().max().item())
            print(f, na, nb, "bit-identical", flush=True)


def test_noalloc_refuses_unpacked_and_oversized():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    b = _sim(3)
    out = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
    b.drop("split_i8")
    # planes missing: QK_ENOTSUP, nothing written
    assert _noalloc(b, 0, 3, b, 0, 3, True, "split_i8", out) == -4
    assert (out == 0).all()
    # a work queue above the 8 MiB scratch: a symmetric Gram of 33,000 MPS
    # has > 524,000 pair tiles for every tile side (8, 16, 32), so the call
    # must refuse it on the host; copies of one 1-qubit MPS keep the batch
    # small (32 KiB each), and `out` holds the whole matrix all the same
    xt = torch.tensor([[0.3]], dtype=torch.float64, device="cuda")
    one = q.simulate(xt, q.CircuitSpec(1, 1, 2), 2, 0.0)
    n = 33000
    big = one.gather([0] * n, forms=("fp64",))
    K = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    assert _noalloc(big, 0, n, big, 0, n, True, "fp64", K) == -1
    assert b"scratch" in q.api._load().qk_last_error()
    assert not K.any()
