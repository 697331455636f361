"""Batch management and the multi-job persistent Gram launch on the GPU."""
import numpy as np
import pytest

import synthdata as sd
from oracle import gram as ogram
from oracle import mps as omps
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _oracle_mps(w, n, chi=None, seed_shift=0):
    X = sd.workload_features(w, n + seed_shift)[seed_shift:]
    return [omps.simulate(x, w.distance, w.reps, chi or w.chi, w.cutoff, w.coef_z, w.coef_xx).tensors for x in X]


def test_import_export_roundtrip():
    import paper_2411_09336_amd as q
    require_gpu()
    mpss = _oracle_mps(sd.WORKLOADS["fp32"], 3, chi=16)
    b = q.import_batch(mpss)
    for i in range(3):
        back = b.export(i)
        assert len(back) == len(mpss[i])
        for t0, t1 in zip(mpss[i], back):
            assert t0.shape == t1.shape
            assert np.array_equal(t0, t1)
    assert list(b.bond_dims()[1]) == [1] + [t.shape[2] for t in mpss[1]]


def test_gather_forms_and_errors():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    mpss = _oracle_mps(sd.WORKLOADS["fp32"], 4, chi=16)
    b = q.import_batch(mpss)
    b.pack("split_bf16")
    b.pack("split_i8")
    g = b.gather([2, 0, 2, 3], forms=("split_bf16", "split_i8"))
    idx = [2, 0, 2, 3]
    for prec in ("split_bf16", "split_i8"):
        Kg = q.gram(g, precision=prec).cpu().numpy()
        Kb = q.gram_block(b, 0, 4, b, 0, 4, precision=prec).cpu().numpy()
        for r in range(4):
            for c in range(r, 4):
                assert Kg[r, c] == Kb[idx[r], idx[c]]    # same inputs, same bits
    assert g.info()["bytes_split_i8"] == 4 * 50 * 67840      # 4 MPS x 50 sites x site block
    with pytest.raises(q.QKError) as e:
        q.gram(g, precision="fp64")
    assert e.value.status == -4                            # QK_ENOTSUP: no FP64 form
    with pytest.raises(q.QKError):
        g.export(0)
    with pytest.raises(q.QKError):
        b.gather([5])                                      # out of range


def test_gram_multi_mixed_batches_one_launch():
    """Three jobs (two qubit counts, symmetric and rectangular) in one launch
    give the same bits as separate launches and match the oracle."""
    import paper_2411_09336_amd as q
    torch = require_gpu()
    wa = sd.Workload("a", 12, 20, 1, 2, 16, 1e-10, seed=0)
    wb = sd.Workload("b", 12, 30, 3, 2, 32, 1e-10, seed=1)
    ma = _oracle_mps(wa, 9)
    mb = _oracle_mps(wb, 7)
    A = q.import_batch(ma)
    Bb = q.import_batch(mb)
    for prec, tol in (("fp64", 1e-12), ("split_bf16", 1e-7), ("split_i8", 1e-7)):
        K1 = torch.zeros((9, 9), dtype=torch.float64, device="cuda")
        K2 = torch.zeros((3, 6), dtype=torch.float64, device="cuda")
        K3 = torch.zeros((7, 7), dtype=torch.float64, device="cuda")
        q.gram_multi([dict(a=A, b=A, na=9, nb=9, upper_only=True, out=K1),
                      dict(a=A, b=A, a0=6, na=3, b0=0, nb=6, out=K2),
                      dict(a=Bb, b=Bb, na=7, nb=7, upper_only=True, out=K3)], precision=prec)
        K1s = q.gram(A, precision=prec)
        K3s = q.gram(Bb, precision=prec)
        assert torch.equal(K1, K1s) and torch.equal(K3, K3s)
        Ka = ogram.gram(ma)
        Kb = ogram.gram(mb)
        assert np.abs(K1.cpu().numpy() - Ka).max() < tol
        assert np.abs(K2.cpu().numpy() - Ka[6:9, 0:6]).max() < tol
        assert np.abs(K3.cpu().numpy() - Kb).max() < tol


def test_invalid_simulation_arguments():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    spec = q.CircuitSpec(6, 1, 1)
    x = torch.rand((3, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(q.QKError) as e:
        q.simulate(x, spec, 129, 0.0)
    assert e.value.status == -4                            # chi above 128
    x[1, 2] = float("nan")
    with pytest.raises(q.QKError) as e:
        q.simulate(x, spec, 16, 0.0)
    assert e.value.status == -1
    with pytest.raises(ValueError):
        q.simulate(torch.rand((3, 5), dtype=torch.float64, device="cuda"), spec, 16, 0.0)


def test_progress_callback_and_abort():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    spec = q.CircuitSpec(8, 2, 1)
    x = torch.rand((2, 8), dtype=torch.float64, device="cuda")
    seen = []
    b = q.simulate(x, spec, 16, 0.0, progress=lambda d, t: seen.append((d, t)) and False, every=3)
    total = b.info()["n_two_qubit_gates"]
    assert seen and seen[-1] == (total, total)
    with pytest.raises(q.QKError) as e:
        q.simulate(x, spec, 16, 0.0, progress=lambda d, t: True, every=1)
    assert e.value.status == -6                            # QK_EABORTED
