"""Gram kernels of the FP64 and FP32 forms at bond dimensions up to 128
(Fig. 2's contraction with E in global scratch: a 128 x 128 complex E is
above one CU's LDS), against the CPU FP64 oracle.

States:
* the paper's feature-map circuit of the 165-qubit, d = 8, chi = 128
  instance of the uneven workload, on its first 18 qubits (the oracle's
  Sec. II-B simulation, routing 1, cutoff 1e-10): bonds 128 on the five
  middle cuts, 6 points plus 2 near-duplicates (mid-range K);
* 165-site random left-canonical states with bonds up to 128 and a
  perturbed copy of one of them (one mid-range entry).

Tolerances: FP64 1e-12 (rounding of ~m chi^3 FP64 operations), FP32 2e-5
(complex64 operands and FP32 accumulation over 18 sites).  The split forms
and the allocation-free entry point refuse pads above 64 (QK_ENOTSUP).
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import gram as ogram
from oracle import mps as omps
from tests import emulate_forms as ef
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

M_SLICE = 18
QK_ENOTSUP = -4


def _sim(x, chi):
    w = sd.WORKLOADS["uneven_165"]
    return omps.simulate(x, w.distance, w.reps, chi, w.cutoff, w.coef_z, w.coef_xx, routing=1).tensors


@pytest.fixture(scope="module")
def sets():
    require_gpu()
    X = sd.workload_features(sd.WORKLOADS["uneven_165"], 6)[:, :M_SLICE]
    X = np.vstack([X, sd.perturb_near_duplicates(X[:2])])
    wide = [_sim(x, 128) for x in X]
    narrow = [_sim(x, 16) for x in X[:6]]
    assert max(t.shape[2] for t in wide[0]) == 128          # saturated bonds
    rng = np.random.default_rng(21)
    a = ef.random_left_canonical(165, 128, rng)
    b = ef.random_left_canonical(165, 128, rng)
    long_ = [a, b, ef.perturbed(a, 0.002, rng)]
    return wide, narrow, long_


def test_fp64_wide_matches_oracle(sets):
    import paper_2411_09336_amd as q
    wide = sets[0]
    K_ref = ogram.gram(wide)
    off = K_ref[~np.eye(len(wide), dtype=bool)]
    assert off.max() > 0.1          # near-duplicates: mid-range entries, not only ~0
    b = q.import_batch(wide)
    assert b.info()["pad_max"] == 128
    st = {}
    K = q.gram(b, precision="fp64", stats=st).cpu().numpy()
    d = np.abs(K - K_ref).max()
    print("fp64 chi 128: max|dK|", d, "off-diagonal max", off.max(), "stats", st)
    assert st["block"] == 128
    assert d < 1e-12
    assert np.abs(np.diag(K) - 1.0).max() < 1e-12


def test_fp32_wide_matches_oracle(sets):
    import paper_2411_09336_amd as q
    wide = sets[0]
    K_ref = ogram.gram(wide)
    K = q.gram(q.import_batch(wide), precision="fp32").cpu().numpy()
    d = np.abs(K - K_ref).max()
    print("fp32 chi 128: max|dK|", d)
    assert d < 2e-5


def test_fp64_wide_165_sites(sets):
    import paper_2411_09336_amd as q
    long_ = sets[2]
    K_ref = ogram.gram(long_)
    assert 0.05 < K_ref[0, 2] < 0.95
    K = q.gram(q.import_batch(long_), precision="fp64").cpu().numpy()
    d = np.abs(K - K_ref).max()
    print("fp64 165 sites chi 128: max|dK|", d, "K[0,2]", K_ref[0, 2])
    assert d < 1e-12


def test_wide_rectangular_mixed_pads_and_blocks(sets):
    """Bra batch with pads up to 128 against a ket batch with pads 32: one
    launch of the wide kernel; a ragged upper-triangle slab of the wide set."""
    import torch

    import paper_2411_09336_amd as q
    wide, narrow, _ = sets
    K_ref = ogram.gram(wide, narrow)
    K = q.gram(q.import_batch(wide), q.import_batch(narrow), precision="fp64").cpu().numpy()
    assert K.shape == (len(wide), len(narrow))
    assert np.abs(K - K_ref).max() < 1e-12
    full = q.import_batch(wide)
    Kf = ogram.gram(wide)
    n = len(wide)
    out = torch.full((3, n), -1.0, dtype=torch.float64, device="cuda")
    q.gram_block(full, 5, 3, full, 0, n, precision="fp64", upper_only=True, out=out)
    o = out.cpu().numpy()
    for r in range(3):
        for c in range(n):
            gi = 5 + r
            if c >= gi or 5 <= c < 8:
                assert abs(o[r, c] - Kf[gi, c]) < 1e-12
            else:
                assert o[r, c] == -1.0


def test_wide_job_in_uneven_multi_launch(sets):
    """A chi = 128 job and a chi = 16 job (different batches, same launch)."""
    import torch

    import paper_2411_09336_amd as q
    wide, narrow, _ = sets
    bw, bn = q.import_batch(wide), q.import_batch(narrow)
    ow = torch.empty((len(wide), len(wide)), dtype=torch.float64, device="cuda")
    on = torch.empty((len(narrow), len(narrow)), dtype=torch.float64, device="cuda")
    st = {}
    q.gram_multi([dict(a=bw, b=bw, na=len(wide), nb=len(wide), upper_only=True, out=ow),
                  dict(a=bn, b=bn, na=len(narrow), nb=len(narrow), upper_only=True, out=on)],
                 precision="fp64", stats=st)
    assert st["block"] == 128
    assert np.abs(ow.cpu().numpy() - ogram.gram(wide)).max() < 1e-12
    assert np.abs(on.cpu().numpy() - ogram.gram(narrow)).max() < 1e-12


def test_wide_deterministic_and_tuned(sets):
    import paper_2411_09336_amd as q
    b = q.import_batch(sets[0])
    k1 = q.gram(b, precision="fp64").cpu().numpy()
    k2 = q.gram(b, precision="fp64").cpu().numpy()
    assert (k1 == k2).all()
    try:
        rep = q.autotune(b, "fp64", sample=10)
        assert rep["maxp"] == 128
        k3 = q.gram(b, precision="fp64").cpu().numpy()
        assert (k1 == k3).all()
    finally:
        q.autotune_reset()


def test_split_forms_and_noalloc_refuse_wide_pads(sets):
    import torch

    import paper_2411_09336_amd as q
    b = q.import_batch(sets[0][:2])
    for prec in ("split_bf16", "split_i8"):
        with pytest.raises(q.QKError) as e:
            q.gram(b, precision=prec)
        assert e.value.status == QK_ENOTSUP
    out = torch.zeros((2, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(q.QKError) as e:
        q.gram_block_noalloc(b, 0, 2, b, 0, 2, out, precision="fp64")
    assert e.value.status == QK_ENOTSUP
    assert (out.cpu().numpy() == 0).all()
