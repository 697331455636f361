"""GPU Gram kernels vs the CPU FP64 oracle, on oracle-simulated MPS.

The MPS are produced by the oracle, uploaded through mps_batch_import, and
K is computed on the GPU in FP64, FP32 and split-BF16; the oracle computes
K from the same tensors.  Tolerances: FP64 1e-12 (rounding of ~m * chi^3
operations in FP64); FP32 1e-5 and split-BF16 1e-5 here (the full-scale
target for split-BF16 is |dK| <= 1e-6 against FP64, checked in the bench).
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import gram as ogram
from oracle import mps as omps
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _oracle_batch(w, n, chi=None, extra_dup=0):
    X = sd.workload_features(w, n)
    if extra_dup:
        X = np.vstack([X, sd.perturb_near_duplicates(X[:extra_dup])])
    return [omps.simulate(x, w.distance, w.reps, chi or w.chi, w.cutoff, w.coef_z, w.coef_xx).tensors for x in X]


@pytest.fixture(scope="module")
def small_sets():
    torch = require_gpu()
    tiny = _oracle_batch(sd.WORKLOADS["tiny"], 20)
    mid = _oracle_batch(sd.WORKLOADS["fp32"], 10, chi=32, extra_dup=4)
    return tiny, mid


@pytest.mark.parametrize("which", [0, 1])
def test_gram_fp64_matches_oracle(small_sets, which):
    import paper_2411_09336_amd as q
    mpss = small_sets[which]
    K_ref = ogram.gram(mpss)
    b = q.import_batch(mpss)
    K = q.gram(b, precision="fp64").cpu().numpy()
    print("fp64 max|dK|", np.abs(K - K_ref).max())
    assert np.abs(K - K_ref).max() < 1e-12
    assert np.allclose(np.diag(K), 1.0, atol=1e-12)


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-5), ("split_bf16", 1e-7), ("split_i8", 1e-7)])
def test_gram_reduced_precision(small_sets, prec, tol):
    """FP32: plain complex64 operands and FP32 accumulation (error grows with
    chain length; 2e-5 bounds 50 sites).  Split-BF16: fixed-point slices with
    an exact leading-slice accumulator, ~1e-8 at 100 sites."""
    import paper_2411_09336_amd as q
    for mpss in small_sets:
        K_ref = ogram.gram(mpss)
        b = q.import_batch(mpss)
        K = q.gram(b, precision=prec).cpu().numpy()
        d = np.abs(K - K_ref)
        print(prec, "max|dK|", d.max(), "mean", d.mean())
        assert d.max() < tol


def test_gram_rectangular_and_blocks(small_sets):
    import paper_2411_09336_amd as q
    import torch
    mpss = small_sets[1]
    a = q.import_batch(mpss[:5])
    b = q.import_batch(mpss[5:])
    K_ref = ogram.gram(mpss[:5], mpss[5:])
    K = q.gram(a, b, precision="fp64").cpu().numpy()
    assert np.abs(K - K_ref).max() < 1e-12
    full = q.import_batch(mpss)
    n = len(mpss)
    Kf = ogram.gram(mpss)
    # a slab of rows with the upper-triangle filter
    out = torch.full((4, n), -1.0, dtype=torch.float64, device="cuda")
    q.gram_block(full, 3, 4, full, 0, n, precision="fp64", upper_only=True, out=out)
    o = out.cpu().numpy()
    for r in range(4):
        for c in range(n):
            gi = 3 + r
            if c >= gi or 3 <= c < 3 + 4:
                # contracted (j >= i) or mirrored from inside the block
                assert abs(o[r, c] - Kf[gi, c]) < 1e-12
            else:
                assert o[r, c] == -1.0


def test_gauge_invariance_fp64():
    """Inserting U U^H on every bond of the ket leaves <a|b> unchanged."""
    import paper_2411_09336_amd as q
    require_gpu()
    rng = np.random.default_rng(3)
    mpss = _oracle_batch(sd.WORKLOADS["fp32"], 3, chi=32)
    b = mpss[1]
    g = []
    Us = [np.eye(1)]
    for l in range(len(b) - 1):
        D = b[l].shape[2]
        z = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
        u, _ = np.linalg.qr(z)
        Us.append(u)
    Us.append(np.eye(1))
    for l, t in enumerate(b):
        g.append(np.einsum("ab,bsc,cd->asd", Us[l].conj().T, t, Us[l + 1]))
    batch = q.import_batch([mpss[0], b, g])
    K = q.gram(batch, precision="fp64").cpu().numpy()
    assert abs(K[0, 1] - K[0, 2]) < 1e-12
    assert abs(K[1, 2] - 1.0) < 1e-12


def test_gram_deterministic(small_sets):
    import paper_2411_09336_amd as q
    b = q.import_batch(small_sets[1])
    for prec in ("fp64", "split_bf16", "split_i8"):
        k1 = q.gram(b, precision=prec).cpu().numpy()
        k2 = q.gram(b, precision=prec).cpu().numpy()
        assert (k1 == k2).all()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["split_bf16", "split_i8"])
def test_split_values_at_top_of_exponent_range(prec):
    """Product states whose amplitudes sit just below 1, just below 1/2 and
    at the int8 form's exponent margin 128/129: after fixed-point rounding
    they reach the largest codes, where a carry mistake would flip a sign or
    overflow the leading digit.  Self-overlaps must be 1 and every entry must
    match the oracle."""
    import paper_2411_09336_amd as q
    require_gpu()
    m = 24
    mps = []
    r = 128.0 / 129.0
    tops = [1.0 - 2.0 ** -40, 1.0 - 2.0 ** -33, 0.5 - 2.0 ** -45, 1.0 - 2.0 ** -31,
            r * (1.0 - 2.0 ** -35), r * (1.0 + 2.0 ** -35), 0.5 * r]
    for k, top in enumerate(tops):
        site = []
        for l in range(m):
            a = top if (l + k) % 3 else np.sqrt(0.5)
            b = np.sqrt(max(1.0 - a * a, 0.0)) * np.exp(1j * 0.3 * (l + 1) * (k + 1))
            if (l + k) % 3 and top < 0.75:
                # amplitude just below 1/2 on |0>, the rest on |1>
                a, b = top, np.sqrt(1.0 - top * top)
            t = np.zeros((1, 2, 1), dtype=np.complex128)
            t[0, 0, 0], t[0, 1, 0] = a, b
            site.append(t)
        mps.append(site)
    b = q.import_batch(mps)
    K = q.gram(b, precision=prec).cpu().numpy()
    Kref = ogram.gram(mps)
    # fixed-point resolution 2^-31 relative per value and site: 24 sites,
    # two operands, |K| = |<a|b>|^2 -> below 4 * 24 * 2^-31 = 4.5e-8
    assert np.abs(np.diag(K) - 1.0).max() < 4.5e-8
    assert np.abs(K - Kref).max() < 4.5e-8


@pytest.mark.gpu
def test_autotune_keeps_results_and_uses_choice(small_sets):
    """The autotuner times every configuration (block size 32 / 64 for the
    plain forms when the pads allow, pair-tile side, queues) and stores the
    fastest if it beats the default by more than 2 %; Gram results afterwards are bit-identical to the defaults (the
    configuration changes scheduling, not arithmetic)."""
    import paper_2411_09336_amd as q
    torch = require_gpu()
    b = q.import_batch(small_sets[0])            # bond dims <= 32: pads 32
    assert b.info()["pad_max"] == 32
    try:
        for prec, ncand in (("fp64", 12), ("fp32", 12), ("split_i8", 6), ("split_bf16", 6)):
            k0 = q.gram(b, precision=prec)
            rep = q.autotune(b, precision=prec, sample=16)
            print(prec, rep)
            assert rep["n_candidates"] == ncand
            assert rep["maxp"] in (32, 64) and rep["tile_side"] in (8, 16, 32) and rep["queues"] in (1, 8)
            assert rep["best_ms"] <= rep["default_ms"]
            default = (64, 16, 8 if prec == "split_i8" else 1)
            if (rep["maxp"], rep["tile_side"], rep["queues"]) != default:
                # a configuration replaces the default only when clearly faster
                assert rep["best_ms"] < 0.98 * rep["default_ms"]
            k1 = q.gram(b, precision=prec)
            assert torch.equal(k0, k1)
    finally:
        q.autotune_reset()
