"""The precision workload (100 qubits, d = 4, two repetitions, chi = 64,
cutoff 1e-10) simulated on the GPU, with every overlap form checked entry by
entry against the oracle's overlaps of the same MPS (Eq. (1), Fig. 2).

Sixteen points of the two-class mixture plus near-duplicates of four of
them (K(x, x') well inside (0, 1), so the reduced-precision forms are tested
on mid-range values and not only on the diagonal and on underflowing
off-diagonal entries).  One circuit is also simulated by the oracle at the
full bond cap: same bond profile and fidelity 1 - 1e-10.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import gram as ogram
from oracle import mps as omps
from tests.gpu_util import fidelity, require_gpu

pytestmark = pytest.mark.gpu

N_POINTS, N_DUP = 16, 4
# FP64: rounding of ~m chi^3 operations; split forms: the fixed-point
# resolution 2^-31 per value and site plus the omitted digit products
# (~1e-8 at 100 sites), bounded at 1e-7; FP32: plain float operands and
# accumulators, about 2e-5 at 100 sites, bounded at 1e-4.
TOL = {"fp64": 1e-12, "split_bf16": 1e-7, "split_i8": 1e-7, "fp32": 1e-4}


@pytest.fixture(scope="module")
def batch():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    w = sd.WORKLOADS["precision"]
    X = sd.workload_features(w, N_POINTS)
    X = np.vstack([X, sd.perturb_near_duplicates(X[:N_DUP])])
    xt = torch.tensor(X, dtype=torch.float64, device="cuda")
    spec = q.CircuitSpec(w.n_qubits, w.distance, w.reps, w.coef_z, w.coef_xx, 1)
    b = q.simulate(xt, spec, w.chi, w.cutoff)
    return w, X, b


def test_precision_workload_every_form_vs_oracle(batch):
    import paper_2411_09336_amd as q
    w, X, b = batch
    inf = b.info()
    print("precision workload: max bond", inf["max_bond"], "unconverged", inf["unconverged_svds"])
    assert inf["max_bond"] == 64 and inf["unconverged_svds"] == 0
    n = len(X)
    Ko = ogram.gram([b.export(i) for i in range(n)])
    nd = Ko[np.arange(N_DUP), N_POINTS + np.arange(N_DUP)]
    print("near-duplicate K", nd)
    assert nd.min() > 0.05
    for prec, tol in TOL.items():
        K = q.gram(b, precision=prec).cpu().numpy()
        d = np.abs(K - Ko)
        print(prec, "max|dK| vs oracle", d.max(), "mean", d.mean(), "entries", n * n)
        assert d.max() < tol
        assert np.array_equal(K, K.T)


def test_precision_workload_simulation_vs_oracle(batch):
    w, X, b = batch
    dims = b.bond_dims()
    disc, deg = b.trunc_stats()
    r = omps.simulate(X[0], w.distance, w.reps, w.chi, w.cutoff, w.coef_z, w.coef_xx, routing=1)
    f = fidelity(b.export(0), r.tensors)
    print("precision circuit 0: fidelity", f, "degenerate", deg[0], r.degenerate_cuts, "max bond", r.max_bond_seen)
    assert r.degenerate_cuts == 0 and deg[0] == 0
    assert f > 1 - 1e-10
    assert list(dims[0]) == r.bond_dims
    assert abs(disc[0] - r.discarded) <= 1e-9 * max(1.0, r.discarded)
