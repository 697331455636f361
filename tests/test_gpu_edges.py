"""Edge cases of the simulation and the Gram on the GPU.

Empty batches (n = 0), the shortest chains (1 to 4 qubits, zero repetitions,
an interaction distance beyond the chain) against the statevector, the
strongest truncation (chi = 1) against the oracle, identical points
(K = 1 off the diagonal), and a Gram between two batches with different bond
profiles (different chi) against the oracle's overlaps.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import gram as ogram
from oracle import mps as omps
from oracle import statevector as sv
from tests.gpu_util import fidelity, require_gpu

pytestmark = pytest.mark.gpu


def _sim(X, m, d, reps, chi, cutoff, routing=0, cz=2.0, cxx=2.0):
    import paper_2411_09336_amd as q
    torch = require_gpu()
    spec = q.CircuitSpec(m, d, reps, cz, cxx, routing)
    xt = torch.tensor(np.asarray(X, dtype=np.float64).reshape(len(X), m), device="cuda")
    return q.simulate(xt, spec, chi, cutoff)


def test_empty_batches():
    import paper_2411_09336_amd as q
    b = _sim(np.zeros((0, 6)), 6, 2, 1, 8, 0.0)
    assert b.n == 0
    c = _sim(sd.make_uniform(3, 6, seed=1), 6, 2, 1, 8, 0.0)
    for prec in ("fp64", "split_bf16", "split_i8"):
        assert tuple(q.gram(b, precision=prec).shape) == (0, 0)
        assert tuple(q.gram(b, c, precision=prec).shape) == (0, 3)
        assert tuple(q.gram(c, b, precision=prec).shape) == (3, 0)


@pytest.mark.parametrize("m,d,reps", [(1, 1, 2), (2, 1, 1), (2, 5, 2), (3, 7, 1), (4, 0, 2), (3, 2, 0)])
def test_shortest_chains_vs_statevector(m, d, reps):
    import paper_2411_09336_amd as q
    X = sd.make_uniform(5, m, seed=10 * m + d)
    b = _sim(X, m, d, reps, 16, 0.0)
    states = np.array([sv.state_logical(x, d, reps, 2.0, 2.0) for x in X])
    for i in range(len(X)):
        psi = omps.to_statevector(b.export(i))
        assert abs(abs(np.vdot(psi, states[i])) ** 2 - 1) < 1e-12
    K_sv = sv.gram_from_states(states)
    for prec, tol in (("fp64", 1e-12), ("split_bf16", 1e-7), ("split_i8", 1e-7)):
        K = q.gram(b, precision=prec).cpu().numpy()
        print(m, d, reps, prec, "max|dK|", np.abs(K - K_sv).max())
        assert np.abs(K - K_sv).max() < tol


def test_chi_one_truncation_vs_oracle():
    X = sd.make_uniform(4, 10, seed=3)
    b = _sim(X, 10, 2, 2, 1, 0.0)
    dims = b.bond_dims()
    disc, deg = b.trunc_stats()
    assert b.info()["max_bond"] == 1
    compared = 0
    for i in range(len(X)):
        r = omps.simulate(X[i], 2, 2, 1, 0.0, 2.0, 2.0)
        print("chi 1", i, "fidelity", fidelity(b.export(i), r.tensors), "degenerate", deg[i], r.degenerate_cuts)
        assert list(dims[i]) == r.bond_dims == [1] * 11
        if deg[i] == 0 and r.degenerate_cuts == 0:
            compared += 1
            assert fidelity(b.export(i), r.tensors) > 1 - 1e-10
            assert abs(disc[i] - r.discarded) <= 1e-9 * max(1.0, r.discarded)
    print("chi 1: circuits compared", compared, "of", len(X))
    assert compared >= 1


def test_identical_points():
    import paper_2411_09336_amd as q
    w = sd.WORKLOADS["fp32"]
    x = sd.workload_features(w, 2)
    X = np.vstack([x[0], x[1], x[0], x[0]])
    b = _sim(X, w.n_qubits, w.distance, w.reps, 32, w.cutoff)
    e0 = b.export(0)
    for j in (2, 3):   # every circuit of a batch follows the same arithmetic
        assert all(np.array_equal(s, t) for s, t in zip(e0, b.export(j)))
    for prec, tol in (("fp64", 1e-12), ("split_i8", 1e-7)):
        K = q.gram(b, precision=prec).cpu().numpy()
        assert abs(K[0, 2] - 1) < tol and abs(K[0, 3] - 1) < tol and abs(K[2, 3] - 1) < tol
        assert abs(K[0, 1] - K[2, 1]) < tol


def test_gram_between_different_bond_profiles():
    import paper_2411_09336_amd as q
    w = sd.WORKLOADS["fp32"]
    X = sd.workload_features(w, 4)
    a = _sim(X[:3], w.n_qubits, w.distance, w.reps, 4, w.cutoff)
    c = _sim(X[1:], w.n_qubits, w.distance, w.reps, 32, w.cutoff)
    assert a.info()["max_bond"] == 4 and c.info()["max_bond"] > 4
    Ko = np.array([[abs(ogram.overlap(a.export(i), c.export(j))) ** 2 for j in range(3)] for i in range(3)])
    for prec, tol in (("fp64", 1e-12), ("split_i8", 1e-7)):
        K = q.gram(a, c, precision=prec).cpu().numpy()
        print(prec, "max|dK|", np.abs(K - Ko).max())
        assert np.abs(K - Ko).max() < tol
