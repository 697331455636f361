"""Two-qubit gates applied through their operator-Schmidt decomposition
(gate_split = 1; the gate SVD before application, footnote of Sec. III-A).

* Untruncated (cutoff 0), features with exact zero Rxx angles: the GPU
  states equal the state vector; with the flag no bond exceeds the oracle's
  split simulation, and the cut bonds of the memory trace never exceed those
  of the same GPU run without the flag.
* Truncated (the fp32 workload's circuit, cutoff 1e-10, bond cap 16): the GPU
  states with the flag match the oracle's split simulation (fidelity
  1 - 1e-10, equal bonds, equal discarded weights) for every circuit with no
  near-degenerate cut.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import mps as omps
from oracle import statevector as sv
from tests.gpu_util import fidelity, require_gpu

pytestmark = pytest.mark.gpu


def _sim(X, d, reps, chi, cutoff, coef_z=2.0, coef_xx=2.0, routing=0, gate_split=1, trace=False):
    import paper_2411_09336_amd as q
    torch = require_gpu()
    xt = torch.tensor(X, dtype=torch.float64, device="cuda")
    spec = q.CircuitSpec(X.shape[1], d, reps, coef_z, coef_xx, routing, gate_split)
    if trace:
        return q.simulate_trace(xt, spec, chi, cutoff)
    return q.simulate(xt, spec, chi, cutoff)


@pytest.mark.parametrize("m,d,reps,routing", [(6, 3, 2, 0), (7, 2, 2, 1), (8, 1, 2, 0), (9, 4, 1, 1)])
def test_untruncated_with_zero_angles(m, d, reps, routing):
    rng = np.random.default_rng(100 + m + d)
    X = rng.random((4, m))
    X[:, 1] = 1.0          # every Rxx on qubit 1 has angle 0: an identity gate
    X[0, m - 2] = 0.0
    b, tr = _sim(X, d, reps, 64, 0.0, routing=routing, trace=True)
    b0, tr0 = _sim(X, d, reps, 64, 0.0, routing=routing, gate_split=0, trace=True)
    dims = b.bond_dims()
    tr, tr0 = tr.cpu().numpy(), tr0.cpu().numpy()
    for i in range(len(X)):
        psi = omps.to_statevector(b.export(i))
        ref = sv.state_logical(X[i], d, reps, 2.0, 2.0)
        assert abs(abs(np.vdot(psi, ref)) ** 2 - 1) < 1e-12
        r = omps.simulate(X[i], d, reps, 64, 0.0, routing=routing, gate_split=True)
        print(i, "gpu", list(dims[i]), "oracle", r.bond_dims)
        assert all(a <= b_ for a, b_ in zip(dims[i], r.bond_dims))
        assert (tr[i, :, 0] <= tr0[i, :, 0]).all()


def test_truncated_vs_oracle_split():
    w = sd.WORKLOADS["fp32"]
    n, chi = 4, 16
    X = sd.workload_features(w, n)
    b = _sim(X, w.distance, w.reps, chi, w.cutoff, w.coef_z, w.coef_xx)
    dims = b.bond_dims()
    disc, deg = b.trunc_stats()
    compared = 0
    for i in range(n):
        r = omps.simulate(X[i], w.distance, w.reps, chi, w.cutoff, w.coef_z, w.coef_xx, gate_split=True)
        f = fidelity(b.export(i), r.tensors)
        print("split", i, "fidelity", f, "bonds equal", list(dims[i]) == r.bond_dims, "disc", disc[i], r.discarded)
        if r.degenerate_cuts == 0 and deg[i] == 0:
            compared += 1
            assert f > 1 - 1e-10
            assert list(dims[i]) == r.bond_dims
            assert abs(disc[i] - r.discarded) <= 1e-9 * max(1.0, r.discarded)
    print("split: circuits compared", compared, "of", n)
    assert compared >= n // 2


def test_gate_split_flag_is_validated():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    xt = torch.zeros((1, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(q.QKError) as e:
        q.simulate(xt, q.CircuitSpec(4, 1, 1, gate_split=2), 8, 0.0)
    assert e.value.status == -1
