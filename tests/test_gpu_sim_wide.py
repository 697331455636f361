"""GPU simulation with bond caps above 64 against the statevector and the
oracle (Sec. II-B truncation).  A two-site step next to a bond above 64 has
a Jacobi matrix of up to 256 x 256 and takes the wide step (columns in
global scratch); the others take the register-resident step.

* Untruncated (chi = 128, cutoff 0) on 14 qubits: the middle bond reaches
  2^7 = 128, so the wide steps run with nothing to truncate; the GPU states
  must equal the exact state, the oracle's untruncated MPS (fidelity
  1 - 1e-12).
* Truncated: the paper's feature-map circuit of the 165-qubit, d = 8,
  chi = 128 instance of the uneven workload on its first 18 qubits (bonds
  capped at 128 on the five middle cuts, cutoff 1e-10): per circuit with no
  near-degenerate cut, fidelity >= 1 - 1e-10 against the oracle's MPS, equal
  bond dimensions and discarded weights within 1e-9 relative; both routings
  and the gate-split option.
* K of the GPU states against the oracle's (FP64 and FP32 Gram).
* Graph replays bit-identical to the eager run; bond caps above 128 refused.
"""
import numpy as np
import pytest

import synthdata as sd
from oracle import gram as ogram
from oracle import mps as omps
from tests.gpu_util import fidelity, require_gpu

pytestmark = pytest.mark.gpu

M_SLICE = 18
QK_ENOTSUP = -4


def _spec(q, m, w, routing=1, gate_split=0):
    return q.CircuitSpec(m, w.distance, w.reps, w.coef_z, w.coef_xx, routing, gate_split)


def _slice(n):
    w = sd.WORKLOADS["uneven_165"]
    return w, sd.workload_features(w, n)[:, :M_SLICE]


def _compare(b, X, w, routing=1, gate_split=False):
    """Per-circuit parity with the oracle; returns the number compared."""
    dims = b.bond_dims()
    disc, deg = b.trunc_stats()
    assert b.info()["unconverged_svds"] == 0
    compared, ref = 0, []
    for i in range(len(X)):
        r = omps.simulate(X[i], w.distance, w.reps, w.chi, w.cutoff, w.coef_z, w.coef_xx, routing=routing,
                          gate_split=gate_split)
        ref.append(r.tensors)
        f = fidelity(b.export(i), r.tensors)
        print(i, "fidelity", f, "max bond", max(dims[i]), "bonds equal", list(dims[i]) == r.bond_dims,
              "disc", disc[i], r.discarded, "degenerate", deg[i], r.degenerate_cuts)
        if r.degenerate_cuts == 0 and deg[i] == 0:
            compared += 1
            assert f > 1 - 1e-10
            assert list(dims[i]) == r.bond_dims
            assert abs(disc[i] - r.discarded) <= 1e-9 * max(1.0, r.discarded)
    return compared, ref


def test_untruncated_chi128_vs_statevector():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    w = sd.Workload("t", 4, 14, 5, 2, 128, 0.0)
    X = sd.make_uniform(4, 14, seed=41)
    for routing in (0, 1):
        b = q.simulate(torch.tensor(X, device="cuda"), _spec(q, 14, w, routing), 128, 0.0)
        assert b.bond_dims().max() == 128
        for i in range(len(X)):
            # 128 is the largest bond of a 14-qubit chain: the oracle's MPS at
            # cutoff 0 is the exact state
            r = omps.simulate(X[i], w.distance, w.reps, 128, 0.0, routing=routing)
            assert r.discarded == 0.0 and max(r.bond_dims) == 128
            assert abs(fidelity(b.export(i), r.tensors) - 1) < 1e-12


@pytest.fixture(scope="module")
def slice_run():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    w, X = _slice(6)
    b = q.simulate(torch.tensor(X, device="cuda"), _spec(q, M_SLICE, w), w.chi, w.cutoff)
    compared, ref = _compare(b, X, w)
    return q, b, X, w, compared, ref


def test_truncated_chi128_vs_oracle(slice_run):
    q, b, X, w, compared, _ = slice_run
    assert b.bond_dims().max() == 128
    print("circuits compared", compared, "of", len(X))
    assert compared >= len(X) // 2


def test_gram_of_chi128_states(slice_run):
    q, b, X, w, _, ref = slice_run
    K_ref = ogram.gram(ref)
    for prec, tol in (("fp64", 1e-9), ("fp32", 2e-5)):
        K = q.gram(b, precision=prec).cpu().numpy()
        d = np.abs(K - K_ref).max()
        print(prec, "max|dK| vs oracle", d)
        assert d < tol


def test_chi128_routing0_and_gate_split():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    w, X = _slice(2)
    xt = torch.tensor(X, device="cuda")
    b0 = q.simulate(xt, _spec(q, M_SLICE, w, routing=0), w.chi, w.cutoff)
    c0, _ = _compare(b0, X, w, routing=0)
    bs = q.simulate(xt, _spec(q, M_SLICE, w, routing=1, gate_split=1), w.chi, w.cutoff)
    cs, _ = _compare(bs, X, w, routing=1, gate_split=True)
    print("compared: routing 0", c0, "gate split", cs)
    assert c0 >= 1 and cs >= 1


def test_chi128_graph_replay_bit_identical():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    w, X = _slice(5)
    xt = torch.tensor(X, device="cuda")
    e = q.simulate(xt, _spec(q, M_SLICE, w), w.chi, w.cutoff)
    g = q.simulate(xt, _spec(q, M_SLICE, w), w.chi, w.cutoff, graph_circuits=2)
    assert (e.bond_dims() == g.bond_dims()).all()
    for i in range(len(X)):
        for te, tg in zip(e.export(i), g.export(i)):
            assert np.array_equal(te, tg)


def test_chi_above_128_not_supported():
    import paper_2411_09336_amd as q
    torch = require_gpu()
    w, X = _slice(1)
    with pytest.raises(q.QKError) as e:
        q.simulate(torch.tensor(X, device="cuda"), _spec(q, M_SLICE, w), 129, w.cutoff)
    assert e.value.status == QK_ENOTSUP
