"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: dense
matrix exponentials of the Hamiltonians, closed forms, Eq. (8), counting
arguments, and the invariants of a Gram matrix of unit vectors.
"""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import circuit, gates, gram, mps
from oracle import statevector as sv
import synthdata as sd


# ---------------------------------------------------------------- gates
def test_gate_matrices_match_exponentials():
    for th in (0.0, 0.3, -1.7, 2.9):
        assert np.allclose(gates.rz(th), expm(-0.5j * th * gates.Z), atol=1e-14)
        assert np.allclose(gates.rxx(th), expm(-0.5j * th * np.kron(gates.X, gates.X)), atol=1e-14)
        for u in (gates.rz(th), gates.rxx(th), gates.SWAP, gates.H):
            assert np.allclose(u.conj().T @ u, np.eye(u.shape[0]), atol=1e-14)
    # SWAP exchanges the two tensor factors: SWAP (a (x) b) = b (x) a
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2), rng.standard_normal(2) + 0j
    assert np.allclose(gates.SWAP @ np.kron(a, b), np.kron(b, a))
    # H|0> = |+>
    assert np.allclose(gates.H @ np.array([1, 0]), np.full(2, 2 ** -0.5))


# ---------------------------------------------------------------- gate list
@pytest.mark.parametrize("m,d,reps", [(8, 1, 1), (8, 3, 2), (50, 2, 2), (100, 4, 2), (165, 8, 2), (5, 9, 1), (1, 2, 1)])
@pytest.mark.parametrize("routing", [0, 1])
def test_gate_counts_closed_form(m, d, reps, routing):
    g = circuit.build_gate_list(m, d, reps, routing)
    counts = tuple(int((g[:, 0] == op).sum()) if len(g) else 0 for op in (0, 1, 2))
    assert counts == circuit.gate_counts_closed_form(m, d, reps, routing)
    if len(g):
        assert g[:, 1].min() >= 0
        two = g[g[:, 0] != 0]
        if len(two):
            assert two[:, 1].max() <= m - 2


def test_full_scale_gate_count():
    # 165 qubits, d = 8, 2 repetitions: 20,376 two-qubit gates with routing 0
    g = circuit.build_gate_list(165, 8, 2, 0)
    assert int((g[:, 0] != 0).sum()) == 20376
    g1 = circuit.build_gate_list(165, 8, 2, 1)
    assert int((g1[:, 0] != 0).sum()) == 7048


def test_routing_moves_the_right_qubits():
    """Track qubit positions through the SWAPs: every Rxx meets its two features."""
    for routing in (0, 1):
        m, d = 9, 4
        g = circuit.build_gate_list(m, d, 1, routing)
        pos = list(range(m))          # pos[site] = qubit
        seen = set()
        for op, p, fi, fj in g:
            if op == 2:
                pos[p], pos[p + 1] = pos[p + 1], pos[p]
            elif op == 1:
                assert {pos[p], pos[p + 1]} == {fi, fj}
                seen.add((min(fi, fj), max(fi, fj)))
            elif op == 0:
                assert pos[p] == fi
        assert pos == list(range(m))
        assert seen == {(i, j) for i in range(m) for j in range(i + 1, min(m, i + d + 1))}


# ---------------------------------------------------------------- statevector vs Hamiltonians
@pytest.mark.parametrize("m,d,reps", [(3, 1, 1), (4, 2, 2), (5, 3, 1), (6, 2, 2)])
def test_statevector_matches_hamiltonian_exponentials(m, d, reps):
    """Eq. (3)-(5): U(x)|+> from expm of dense H_Z, H_XX equals the gate circuit.

    gamma_z = coef_z / 2 and gamma_xx = coef_xx / 2 under Rz(t)=exp(-itZ/2),
    Rxx(t)=exp(-itXX/2); coef_z = 2 gamma, coef_xx = gamma^2 pi is the paper.
    """
    rng = np.random.default_rng(m * 10 + d)
    x = rng.random(m)
    for gamma in (1.0, 0.37):
        cz, cxx = 2 * gamma, gamma ** 2 * np.pi
        U = sv.unitary_from_hamiltonians(x, d, reps, gamma, gamma ** 2 * np.pi / 2)
        ref = U @ sv.plus_state(m)
        psi = sv.state_logical(x, d, reps, cz, cxx)
        assert np.allclose(psi, ref, atol=1e-12)
        for routing in (0, 1):
            g = circuit.build_gate_list(m, d, reps, routing)
            psi2 = sv.state_from_gate_list(x, g, cz, cxx)
            assert np.allclose(psi2, ref, atol=1e-12)


# ---------------------------------------------------------------- MPS vs statevector
@pytest.mark.parametrize("m,d,reps", [(8, 1, 1), (8, 3, 2), (10, 5, 2), (7, 6, 1), (11, 2, 2)])
@pytest.mark.parametrize("routing", [0, 1])
def test_untruncated_mps_equals_statevector(m, d, reps, routing):
    rng = np.random.default_rng(100 + m + d)
    X = rng.random((3, m))
    states, mps_states = [], []
    for x in X:
        r = mps.simulate(x, d, reps, chi=2 ** (m // 2), cutoff=0.0, routing=routing)
        assert r.discarded < 1e-24
        psi = mps.to_statevector(r.tensors)
        ref = sv.state_logical(x, d, reps, 2.0, 2.0)
        assert abs(abs(np.vdot(psi, ref)) ** 2 - 1.0) < 1e-12
        assert abs(np.linalg.norm(psi) - 1) < 1e-13
        states.append(ref)
        mps_states.append(r.tensors)
        # bond dims never exceed the exact Schmidt-rank bound
        for l, D in enumerate(r.bond_dims):
            assert D <= 2 ** min(l, m - l)
        # left-canonical: every site but the last is a left isometry
        for t in r.tensors[:-1]:
            M = t.reshape(-1, t.shape[2])
            assert np.allclose(M.conj().T @ M, np.eye(M.shape[1]), atol=1e-13)
    K_sv = sv.gram_from_states(np.array(states))
    K_mps = gram.gram(mps_states)
    assert np.allclose(K_mps, K_sv, atol=1e-12)


def test_overlap_against_statevector_inner_product():
    """Fig. 2 contraction == <a|b> of the contracted vectors (catches a missing conj)."""
    rng = np.random.default_rng(5)
    for _ in range(4):
        xa, xb = rng.random(7), rng.random(7)
        ra = mps.simulate(xa, 2, 2, 64, 0.0)
        rb = mps.simulate(xb, 2, 2, 64, 0.0)
        ov = gram.overlap(ra.tensors, rb.tensors)
        ref = np.vdot(mps.to_statevector(ra.tensors), mps.to_statevector(rb.tensors))
        assert abs(ov - ref) < 1e-13
        assert abs(gram.overlap(rb.tensors, ra.tensors) - np.conj(ov)) < 1e-13


# ---------------------------------------------------------------- closed forms
def test_product_state_closed_form_full_scale():
    """coef_xx = 0: K = prod_i cos^2(reps coef_z (x_i - x'_i) / 2), any m, through all SWAPs."""
    X = sd.workload_features(sd.WORKLOADS["full"], 3)
    X = 0.5 + 0.02 * (X - 0.5)      # keep K well above underflow
    reps, cz = 2, 2.0
    res = [mps.simulate(x, 8, reps, 64, 1e-12, coef_z=cz, coef_xx=0.0) for x in X]
    for r in res:
        assert max(r.bond_dims) == 1
    K = gram.gram([r.tensors for r in res])
    for i in range(3):
        for j in range(3):
            ref = np.prod(np.cos(reps * cz * (X[i] - X[j]) / 2) ** 2)
            assert abs(K[i, j] - ref) < 1e-12


def test_rxx_only_gives_all_ones():
    """coef_z = 0: |+>^m is an eigenvector of every X_i X_j, so K == 1."""
    X = sd.make_uniform(3, 30, seed=4)
    res = [mps.simulate(x, 4, 2, 64, 1e-12, coef_z=0.0, coef_xx=2.0) for x in X]
    K = gram.gram([r.tensors for r in res])
    assert np.allclose(K, 1.0, atol=1e-12)


# ---------------------------------------------------------------- memory trace (Fig. 6)
@pytest.mark.parametrize("m,d,reps,routing", [(7, 2, 2, 0), (8, 3, 1, 1), (6, 5, 2, 0), (8, 2, 2, 1)])
def test_trace_cut_bond_is_schmidt_rank(m, d, reps, routing):
    """After every two-qubit gate, the recorded bond at the gate's cut is the
    Schmidt rank (discarded tail weight <= cutoff, Eq. (8)) of the state
    vector obtained by applying the same gate prefix, SWAPs included, across
    that cut; the memory sum of the last gate is that of the final tensors."""
    rng = np.random.default_rng(7 * m + d + routing)
    x = rng.random(m)
    cutoff = 1e-12
    glist = circuit.build_gate_list(m, d, reps, routing)
    r = mps.simulate(x, d, reps, 64, cutoff, routing=routing, glist=glist)
    two_q = [i for i, rec in enumerate(glist) if int(rec[0]) != circuit.OP_RZ]
    assert len(r.trace) == len(two_q)
    for g, gi in enumerate(two_q):
        p = int(glist[gi][1])
        psi = sv.state_from_gate_list(x, glist[:gi + 1], 2.0, 2.0)
        s = np.linalg.svd(psi.reshape(2 ** (p + 1), -1), compute_uv=False)
        w = s ** 2
        tail = np.concatenate([np.cumsum(w[::-1])[::-1], [0.0]])
        rank = next(k for k in range(len(w) + 1) if tail[k] <= cutoff * w.sum())
        assert r.trace[g][0] == max(1, rank), (g, p)
    assert r.trace[-1][1] == sum(t.shape[0] * t.shape[2] for t in r.tensors)


def test_trace_of_product_states():
    """coef_xx = 0: every bond stays 1, so each entry is (1, m)."""
    x = sd.make_uniform(1, 40, seed=9)[0]
    r = mps.simulate(x, 4, 2, 64, 1e-12, coef_z=2.0, coef_xx=0.0, routing=1)
    _, n_rxx, n_swap = circuit.gate_counts_closed_form(40, 4, 2, 1)
    assert len(r.trace) == n_rxx + n_swap
    assert set(r.trace) == {(1, 40)}


# ---------------------------------------------------------------- Eq. (8)
def test_single_truncation_fidelity_eq8():
    """Truncating one bond of a normalised canonical state: |<psi|psi_tr>|^2 = 1 - eps."""
    rng = np.random.default_rng(11)
    m = 10
    x = rng.random(m)
    r = mps.simulate(x, 4, 2, 64, 0.0)
    A_full = [t.copy() for t in r.tensors]
    psi = mps.to_statevector(A_full)
    # centre currently at m-1; move it to p and apply an identity gate with a cap
    for p in (3, 4, 5):
        A = [t.copy() for t in A_full]
        c = mps.move_center(A, m - 1, p + 1)
        res = mps.MPSResult(tensors=A)
        theta = np.tensordot(A[p], A[p + 1], axes=(2, 0)).reshape(A[p].shape[0] * 2, -1)
        s = np.linalg.svd(theta, compute_uv=False)
        k = 5
        eps = float(np.sum(s[k:] ** 2) / np.sum(s ** 2))
        assert eps > 1e-6
        mps.apply_two_qubit(A, p, np.eye(4, dtype=complex), k, 0.0, True, res)
        psi_tr = mps.to_statevector(A)
        assert abs(np.linalg.norm(psi_tr) - 1) < 1e-12
        assert abs(abs(np.vdot(psi, psi_tr)) ** 2 - (1 - eps)) < 1e-12
        assert abs(res.discarded - eps) < 1e-14


def test_truncation_rank_rule():
    s = np.sqrt(np.array([0.5, 0.3, 0.15, 0.04, 0.009, 0.001]))
    assert mps.truncation_rank(s, 64, 0.0) == 6
    assert mps.truncation_rank(s, 3, 0.0) == 3
    assert mps.truncation_rank(s, 64, 0.001) == 5          # tail 0.001 <= 0.001
    assert mps.truncation_rank(s, 64, 0.0009) == 6
    assert mps.truncation_rank(s, 64, 0.0101) == 4          # 0.009 + 0.001 = 0.010
    assert mps.truncation_rank(s, 64, 0.99) == 1            # never below one
    assert mps.truncation_rank(s, 2, 0.0101) == 2


# ---------------------------------------------------------------- invariants under truncation
def test_truncated_gram_invariants():
    w = sd.WORKLOADS["fp32"]
    X = sd.workload_features(w, 12)
    X = np.vstack([X, sd.perturb_near_duplicates(X[:4])])
    res = [mps.simulate(x, w.distance, w.reps, 8, w.cutoff) for x in X]
    for r in res:
        assert max(r.bond_dims) <= 8
        assert r.max_discarded > 0
    K = gram.gram([r.tensors for r in res])
    assert np.allclose(np.diag(K), 1.0, atol=1e-12)
    assert np.allclose(K, K.T, atol=0)
    assert K.min() >= 0 and K.max() <= 1 + 1e-12
    # |G|^2 of unit vectors is PSD (Schur product of a PSD Gram with its conjugate)
    assert np.linalg.eigvalsh(K).min() > -1e-12
    # the near-duplicates give mid-range kernel values
    assert K[np.arange(4), 12 + np.arange(4)].min() > 0.05


def test_tiny_workload_matches_golden_statevector_gram():
    """The stored statevector Gram (tests/golden/make_golden.py) pins the MPS
    oracle on the tiny workload end to end."""
    import os
    K_gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "tiny_gram_statevector.npy"))
    w = sd.WORKLOADS["tiny"]
    X = sd.workload_features(w)
    res = [mps.simulate(x, w.distance, w.reps, w.chi, w.cutoff, w.coef_z, w.coef_xx) for x in X[:16]]
    K = gram.gram([r.tensors for r in res])
    assert np.abs(K - K_gold[:16, :16]).max() < 1e-12
    assert np.allclose(np.diag(K_gold), 1.0, atol=1e-12)


# ---------------------------------------------------------------- near-degenerate cuts (Eq. (8) ties)
def _two_site_with_spectrum(s, seed=0):
    """Sites (0, 1) of a 2-site chain with bond dimensions 1 | 2 | ... whose
    two-site matrix theta = U diag(s) V^H has the given singular values
    (random unitaries U, V; len(s) = 4 gives outer bonds 2 and 2)."""
    rng = np.random.default_rng(seed)
    n = len(s)
    dl = n // 2

    def unitary(k):
        z = rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))
        return np.linalg.qr(z)[0]

    U, V = unitary(n), unitary(n)
    left = U.reshape(dl, 2, n)
    right = (np.diag(np.asarray(s, dtype=float)) @ V.conj().T).reshape(n, 2, dl)
    return [left, right]


@pytest.mark.parametrize("s,chi,flag", [
    ([2 ** -0.5, 2 ** -0.5], 1, True),        # kept and discarded value exactly equal
    ([0.8, 0.6], 1, False),                   # clearly gapped
    ([0.6, 0.6, np.sqrt(0.14), np.sqrt(0.14)], 1, True),
    ([0.6, 0.6, np.sqrt(0.14), np.sqrt(0.14)], 2, False),   # the cut falls between the two pairs
    ([0.6, 0.6, np.sqrt(0.14), np.sqrt(0.14)], 3, True),
    ([0.6, 0.6, np.sqrt(0.14), np.sqrt(0.14)], 4, False),   # nothing discarded
])
def test_degenerate_cut_flag(s, chi, flag):
    """The oracle flags a truncation whose last kept and first discarded
    singular values coincide (several truncated states are then equally
    optimal, Eq. (8)), and only then."""
    s = np.asarray(s, dtype=float)
    assert abs(np.sum(s ** 2) - 1) < 1e-15
    A = _two_site_with_spectrum(s)
    res = mps.MPSResult(tensors=A)
    mps.apply_two_qubit(A, 0, np.eye(4, dtype=complex), chi, 0.0, True, res)
    assert res.degenerate_cuts == int(flag)
    k = min(chi, len(s))
    assert A[0].shape[2] == k
    assert abs(res.discarded - float(np.sum(s[k:] ** 2))) < 1e-14


@pytest.mark.parametrize("gap,flag", [(1e-13, True), (1e-11, True), (1e-8, False), (1e-3, False)])
def test_degenerate_cut_threshold(gap, flag):
    """The relative gap (s_k - s_{k+1}) / s_1 at the cut is compared with the
    stated threshold 1e-10: well below it flags, well above it does not."""
    a = 0.7
    b = a - gap * a
    c = np.sqrt(1 - a * a - b * b)
    s = np.array([a, b, c, 0.0])
    s = s[np.argsort(-s)]
    top = s[0]
    A = _two_site_with_spectrum(s, seed=5)
    res = mps.MPSResult(tensors=A)
    mps.apply_two_qubit(A, 0, np.eye(4, dtype=complex), 1, 0.0, True, res)
    assert (a - b) / top == pytest.approx(gap, rel=1e-3)
    assert res.degenerate_cuts == int(flag)


# ---------------------------------------------------------------- gate pre-decomposition (Sec. III-A footnote)
@pytest.mark.parametrize("th,rank", [(0.3, 2), (-1.7, 2), (2.9, 2), (0.0, 1), (np.pi, 1), (-np.pi, 1)])
def test_gate_factors_of_rxx_closed_form(th, rank):
    """Rxx(t) = cos(t/2) II - i sin(t/2) XX: two operator-Schmidt terms of
    weight 2|cos(t/2)| and 2|sin(t/2)| (Hilbert-Schmidt norm 2 of II and XX);
    one at t = 0 and t = pi, where the other coefficient vanishes."""
    L, R = mps.gate_factors(gates.rxx(th))
    assert L.shape[0] == rank
    u4 = np.einsum("kSs,kTt->STst", L, R).reshape(4, 4)
    assert np.allclose(u4, gates.rxx(th), atol=1e-14)
    weights = sorted(np.linalg.norm(L[k]) * np.linalg.norm(R[k]) for k in range(rank))
    expect = sorted(w for w in (2 * abs(np.cos(th / 2)), 2 * abs(np.sin(th / 2))) if w > 1e-12)
    assert np.allclose(weights, expect, atol=1e-13)


def test_gate_factors_of_swap():
    """SWAP = (II + XX + YY + ZZ) / 2: four terms of weight 1."""
    L, R = mps.gate_factors(gates.SWAP)
    assert L.shape[0] == 4
    assert np.allclose(np.einsum("kSs,kTt->STst", L, R).reshape(4, 4), gates.SWAP, atol=1e-14)
    assert np.allclose([np.linalg.norm(L[k]) * np.linalg.norm(R[k]) for k in range(4)], 1.0, atol=1e-13)


def test_gate_split_application_equals_dense_theta():
    """Both ways of applying a gate to sites with a small middle bond give the
    same two-site tensor; the split way keeps at most rank(G) x D_c values,
    while the dense theta's SVD also returns the gate's zero singular values as
    rounding noise, which cutoff 0 keeps."""
    rng = np.random.default_rng(21)
    Dl, Dc, Dr = 4, 1, 4
    for u4, rank in ((gates.rxx(0.7), 2), (gates.rxx(0.0), 1), (gates.SWAP, 4)):
        ap = rng.standard_normal((Dl, 2, Dc)) + 1j * rng.standard_normal((Dl, 2, Dc))
        aq = rng.standard_normal((Dc, 2, Dr)) + 1j * rng.standard_normal((Dc, 2, Dr))
        ref = np.einsum("STst,astb->aSTb", u4.reshape(2, 2, 2, 2), np.tensordot(ap, aq, axes=(2, 0)))
        for split in (False, True):
            A = [ap.copy(), aq.copy()]
            res = mps.MPSResult(tensors=A)
            mps.apply_two_qubit(A, 0, u4, 64, 0.0, True, res, gate_split=split)
            got = np.tensordot(A[0], A[1], axes=(2, 0))
            scale = np.linalg.norm(ref)    # the kept values are renormalised to unit weight
            assert np.allclose(got * scale, ref, atol=1e-13 * scale)
            k = A[0].shape[2]
            if split:
                assert k == min(rank * Dc, 2 * Dl, 2 * Dr)
            elif rank * Dc < 2 * Dl:
                assert k > rank * Dc    # the noise values survive


@pytest.mark.parametrize("m,d,reps,routing", [(6, 3, 2, 0), (7, 2, 2, 1), (8, 1, 2, 0), (5, 4, 1, 1)])
def test_gate_split_untruncated_equals_statevector(m, d, reps, routing):
    """With features at the ends of [0, 1] some Rxx angles are exactly zero
    (identity gates); the split simulation still reproduces the state vector,
    with bonds no larger than the dense one's."""
    rng = np.random.default_rng(m + 10 * d + routing)
    x = rng.random(m)
    x[1], x[m - 2] = 1.0, 0.0
    psi = sv.state_logical(x, d, reps, 2.0, 2.0)
    r = mps.simulate(x, d, reps, 64, 0.0, routing=routing, gate_split=True)
    assert abs(np.vdot(psi, mps.to_statevector(r.tensors))) ** 2 > 1 - 1e-13
    plain = mps.simulate(x, d, reps, 64, 0.0, routing=routing)
    assert all(a <= b for a, b in zip(r.bond_dims, plain.bond_dims))
    assert sum(t[0] for t in r.trace) < sum(t[0] for t in plain.trace)
