"""Truncated MPS simulation of the feature-map circuit (Sec. II-B, Fig. 1).

An MPS on m sites is a list of complex128 tensors ``A[l]`` of shape
(D_l, 2, D_{l+1}) with D_0 = D_m = 1.  The state starts as |+>^m (all bonds
of dimension 1).  Gates are applied in gate-list order:

* Rz on a site: contract the 2x2 gate with the site's physical leg
  (Fig. 1a).  Being unitary, it leaves the canonical form intact.
* Rxx / SWAP on sites (p, p+1): first move the orthogonality centre next to
  the gate with QR (left-to-right) or LQ (right-to-left) steps, so that the
  truncation is optimal (canonicalisation footnote of Sec. II-B); contract
  both sites and the gate into theta of shape (2 D_p) x (2 D_{p+2}); take its
  SVD; keep k singular values; contract S into the site on the side of the
  next two-qubit gate (Fig. 1b).

Truncation (Sec. II-B, Eq. (8)): with s sorted descending and total
W = sum s_i^2, k_cut is the smallest k whose discarded weight
sum_{i>=k} s_i^2 <= cutoff * W; the kept count is max(1, min(chi, k_cut)).
With cutoff <= 0 no weight truncation happens (k_cut = full rank).  The
kept values are rescaled to sum s^2 = 1, so the state stays normalised and
Eq. (8) gives the fidelity 1 - eps of each truncation, eps being the
discarded relative weight.

Finally the centre is swept to the last site (left-canonical form) and the
last tensor is normalised to unit norm.

Memory trace (the memory evolution of Sec. III-A, Fig. 6): after every
two-qubit gate the result records the bond dimension at the gate's cut and
sum_l D_l D_{l+1} over all sites, so the FP64 tensors take 32 bytes times
that sum (two physical values, 16-byte complex entries).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from . import gates
from .circuit import OP_RZ, OP_RXX, OP_SWAP, build_gate_list, gate_angle

DEGENERATE_GAP = 1e-10


@dataclass
class MPSResult:
    tensors: List[np.ndarray]
    discarded: float = 0.0            # sum of discarded relative weights
    max_discarded: float = 0.0        # largest single-truncation discarded weight
    degenerate_cuts: int = 0          # truncations with a near-degenerate cut
    n_svd: int = 0
    max_bond_seen: int = 1
    trace: List[tuple] = field(default_factory=list)   # per two-qubit gate: (cut bond, sum_l D_l D_{l+1})

    @property
    def bond_dims(self) -> List[int]:
        return [1] + [t.shape[2] for t in self.tensors]


def plus_mps(m: int) -> List[np.ndarray]:
    t = np.full((1, 2, 1), 1.0 / np.sqrt(2.0), dtype=np.complex128)
    return [t.copy() for _ in range(m)]


def _move_right(A: List[np.ndarray], l: int) -> None:
    """QR step: make A[l] left-isometric, push R into A[l+1]."""
    Dl, _, Dr = A[l].shape
    q, r = np.linalg.qr(A[l].reshape(Dl * 2, Dr))
    k = q.shape[1]
    A[l] = q.reshape(Dl, 2, k)
    A[l + 1] = np.tensordot(r, A[l + 1], axes=(1, 0))


def _move_left(A: List[np.ndarray], l: int) -> None:
    """LQ step: make A[l] right-isometric, push L into A[l-1]."""
    Dl, _, Dr = A[l].shape
    q, r = np.linalg.qr(A[l].reshape(Dl, 2 * Dr).conj().T)   # M^H = Q R  ->  M = R^H Q^H
    k = q.shape[1]
    A[l] = q.conj().T.reshape(k, 2, Dr)
    A[l - 1] = np.tensordot(A[l - 1], r.conj().T, axes=(2, 0))


def move_center(A: List[np.ndarray], center: int, target: int) -> int:
    while center < target:
        _move_right(A, center)
        center += 1
    while center > target:
        _move_left(A, center)
        center -= 1
    return center


def truncation_rank(s: np.ndarray, chi: int, cutoff: float) -> int:
    """Kept count k = max(1, min(chi, k_cut)) of the rule above."""
    n = len(s)
    if cutoff > 0.0:
        w = s.astype(np.float64) ** 2
        total = w.sum()
        # tail[k] = sum_{i >= k} w_i
        tail = np.concatenate([np.cumsum(w[::-1])[::-1], [0.0]])
        k_cut = n
        for k in range(n + 1):
            if tail[k] <= cutoff * total:
                k_cut = k
                break
    else:
        k_cut = n
    return max(1, min(chi, k_cut))


def gate_factors(u4: np.ndarray, tol: float = 1e-12):
    """Operator-Schmidt factors of a two-qubit gate (its SVD before
    application, footnote of Sec. III-A): u4[(S,T),(s,t)] =
    sum_k L[k][S,s] R[k][T,t], terms whose singular value is below tol times
    the largest dropped (Rxx: two terms, 2|cos(t/2)| and 2|sin(t/2)|; one at
    a zero angle; SWAP: four)."""
    m = u4.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)   # (S s), (T t)
    u, sv, vh = np.linalg.svd(m)
    r = int(np.sum(sv > tol * sv[0]))
    L = (u[:, :r] * np.sqrt(sv[:r])).T.reshape(r, 2, 2)
    R = (np.sqrt(sv[:r])[:, None] * vh[:r]).reshape(r, 2, 2)
    return L, R


def _split_svd(A: List[np.ndarray], p: int, u4: np.ndarray):
    """SVD of theta applied through the gate's factors: theta = Bp Bq with
    Bp[(a,S),(c,k)] = sum_s L[k][S,s] A_p[a,s,c] and Bq[(c,k),(T,b)] =
    sum_t R[k][T,t] A_{p+1}[c,t,b]; with Bp = Q1 R1 and Bq^H = Q2 R2 the SVD
    of the core R1 R2^H gives those of theta, at most rank(G) D_c values."""
    L, R = gate_factors(u4)
    r = L.shape[0]
    Dl, _, Dc = A[p].shape
    Dr = A[p + 1].shape[2]
    Bp = np.einsum("kSs,asc->aSck", L, A[p]).reshape(Dl * 2, Dc * r)
    Bq = np.einsum("kTt,ctb->ckTb", R, A[p + 1]).reshape(Dc * r, 2 * Dr)
    q1, r1 = np.linalg.qr(Bp)
    q2, r2 = np.linalg.qr(Bq.conj().T)
    u, s, vh = np.linalg.svd(r1 @ r2.conj().T, full_matrices=False)
    return q1 @ u, s, vh @ q2.conj().T


def apply_two_qubit(A: List[np.ndarray], p: int, u4: np.ndarray, chi: int, cutoff: float,
                    absorb_right: bool, res: MPSResult, gate_split: bool = False) -> None:
    """Fig. 1b on sites (p, p+1); the orthogonality centre must be p or p+1.
    With gate_split the gate is applied through its operator-Schmidt factors
    (_split_svd) instead of as the dense two-site theta."""
    Dl = A[p].shape[0]
    Dr = A[p + 1].shape[2]
    if gate_split:
        u, s, vh = _split_svd(A, p, u4)
    else:
        theta = np.tensordot(A[p], A[p + 1], axes=(2, 0))            # (Dl, s, t, Dr)
        g = u4.reshape(2, 2, 2, 2)                                      # (s', t', s, t)
        theta = np.einsum("STst,astb->aSTb", g, theta)
        mat = theta.reshape(Dl * 2, 2 * Dr)
        u, s, vh = np.linalg.svd(mat, full_matrices=False)
    k = truncation_rank(s, chi, cutoff)
    w = s ** 2
    total = w.sum()
    disc = float(w[k:].sum() / total) if total > 0 else 0.0
    if k < len(s) and s[0] > 0 and (s[k - 1] - s[k]) / s[0] < DEGENERATE_GAP:
        res.degenerate_cuts += 1
    res.discarded += disc
    res.max_discarded = max(res.max_discarded, disc)
    res.n_svd += 1
    sk = s[:k] / np.sqrt(np.sum(s[:k] ** 2))
    u = u[:, :k]
    vh = vh[:k, :]
    if absorb_right:
        A[p] = u.reshape(Dl, 2, k)
        A[p + 1] = (sk[:, None] * vh).reshape(k, 2, Dr)
    else:
        A[p] = (u * sk[None, :]).reshape(Dl, 2, k)
        A[p + 1] = vh.reshape(k, 2, Dr)
    res.max_bond_seen = max(res.max_bond_seen, k)


def simulate(x: np.ndarray, d: int, reps: int, chi: int, cutoff: float,
             coef_z: float = 2.0, coef_xx: float = 2.0, routing: int = 0,
             glist: np.ndarray | None = None, gate_split: bool = False) -> MPSResult:
    """MPS of |psi(x)> = U(x)|+>^m, truncated at bond cap ``chi``; with
    ``gate_split`` every two-qubit gate is applied through its
    operator-Schmidt factors (footnote of Sec. III-A)."""
    x = np.asarray(x, dtype=np.float64)
    m = len(x)
    if glist is None:
        glist = build_gate_list(m, d, reps, routing)
    A = plus_mps(m)
    res = MPSResult(tensors=A)
    center = 0
    two_q = [i for i, r in enumerate(glist) if int(r[0]) != OP_RZ]
    nxt = {two_q[i]: (int(glist[two_q[i + 1]][1]) if i + 1 < len(two_q) else None)
           for i in range(len(two_q))}
    for gi, rec in enumerate(glist):
        op, p = int(rec[0]), int(rec[1])
        th = gate_angle(rec, x, coef_z, coef_xx)
        if op == OP_RZ:
            A[p] = np.einsum("ts,asb->atb", gates.rz(th), A[p])
            continue
        u4 = gates.rxx(th) if op == OP_RXX else gates.SWAP
        if center < p:
            center = move_center(A, center, p)
        elif center > p + 1:
            center = move_center(A, center, p + 1)
        p_next = nxt[gi]
        absorb_right = p_next is None or p_next > p
        apply_two_qubit(A, p, u4, chi, cutoff, absorb_right, res, gate_split)
        res.trace.append((A[p].shape[2], sum(t.shape[0] * t.shape[2] for t in A)))
        center = p + 1 if absorb_right else p
    move_center(A, center, m - 1)
    A[m - 1] = A[m - 1] / np.linalg.norm(A[m - 1])
    return res


def to_statevector(A: List[np.ndarray]) -> np.ndarray:
    """Contract all bonds (small m only): amplitudes in the statevector basis."""
    v = A[0]
    for t in A[1:]:
        v = np.tensordot(v, t, axes=(v.ndim - 1, 0))
    return v.reshape(-1)


def simulate_batch(X: np.ndarray, d: int, reps: int, chi: int, cutoff: float,
                   coef_z: float = 2.0, coef_xx: float = 2.0, routing: int = 0) -> List[MPSResult]:
    X = np.asarray(X, dtype=np.float64)
    glist = build_gate_list(X.shape[1], d, reps, routing)
    return [simulate(x, d, reps, chi, cutoff, coef_z, coef_xx, routing, glist) for x in X]
