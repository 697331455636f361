"""Gate list of the feature-map circuit (Eq. (3); Sec. II-C).

|psi(x)> = U(x)|+>^m with U(x) = (exp(-i H_XX) exp(-i H_Z))^reps, so each
repetition applies the Z layer first (one Rz per qubit, angle coef_z * x_i)
and then the XX layer: one Rxx per edge (i, j) of the linear chain with
1 <= j - i <= d, angle coef_xx * (1 - x_i)(1 - x_j).

The Rxx gates commute; the paper reorders them for depth without printing
the order.  We use the E_i-block order: for i = 0..m-2, for k = 1..min(d,
m-1-i): Rxx(i, i+k).  Qubits are MPS sites; a gate on sites (p, p+1) is
"at p".  Non-adjacent Rxx are routed with SWAPs (Sec. II-C): to couple qubit
i with qubit i+k, SWAPs at p = i, ..., i+k-2 carry qubit i to site i+k-1,
the Rxx acts at i+k-1, and the same SWAPs are undone in reverse order, i.e.
2(k-1) SWAPs per Rxx (routing 0, the paper's scheme).

Routing 1 cancels the back-to-back inverse SWAP pairs between consecutive
Rxx of one E_i block, so qubit i walks out once and back once: 2(K-1) SWAPs
per block with K = min(d, m-1-i).  Both orders give the same state when no
truncation happens; truncated results differ.

Records are int32 rows (op, site, feat_i, feat_j) with op 0 = RZ, 1 = RXX,
2 = SWAP and -1 for unused features.
"""
from __future__ import annotations

import numpy as np

OP_RZ, OP_RXX, OP_SWAP = 0, 1, 2


def build_gate_list(m: int, d: int, reps: int, routing: int = 0) -> np.ndarray:
    if m < 1 or d < 0 or reps < 0 or routing not in (0, 1):
        raise ValueError("invalid circuit spec")
    rows = []
    for _ in range(reps):
        for i in range(m):
            rows.append((OP_RZ, i, i, -1))
        for i in range(m - 1):
            kmax = min(d, m - 1 - i)
            if routing == 0:
                for k in range(1, kmax + 1):
                    for p in range(i, i + k - 1):
                        rows.append((OP_SWAP, p, -1, -1))
                    rows.append((OP_RXX, i + k - 1, i, i + k))
                    for p in range(i + k - 2, i - 1, -1):
                        rows.append((OP_SWAP, p, -1, -1))
            else:
                for k in range(1, kmax + 1):
                    if k > 1:
                        rows.append((OP_SWAP, i + k - 2, -1, -1))
                    rows.append((OP_RXX, i + k - 1, i, i + k))
                for p in range(i + kmax - 2, i - 1, -1):
                    rows.append((OP_SWAP, p, -1, -1))
    if not rows:
        return np.zeros((0, 4), dtype=np.int32)
    return np.asarray(rows, dtype=np.int32)


def gate_counts_closed_form(m: int, d: int, reps: int, routing: int = 0):
    """(n_rz, n_rxx, n_swap) from the counting argument of Sec. II-C."""
    n_rz = reps * m
    n_rxx = reps * sum(m - k for k in range(1, min(d, m - 1) + 1))
    if routing == 0:
        n_swap = reps * sum(2 * (k - 1) * (m - k) for k in range(1, min(d, m - 1) + 1))
    else:
        n_swap = reps * sum(2 * (min(d, m - 1 - i) - 1) for i in range(m - 1)
                            if min(d, m - 1 - i) >= 1)
    return n_rz, n_rxx, n_swap


def gate_angle(rec, x: np.ndarray, coef_z: float, coef_xx: float) -> float:
    """Rotation angle of a gate record for features ``x`` (Eqs. (4), (5))."""
    op, _, fi, fj = (int(v) for v in rec)
    if op == OP_RZ:
        return coef_z * x[fi]
    if op == OP_RXX:
        return coef_xx * (1.0 - x[fi]) * (1.0 - x[fj])
    return 0.0
