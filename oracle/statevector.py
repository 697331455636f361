"""Brute-force state vectors (Eqs. (1)-(5)) for small qubit counts.

Basis index convention: qubit 0 is the most significant bit, so the state
reshaped to shape (2,)*m has axis q for qubit q (= MPS site q).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from . import gates
from .circuit import OP_RZ, OP_RXX, OP_SWAP, gate_angle

MAX_QUBITS = 12


def plus_state(m: int) -> np.ndarray:
    """|+>^m = H^{(x)m}|0>^m (Eq. (2))."""
    return np.full(2 ** m, 2.0 ** (-0.5 * m), dtype=np.complex128)


def apply_1q(psi: np.ndarray, u: np.ndarray, q: int, m: int) -> np.ndarray:
    t = psi.reshape((2 ** q, 2, 2 ** (m - q - 1)))
    return np.einsum("ab,xby->xay", u, t).reshape(-1)


def apply_2q(psi: np.ndarray, u4: np.ndarray, q0: int, q1: int, m: int) -> np.ndarray:
    """Apply a 4x4 gate to qubits (q0, q1); q0 is the first tensor factor."""
    t = psi.reshape((2,) * m)
    t = np.moveaxis(t, (q0, q1), (0, 1))
    shp = t.shape
    t = (u4 @ t.reshape(4, -1)).reshape(shp)
    t = np.moveaxis(t, (0, 1), (q0, q1))
    return t.reshape(-1)


def state_logical(x: np.ndarray, d: int, reps: int, coef_z: float, coef_xx: float) -> np.ndarray:
    """|psi(x)> applying every Rxx directly on qubits (i, j), no routing."""
    m = len(x)
    if m > MAX_QUBITS:
        raise ValueError("statevector oracle is limited to 12 qubits")
    psi = plus_state(m)
    for _ in range(reps):
        for i in range(m):
            psi = apply_1q(psi, gates.rz(coef_z * x[i]), i, m)
        for i in range(m - 1):
            for k in range(1, min(d, m - 1 - i) + 1):
                j = i + k
                psi = apply_2q(psi, gates.rxx(coef_xx * (1 - x[i]) * (1 - x[j])), i, j, m)
    return psi


def state_from_gate_list(x: np.ndarray, glist: np.ndarray, coef_z: float, coef_xx: float) -> np.ndarray:
    """|psi(x)> applying a site-level gate list (with SWAPs) to a state vector."""
    m = len(x)
    if m > MAX_QUBITS:
        raise ValueError("statevector oracle is limited to 12 qubits")
    psi = plus_state(m)
    for rec in glist:
        op, p = int(rec[0]), int(rec[1])
        th = gate_angle(rec, x, coef_z, coef_xx)
        if op == OP_RZ:
            psi = apply_1q(psi, gates.rz(th), p, m)
        elif op == OP_RXX:
            psi = apply_2q(psi, gates.rxx(th), p, p + 1, m)
        elif op == OP_SWAP:
            psi = apply_2q(psi, gates.SWAP, p, p + 1, m)
        else:
            raise ValueError("bad op")
    return psi


def _op_on(op1: np.ndarray, q: int, m: int) -> np.ndarray:
    out = np.array([[1.0 + 0j]])
    for k in range(m):
        out = np.kron(out, op1 if k == q else gates.I2)
    return out


def unitary_from_hamiltonians(x: np.ndarray, d: int, reps: int, gamma_z: float, gamma_xx: float) -> np.ndarray:
    """U(x) = (exp(-i H_XX) exp(-i H_Z))^reps from the Hamiltonians (Eqs. (3)-(5)).

    ``H_Z = gamma_z * sum_i x_i Z_i`` and
    ``H_XX = gamma_xx * sum_{1<=j-i<=d} (1-x_i)(1-x_j) X_i X_j`` are built as
    dense 2^m matrices and exponentiated with ``scipy.linalg.expm``; the
    paper's choice is gamma_z = gamma and gamma_xx = gamma^2 pi / 2.
    Only for m <= 6.
    """
    m = len(x)
    if m > 6:
        raise ValueError("dense-Hamiltonian reference is limited to 6 qubits")
    dim = 2 ** m
    hz = np.zeros((dim, dim), dtype=np.complex128)
    for i in range(m):
        hz += gamma_z * x[i] * _op_on(gates.Z, i, m)
    hxx = np.zeros((dim, dim), dtype=np.complex128)
    for i in range(m):
        for j in range(i + 1, min(m, i + d + 1)):
            hxx += gamma_xx * (1 - x[i]) * (1 - x[j]) * (_op_on(gates.X, i, m) @ _op_on(gates.X, j, m))
    layer = expm(-1j * hxx) @ expm(-1j * hz)
    return np.linalg.matrix_power(layer, reps)


def gram_from_states(psi_a: np.ndarray, psi_b: np.ndarray | None = None) -> np.ndarray:
    """K_ij = |<psi_a_i | psi_b_j>|^2 for rows of state matrices (Eq. (1))."""
    if psi_b is None:
        psi_b = psi_a
    ov = np.conj(psi_a) @ psi_b.T
    return np.abs(ov) ** 2
