"""MPS inner products and Gram matrices (Eq. (1), Fig. 2).

<a|b> is contracted left to right: E_0 = [[1]], then for each site
E_{l+1} = sum_s A_a[l][:, s, :]^H E_l A_b[l][:, s, :]; the overlap is the
single entry of E_m, and K = |<a|b>|^2.  Plain complex128, no rescaling.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np


def overlap(a: Sequence[np.ndarray], b: Sequence[np.ndarray]) -> complex:
    if len(a) != len(b):
        raise ValueError("MPS of different lengths")
    E = np.ones((1, 1), dtype=np.complex128)
    for ta, tb in zip(a, b):
        En = np.zeros((ta.shape[2], tb.shape[2]), dtype=np.complex128)
        for s in range(2):
            En += ta[:, s, :].conj().T @ E @ tb[:, s, :]
        E = En
    return complex(E[0, 0])


def gram(batch_a: List[Sequence[np.ndarray]], batch_b: List[Sequence[np.ndarray]] | None = None,
         symmetric_diag: bool = True) -> np.ndarray:
    """K[i, j] = |<a_i|b_j>|^2.  With ``batch_b`` None the matrix is symmetric
    and only i <= j is contracted (mirrored)."""
    if batch_b is None:
        n = len(batch_a)
        K = np.zeros((n, n))
        for i in range(n):
            for j in range(i, n):
                if i == j and not symmetric_diag:
                    continue
                K[i, j] = abs(overlap(batch_a[i], batch_a[j])) ** 2
                K[j, i] = K[i, j]
        return K
    K = np.zeros((len(batch_a), len(batch_b)))
    for i, a in enumerate(batch_a):
        for j, b in enumerate(batch_b):
            K[i, j] = abs(overlap(a, b)) ** 2
    return K
