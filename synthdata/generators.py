"""Seeded feature generators.  All use ``numpy.random.default_rng``."""
from __future__ import annotations

import numpy as np


def make_uniform(n: int, m: int, seed: int = 0) -> np.ndarray:
    """``n`` points with ``m`` features drawn i.i.d. uniform on [0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, m))


def minmax_scale(x: np.ndarray) -> np.ndarray:
    """Per-feature min-max scaling into [0, 1] over all rows of ``x``.

    A constant feature maps to 0.5.
    """
    lo = x.min(axis=0)
    hi = x.max(axis=0)
    span = hi - lo
    out = np.empty_like(x, dtype=np.float64)
    ok = span > 0
    out[:, ok] = (x[:, ok] - lo[ok]) / span[ok]
    out[:, ~ok] = 0.5
    return out


def unit_directions(k: int, m: int, seed: int) -> np.ndarray:
    """``k`` random unit vectors in R^m (rows), seeded."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((k, m))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def make_mixture(n: int, m: int, *, n_dirs: int = 1, mean_scale: float = 0.5,
                 sigma: float = 1.0, seed: int = 0, dir_seed: int = 1,
                 return_labels: bool = False):
    """Balanced two-class Gaussian mixture, min-max scaled to [0, 1].

    Class means are ``+/- mean_scale * sum_k u_k`` for ``n_dirs`` random unit
    directions ``u_k`` (drawn with ``dir_seed``); both classes are isotropic
    with standard deviation ``sigma``.  Rows are shuffled with ``seed``.
    """
    rng = np.random.default_rng(seed)
    mu = mean_scale * unit_directions(n_dirs, m, dir_seed).sum(axis=0)
    n_pos = n // 2
    labels = np.concatenate([np.ones(n_pos, dtype=np.int64),
                             -np.ones(n - n_pos, dtype=np.int64)])
    x = rng.standard_normal((n, m)) * sigma + labels[:, None] * mu[None, :]
    perm = rng.permutation(n)
    x = minmax_scale(x[perm])
    if return_labels:
        return x, labels[perm]
    return x


def perturb_near_duplicates(x: np.ndarray, scale: float = 0.01, seed: int = 7) -> np.ndarray:
    """Near-duplicate copies ``clip(x + scale * N(0, 1), 0, 1)``.

    Pairs (x, x') then have mid-range kernel values, so precision checks are
    not decided by the (near-zero) off-diagonal bulk alone.
    """
    rng = np.random.default_rng(seed)
    return np.clip(x + scale * rng.standard_normal(x.shape), 0.0, 1.0)
