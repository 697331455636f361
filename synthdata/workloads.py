"""Workload definitions: data shape, circuit and truncation parameters.

Notation: ``d`` is the interaction distance of the chain (edges (i, j) with
1 <= j - i <= d) and ``reps`` is the number of repetitions of the Z layer
followed by the XX layer (the paper's r in Eq. (3)).  Rotation angles are
``coef_z * x_i`` for Rz and ``coef_xx * (1 - x_i)(1 - x_j)`` for Rxx.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

from .generators import make_mixture, make_uniform


@dataclass(frozen=True)
class Workload:
    name: str
    n_points: int
    n_qubits: int
    distance: int
    reps: int
    chi: int
    cutoff: float
    coef_z: float = 2.0
    coef_xx: float = 2.0
    generator: str = "mixture"          # "uniform" | "mixture"
    n_dirs: int = 1
    mean_scale: float = 0.5
    seed: int = 0
    dir_seed: int = 1
    n_test: int = 0                     # trailing rows used as test points
    note: str = ""


WORKLOADS = {
    # 8 qubits, 64 points, untruncated: checked against an 8-qubit statevector.
    "tiny": Workload("tiny", 64, 8, 1, 1, 16, 0.0, generator="uniform", seed=0),
    # 50 qubits, 512 points: FP64 vs FP32 overlaps.
    "fp32": Workload("fp32", 512, 50, 2, 2, 32, 1e-10),
    # 100 qubits, 2048 points: FP64 / FP32 / split-BF16 overlaps.
    "precision": Workload("precision", 2048, 100, 4, 2, 64, 1e-10),
    # uneven batch: four instances in one launch (1600 train + 400 test each).
    "uneven_20": Workload("uneven_20", 2000, 20, 1, 2, 16, 1e-10, seed=0, n_test=400),
    "uneven_60": Workload("uneven_60", 2000, 60, 3, 2, 32, 1e-10, seed=1, n_test=400),
    "uneven_110": Workload("uneven_110", 2000, 110, 5, 2, 64, 1e-10, seed=2, n_test=400),
    "uneven_165": Workload("uneven_165", 2000, 165, 8, 2, 128, 1e-10, seed=3, n_test=400),
    # full scale: 165 qubits, 6400 points, chi = 64.
    "full": Workload("full", 6400, 165, 8, 2, 64, 1e-8, n_dirs=10, mean_scale=0.3),
    # the full-scale circuit on 2048 distinct points (every point simulated):
    # the precision of every form at 165 qubits beyond the timed workload's
    # 240 distinct states.
    "full_distinct": Workload("full_distinct", 2048, 165, 8, 2, 64, 1e-8, n_dirs=10, mean_scale=0.3),
    # paper-faithful bandwidth at 165 qubits (gamma = 0.1: coef_z = 2 gamma,
    # coef_xx = gamma^2 pi), d = 1, two repetitions.
    "paper_d1": Workload("paper_d1", 6400, 165, 1, 2, 64, 1e-8,
                         coef_z=0.2, coef_xx=0.01 * np.pi, n_dirs=10, mean_scale=0.3),
    # memory evolution during simulation (the setting of Fig. 6): 100 qubits,
    # d = 6 and d = 12, two repetitions, gamma = 1 (coef_z = 2, coef_xx = pi),
    # truncation at discarded weight 1e-16; 8 samples each, bond cap 64.
    "fig6_d6": Workload("fig6_d6", 8, 100, 6, 2, 64, 1e-16,
                        coef_z=2.0, coef_xx=np.pi, n_dirs=10, mean_scale=0.3),
    "fig6_d12": Workload("fig6_d12", 8, 100, 12, 2, 64, 1e-16,
                         coef_z=2.0, coef_xx=np.pi, n_dirs=10, mean_scale=0.3),
}


def workload_features(w: Workload, n: int | None = None) -> np.ndarray:
    """Feature matrix (n x m, float64, row-major) of workload ``w``."""
    if w.generator == "uniform":
        x = make_uniform(w.n_points, w.n_qubits, seed=w.seed)
    else:
        x = make_mixture(w.n_points, w.n_qubits, n_dirs=w.n_dirs,
                         mean_scale=w.mean_scale, seed=w.seed, dir_seed=w.dir_seed)
    if n is not None:
        x = x[:n]
    return np.ascontiguousarray(x, dtype=np.float64)
