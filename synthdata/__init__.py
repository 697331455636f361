"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds only data generation and workload definitions: feature
matrices shaped like the paper's workloads (one feature per qubit, features
min-max scaled into [0, 1]) and the circuit / truncation parameters of each
workload.  It contains none of the method's arithmetic (no gates, no MPS, no
overlaps), so both the oracle and the GPU path may import it.

The paper's own dataset (Elliptic, 165 features, balanced classes; Sec. III-B)
is not available; the Gaussian-mixture generators below stand in for it.
"""
from .generators import make_uniform, make_mixture, minmax_scale, perturb_near_duplicates
from .workloads import WORKLOADS, Workload, workload_features

__all__ = [
    "make_uniform", "make_mixture", "minmax_scale", "perturb_near_duplicates",
    "WORKLOADS", "Workload", "workload_features",
]
