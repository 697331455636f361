"""Helpers shared by the GPU tests (not collected by pytest)."""
import numpy as np


def require_gpu():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_09336_amd as q
    q.api._load()          # fail loudly if the HIP library is missing
    return torch


def fidelity(mps_a, mps_b):
    from oracle import gram
    return abs(gram.overlap(mps_a, mps_b)) ** 2
