"""Host-side argument checks of the Python binding (no GPU needed): a
caller-supplied K block that the kernels could not write safely (wrong
dtype, too small, transposed, rows closer than the columns written, host
memory) is rejected with ValueError before any library call."""
import pytest
import torch

import paper_2411_09336_amd as q


class _FakeBatch:
    """Stands in for an MPSBatch: the checks run before the handle is used."""

    def __init__(self, n):
        self.n = n
        self.handle = None


BAD_OUTS = [
    (lambda: torch.zeros((4, 4), dtype=torch.float32), "float64"),
    (lambda: torch.zeros((3, 4), dtype=torch.float64), "cannot hold"),
    (lambda: torch.zeros((4, 3), dtype=torch.float64), "cannot hold"),
    (lambda: torch.zeros((4, 4), dtype=torch.float64).t(), "unit column stride"),
    (lambda: torch.zeros((8, 8), dtype=torch.float64)[:, ::2], "unit column stride"),
    (lambda: torch.zeros(64, dtype=torch.float64).as_strided((4, 4), (2, 1)), "row stride"),
    (lambda: torch.zeros(16, dtype=torch.float64), "2-D"),
    (lambda: torch.zeros((4, 4), dtype=torch.float64), "GPU"),
]


@pytest.mark.parametrize("make,msg", BAD_OUTS)
def test_gram_block_rejects_bad_out(make, msg):
    with pytest.raises(ValueError, match=msg):
        q.gram_block(_FakeBatch(4), 0, 4, _FakeBatch(4), 0, 4, out=make())


@pytest.mark.parametrize("make,msg", BAD_OUTS)
def test_gram_rejects_bad_out(make, msg):
    with pytest.raises(ValueError, match=msg):
        q.gram(_FakeBatch(4), _FakeBatch(4), out=make())


@pytest.mark.parametrize("make,msg", BAD_OUTS)
def test_gram_multi_rejects_bad_out(make, msg):
    good = dict(a=_FakeBatch(4), b=_FakeBatch(4), na=2, nb=2, out=torch.zeros((2, 2), dtype=torch.float64))
    bad = dict(a=_FakeBatch(4), b=_FakeBatch(4), na=4, nb=4, out=make())
    with pytest.raises(ValueError, match=msg):
        q.gram_multi([bad, good])
