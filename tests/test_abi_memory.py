"""Host-side checks of the device-memory hook and the batch file format (no
GPU needed): an allocator that returns NULL makes every allocating call fail
with QK_ENOMEM before any device work, malformed allocators and batch files
are rejected with QK_EINVAL, and a well-formed file passes the parser."""
import ctypes as C
import struct

import numpy as np
import pytest

import paper_2411_09336_amd as q
from paper_2411_09336_amd import api

QK_EINVAL, QK_ENOMEM = -1, -2


@pytest.fixture()
def lib():
    L = api._load()
    yield L
    L.qk_init(0, None)          # back to hipMalloc (fails harmlessly without a device)


def _null_allocator(calls):
    def alloc(nbytes, ctx, stream):
        calls.append(("alloc", int(nbytes)))
        return None

    def free(ptr, ctx, stream):
        calls.append(("free", ptr))
    return api._Allocator(api._ALLOC_FN(alloc), api._FREE_FN(free), None)


def test_allocator_returning_null_gives_enomem(lib):
    calls = []
    a = _null_allocator(calls)
    lib.qk_init(0, C.byref(a))        # registered even where no device can be selected
    dims = np.array([[1, 2, 1]], dtype=np.int32)
    t = np.zeros(2 * (2 * 1 * 2 + 2 * 2 * 1), dtype=np.float64)
    t[0] = 1.0
    h = C.c_void_p(0)
    st = lib.mps_batch_import(t.ctypes.data, dims.ctypes.data, 1, 2, None, C.byref(h))
    assert st == QK_ENOMEM
    assert h.value is None
    assert b"allocation" in lib.qk_last_error()
    assert calls and calls[0][0] == "alloc" and not any(c[0] == "free" for c in calls)


def test_invalid_allocators_are_rejected(lib):
    assert lib.qk_init(-1, None) == QK_EINVAL
    a = api._Allocator(api._ALLOC_FN(lambda n, c, s: None), api._FREE_FN(0), None)
    assert lib.qk_init(0, C.byref(a)) == QK_EINVAL
    assert b"NULL function" in lib.qk_last_error()


def _batch_file(m=2, n=1, pad=(32, 32, 32), dims=((1, 2, 1),), magic=b"QKMPSB01", extra=b"", cut=0):
    pad = list(pad)
    stride = sum(2 * pad[l] * pad[l + 1] for l in range(m))
    body = magic + struct.pack("<iiq", m, 7, n) + struct.pack(f"<{m + 1}i", *pad)
    for d in dims:
        body += struct.pack(f"<{m + 1}i", *d)
    body += struct.pack(f"<{n}d", *([0.0] * n)) * 2 + struct.pack(f"<{n}i", *([0] * n)) * 2
    body += np.zeros(2 * stride * n).tobytes() + extra
    return body[:len(body) - cut] if cut else body


@pytest.mark.parametrize("kind", ["missing", "magic", "short_header", "bad_pad", "bad_dims", "truncated",
                                  "trailing"])
def test_malformed_batch_files_are_rejected(lib, tmp_path, kind):
    p = tmp_path / "b.qkmps"
    if kind != "missing":
        data = {"magic": lambda: _batch_file(magic=b"NOTMPS01"),
                "short_header": lambda: _batch_file()[:12],
                "bad_pad": lambda: _batch_file(pad=(32, 48, 32)),
                "bad_dims": lambda: _batch_file(dims=((1, 40, 1),)),
                "truncated": lambda: _batch_file(cut=8),
                "trailing": lambda: _batch_file(extra=b"x")}[kind]()
        p.write_bytes(data)
    h = C.c_void_p(0)
    assert lib.mps_batch_load(str(p).encode(), None, C.byref(h)) == QK_EINVAL
    assert h.value is None


def test_well_formed_batch_file_reaches_allocation(lib, tmp_path):
    """The parser accepts a file laid out as the header documents; with an
    allocator that returns NULL the load then stops with QK_ENOMEM."""
    p = tmp_path / "b.qkmps"
    p.write_bytes(_batch_file())
    calls = []
    a = _null_allocator(calls)
    lib.qk_init(0, C.byref(a))
    h = C.c_void_p(0)
    assert lib.mps_batch_load(str(p).encode(), None, C.byref(h)) == QK_ENOMEM
    assert calls and calls[0][0] == "alloc"


def test_save_rejects_null(lib):
    assert lib.mps_batch_save(None, b"/tmp/x") == QK_EINVAL
