"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/qkmps.h, and its gate lists agree
byte for byte with the oracle's independent gate-list builder."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2411_09336_amd as q
from oracle import circuit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "qkmps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:qk_status|void|const char\s*\*)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(q.library_path())
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert q.version().startswith("qkmps")


@pytest.mark.parametrize("m,d,reps,routing", [(8, 1, 1, 0), (50, 2, 2, 0), (100, 4, 2, 0), (165, 8, 2, 0),
                                             (165, 8, 2, 1), (20, 1, 2, 1), (3, 7, 3, 0), (1, 1, 1, 0)])
def test_gate_list_matches_oracle_bytes(m, d, reps, routing):
    g = q.circuit_compile(q.CircuitSpec(m, d, reps, routing=routing))
    o = circuit.build_gate_list(m, d, reps, routing)
    assert g.shape == o.shape
    assert g.tobytes() == o.tobytes()


@pytest.mark.parametrize("bad", [dict(n_qubits=0, distance=1, reps=1), dict(n_qubits=4, distance=-1, reps=1),
                                 dict(n_qubits=4, distance=1, reps=-2), dict(n_qubits=4, distance=1, reps=1, routing=5),
                                 dict(n_qubits=4, distance=1, reps=1, coef_z=float("nan")),
                                 dict(n_qubits=4, distance=1, reps=1, gate_split=2)])
def test_invalid_spec_is_rejected(bad):
    with pytest.raises(q.QKError) as e:
        q.circuit_compile(q.CircuitSpec(**bad))
    assert e.value.status == -1


def test_invalid_calls_fail_before_device_work():
    lib = ctypes.CDLL(q.library_path())
    lib.qk_last_error.restype = ctypes.c_char_p
    # NULL outputs / handles are rejected with QK_EINVAL
    assert lib.mps_simulate(None, ctypes.c_int64(4), None, 16, ctypes.c_double(0.0), None, None) == -1
    assert lib.mps_gram(None, None, 0, None, ctypes.c_int64(0), None) == -1
    assert lib.mps_gram_block_noalloc(None, ctypes.c_int64(0), ctypes.c_int64(1), None, ctypes.c_int64(0),
                                      ctypes.c_int64(1), 0, 0, None, ctypes.c_int64(1), None) == -1
    assert lib.mps_batch_info(None, None) == -1
    assert lib.qk_last_error()
