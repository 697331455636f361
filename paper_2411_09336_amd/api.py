"""ctypes binding of the C ABI in ``include/qkmps.h`` (argument marshalling only).

Every computation happens in the HIP library; these wrappers convert Python
and torch arguments into plain pointers, sizes and stream handles.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libqkmps.so")
_lib = None


def library_path() -> str:
    return _LIB_PATH


class QKError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qkmps status {status}: {msg}")
        self.status = status


class Precision:
    FP64 = 0
    FP32 = 1
    SPLIT_BF16 = 2
    SPLIT_I8 = 3
    _names = {"fp64": 0, "fp32": 1, "split_bf16": 2, "split_i8": 3}

    @classmethod
    def of(cls, p) -> int:
        if isinstance(p, str):
            try:
                return cls._names[p.lower()]
            except KeyError:
                raise ValueError(f"unknown precision {p!r}: use one of {sorted(cls._names)}") from None
        if int(p) not in (0, 1, 2, 3):
            raise ValueError("precision must be fp64, fp32, split_bf16 or split_i8")
        return int(p)


class _Spec(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("interaction_distance", C.c_int32),
                ("repetitions", C.c_int32), ("routing", C.c_int32),
                ("coef_z", C.c_double), ("coef_xx", C.c_double),
                ("gate_split", C.c_int32), ("reserved", C.c_int32 * 3)]


class _Gate(C.Structure):
    _fields_ = [("op", C.c_int32), ("site", C.c_int32), ("feat_i", C.c_int32), ("feat_j", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int32), ("max_bond", C.c_int32), ("pad_max", C.c_int32),
                ("n_two_qubit_gates", C.c_int32), ("max_discarded", C.c_double),
                ("mean_total_discarded", C.c_double), ("degenerate_cuts", C.c_int64),
                ("unconverged_svds", C.c_int64), ("bytes_f64", C.c_int64), ("bytes_f32", C.c_int64),
                ("bytes_split_bf16", C.c_int64), ("bytes_split_i8", C.c_int64)]


class _Job(C.Structure):
    _fields_ = [("a", C.c_void_p), ("b", C.c_void_p), ("a0", C.c_int64), ("na", C.c_int64),
                ("b0", C.c_int64), ("nb", C.c_int64), ("upper_only", C.c_int32), ("reserved", C.c_int32),
                ("K_dev", C.c_void_p), ("ldk", C.c_int64)]


class _GramStats(C.Structure):
    _fields_ = [("entries", C.c_int64), ("tiles", C.c_int64), ("workgroups", C.c_int32),
                ("tile_side", C.c_int32), ("queues", C.c_int32), ("block", C.c_int32),
                ("flops", C.c_double), ("kernel_ms", C.c_double)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


class _Tune(C.Structure):
    _fields_ = [("maxp", C.c_int32), ("tile_side", C.c_int32), ("queues", C.c_int32),
                ("n_candidates", C.c_int32), ("best_ms", C.c_double), ("default_ms", C.c_double)]


_PROGRESS = C.CFUNCTYPE(C.c_int, C.c_int64, C.c_int64, C.c_void_p)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run `python -m paper_2411_09336_amd.build`")
    L = C.CDLL(_LIB_PATH)
    P, I32, I64, D, S = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_int
    sig = {
        "qk_init": (S, [C.c_int, C.POINTER(_Allocator)]),
        "qk_last_error": (C.c_char_p, []),
        "qk_version": (C.c_char_p, []),
        "qk_circuit_compile": (S, [C.POINTER(_Spec), P, I64, C.POINTER(I64)]),
        "mps_simulate": (S, [P, I64, C.POINTER(_Spec), I32, D, P, C.POINTER(P)]),
        "mps_simulate_progress": (S, [P, I64, C.POINTER(_Spec), I32, D, P, _PROGRESS, P, I64, C.POINTER(P)]),
        "mps_simulate_graph": (S, [P, I64, C.POINTER(_Spec), I32, D, I64, P, C.POINTER(P)]),
        "mps_simulate_trace": (S, [P, I64, C.POINTER(_Spec), I32, D, P, P, C.POINTER(P)]),
        "mps_gram": (S, [P, P, C.c_int, P, I64, P, C.POINTER(_GramStats)]),
        "mps_gram_block": (S, [P, I64, I64, P, I64, I64, I32, C.c_int, P, I64, P, C.POINTER(_GramStats)]),
        "mps_gram_block_noalloc": (S, [P, I64, I64, P, I64, I64, I32, C.c_int, P, I64, P]),
        "mps_gram_multi": (S, [C.POINTER(_Job), I32, C.c_int, P, C.POINTER(_GramStats)]),
        "mps_batch_save": (S, [P, C.c_char_p]),
        "mps_batch_load": (S, [C.c_char_p, P, C.POINTER(P)]),
        "mps_batch_import": (S, [P, P, I64, I32, P, C.POINTER(P)]),
        "mps_batch_info": (S, [P, C.POINTER(_Info)]),
        "mps_batch_bond_dims": (S, [P, P]),
        "mps_batch_trunc_stats": (S, [P, P, P]),
        "mps_batch_export": (S, [P, I64, P, I64, C.POINTER(I64)]),
        "mps_batch_pack": (S, [P, C.c_int, P]),
        "mps_batch_drop": (S, [P, C.c_int]),
        "mps_batch_gather": (S, [P, P, I64, C.c_uint32, P, C.POINTER(P)]),
        "mps_batch_free": (None, [P]),
        "mps_gram_autotune": (S, [P, C.c_int, I64, P, C.POINTER(_Tune)]),
        "mps_gram_tune_reset": (S, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    _default_allocator(L)
    return L


def _default_allocator(L):
    """Batches and scratch buffers of the current device come from PyTorch's
    caching allocator unless QKMPS_ALLOCATOR=hip (then hipMalloc)."""
    if os.environ.get("QKMPS_ALLOCATOR", "torch") != "torch":
        return
    try:
        import torch
        if not torch.cuda.is_available():
            return
        dev = torch.cuda.current_device()
    except Exception:
        return
    _register(L, dev, "torch")


def _check(st: int):
    if st != 0:
        raise QKError(st, _load().qk_last_error().decode())


def version() -> str:
    return _load().qk_version().decode()


# An allocator registered with the library must outlive every batch made
# through it (a batch frees its memory through the allocator that made it):
# the callbacks are kept here for the life of the process, and the batches
# still alive when the interpreter exits are freed first (while torch can
# still take their memory back).
_ALLOCATOR_KEEP = []
_LIVE = None


def _torch_alloc(nbytes, _ctx, stream):
    try:
        import torch
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=torch.cuda.current_device(),
                                                  stream=int(stream or 0))
    except Exception:       # out of memory or no device: the library reports QK_ENOMEM
        return None


def _torch_free(ptr, _ctx, _stream):
    try:
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


def _free_live_batches():
    if _LIVE is not None:
        for b in list(_LIVE):
            b.free()


def init(device: int = 0, allocator="torch") -> None:
    """Select ``device`` and the device memory the library uses for batches
    and scratch buffers: "torch" (PyTorch's caching allocator, so the batches
    count in torch.cuda.memory_allocated() and share its pool), None
    (hipMalloc / hipMallocAsync), or a pair of callables
    ``(alloc(nbytes, stream) -> int pointer or 0, free(pointer, stream))``."""
    L = _load()
    if allocator is None:
        _check(L.qk_init(int(device), None))
        return
    _register(L, device, allocator)


def _register(L, device, allocator):
    global _LIVE
    import atexit
    import weakref
    if allocator == "torch":
        a = _Allocator(_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free), None)
    else:
        fa, ff = allocator

        def _a(nbytes, _ctx, stream):
            try:
                return fa(int(nbytes), int(stream or 0)) or None
            except Exception:
                return None

        def _f(ptr, _ctx, stream):
            try:
                ff(int(ptr), int(stream or 0))
            except Exception:
                pass
        a = _Allocator(_ALLOC_FN(_a), _FREE_FN(_f), None)
    _ALLOCATOR_KEEP.append(a)
    if _LIVE is None:
        _LIVE = weakref.WeakSet()
        atexit.register(_free_live_batches)
    _check(L.qk_init(int(device), C.byref(a)))


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


@dataclass(frozen=True)
class CircuitSpec:
    """Circuit of Sec. II-C: Rz(coef_z x_i), Rxx(coef_xx (1-x_i)(1-x_j)) at distance <= d."""
    n_qubits: int
    distance: int
    reps: int
    coef_z: float = 2.0
    coef_xx: float = 2.0
    routing: int = 0
    gate_split: int = 0

    def _c(self) -> _Spec:
        s = _Spec()
        s.n_qubits, s.interaction_distance, s.repetitions, s.routing = (
            self.n_qubits, self.distance, self.reps, self.routing)
        s.coef_z, s.coef_xx = float(self.coef_z), float(self.coef_xx)
        s.gate_split = int(self.gate_split)
        return s


def circuit_compile(spec: CircuitSpec) -> np.ndarray:
    """Gate list (n_gates x 4 int32: op, site, feat_i, feat_j) built by the library."""
    L = _load()
    cs = spec._c()
    n = C.c_int64(0)
    _check(L.qk_circuit_compile(C.byref(cs), None, 0, C.byref(n)))
    out = np.zeros((n.value, 4), dtype=np.int32)
    if n.value:
        _check(L.qk_circuit_compile(C.byref(cs), out.ctypes.data, n.value, C.byref(n)))
    return out


class MPSBatch:
    """Owning handle of a device-resident MPS batch."""

    def __init__(self, handle: int):
        self._h = C.c_void_p(handle)
        if _LIVE is not None:
            _LIVE.add(self)

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h and self._h.value:
            _load().mps_batch_free(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self) -> dict:
        inf = _Info()
        _check(_load().mps_batch_info(self._h, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _Info._fields_}

    @property
    def n(self) -> int:
        return self.info()["n"]

    @property
    def m(self) -> int:
        return self.info()["m"]

    def bond_dims(self) -> np.ndarray:
        inf = self.info()
        out = np.zeros((inf["n"], inf["m"] + 1), dtype=np.int32)
        _check(_load().mps_batch_bond_dims(self._h, out.ctypes.data))
        return out

    def trunc_stats(self):
        n = self.info()["n"]
        disc = np.zeros(n)
        deg = np.zeros(n, dtype=np.int32)
        _check(_load().mps_batch_trunc_stats(self._h, disc.ctypes.data, deg.ctypes.data))
        return disc, deg

    def export(self, idx: int) -> List[np.ndarray]:
        """FP64 tensors of MPS ``idx`` as a list of (D_l, 2, D_{l+1}) complex arrays."""
        dims = self.bond_dims()[idx]
        m = len(dims) - 1
        need = int(sum(4 * dims[l] * dims[l + 1] for l in range(m)))
        buf = np.zeros(need)
        wr = C.c_int64(0)
        _check(_load().mps_batch_export(self._h, idx, buf.ctypes.data, need, C.byref(wr)))
        out, off = [], 0
        for l in range(m):
            dl, dr = int(dims[l]), int(dims[l + 1])
            cnt = 2 * dl * dr
            z = buf[2 * off: 2 * (off + cnt)].view(np.complex128).reshape(2, dl, dr)
            out.append(np.ascontiguousarray(z.transpose(1, 0, 2)))
            off += cnt
        return out

    def pack(self, precision, stream=None):
        _check(_load().mps_batch_pack(self._h, Precision.of(precision), _stream_ptr(stream)))

    def drop(self, precision):
        _check(_load().mps_batch_drop(self._h, Precision.of(precision)))

    def save(self, path: str) -> None:
        """Write the batch (bond dimensions, statistics, FP64 tensors) to ``path``."""
        _check(_load().mps_batch_save(self._h, os.fsencode(path)))

    def gather(self, indices: Sequence[int], forms=("fp64",), stream=None) -> "MPSBatch":
        """Copies of MPS ``indices`` in the given forms ("fp64", "fp32", "split_bf16", "split_i8")."""
        idx = np.ascontiguousarray(np.asarray(indices, dtype=np.int64))
        mask = 0
        for f in forms:
            mask |= 1 << Precision.of(f)
        h = C.c_void_p(0)
        _check(_load().mps_batch_gather(self._h, idx.ctypes.data, len(idx), mask, _stream_ptr(stream),
                                        C.byref(h)))
        return MPSBatch(h.value)


def load_batch(path: str, stream=None) -> MPSBatch:
    """A batch written by ``MPSBatch.save``, on the current device."""
    h = C.c_void_p(0)
    _check(_load().mps_batch_load(os.fsencode(path), _stream_ptr(stream), C.byref(h)))
    return MPSBatch(h.value)


def import_batch(mps_list: Sequence[Sequence[np.ndarray]], stream=None) -> MPSBatch:
    """Upload MPS given as lists of (D_l, 2, D_{l+1}) complex arrays."""
    n = len(mps_list)
    if n == 0:
        raise ValueError("empty MPS list")
    m = len(mps_list[0])
    dims = np.zeros((n, m + 1), dtype=np.int32)
    parts = []
    for i, mps in enumerate(mps_list):
        if len(mps) != m:
            raise ValueError("MPS of different lengths")
        dims[i, 0] = mps[0].shape[0]
        for l, t in enumerate(mps):
            dims[i, l + 1] = t.shape[2]
            parts.append(np.ascontiguousarray(np.asarray(t, dtype=np.complex128).transpose(1, 0, 2)).reshape(-1))
    flat = np.ascontiguousarray(np.concatenate(parts)).view(np.float64)
    h = C.c_void_p(0)
    _check(_load().mps_batch_import(flat.ctypes.data, dims.ctypes.data, n, m, _stream_ptr(stream), C.byref(h)))
    return MPSBatch(h.value)


def simulate(features, spec: CircuitSpec, chi: int, cutoff: float, stream=None, progress=None,
             every: int = 0, graph_circuits=None) -> MPSBatch:
    """Truncated MPS simulation of every row of ``features`` (a CUDA float64 tensor, n x m).

    ``progress(done, total)`` (optional) is called every ``every`` two-qubit
    gates; returning True aborts.  ``graph_circuits`` (not with ``progress``)
    records the simulation of that many circuits as one HIP graph and
    replays it over the batch (0: equal chunks of at most 1024 circuits)."""
    import torch
    if not isinstance(features, torch.Tensor) or features.device.type != "cuda":
        raise TypeError("features must be a CUDA tensor")
    x = features.to(torch.float64).contiguous()
    if x.dim() != 2 or x.shape[1] != spec.n_qubits:
        raise ValueError("features must be n x n_qubits")
    cs = spec._c()
    h = C.c_void_p(0)
    if graph_circuits is not None:
        if progress is not None:
            raise ValueError("progress callbacks are not available with graph replay")
        _check(_load().mps_simulate_graph(C.c_void_p(x.data_ptr()), x.shape[0], C.byref(cs), int(chi),
                                          float(cutoff), int(graph_circuits), _stream_ptr(stream), C.byref(h)))
    elif progress is None:
        _check(_load().mps_simulate(C.c_void_p(x.data_ptr()), x.shape[0], C.byref(cs), int(chi), float(cutoff),
                                    _stream_ptr(stream), C.byref(h)))
    else:
        cb = _PROGRESS(lambda done, total, _u: 1 if progress(int(done), int(total)) else 0)
        _check(_load().mps_simulate_progress(C.c_void_p(x.data_ptr()), x.shape[0], C.byref(cs), int(chi),
                                             float(cutoff), _stream_ptr(stream), cb, None, int(every),
                                             C.byref(h)))
    return MPSBatch(h.value)


def simulate_trace(features, spec: CircuitSpec, chi: int, cutoff: float, stream=None):
    """``simulate`` that also returns the memory trace: an int32 CUDA tensor
    (n, n_two_qubit_gates, 2) holding, after each two-qubit gate, the bond
    dimension at its cut and sum_l D_l D_{l+1} over the MPS (its FP64 tensors
    take 32 bytes times that value)."""
    import torch
    if not isinstance(features, torch.Tensor) or features.device.type != "cuda":
        raise TypeError("features must be a CUDA tensor")
    x = features.to(torch.float64).contiguous()
    if x.dim() != 2 or x.shape[1] != spec.n_qubits:
        raise ValueError("features must be n x n_qubits")
    n2q = int((circuit_compile(spec)[:, 0] != 0).sum())
    trace = torch.zeros((x.shape[0], n2q, 2), dtype=torch.int32, device=x.device)
    cs = spec._c()
    h = C.c_void_p(0)
    _check(_load().mps_simulate_trace(C.c_void_p(x.data_ptr()), x.shape[0], C.byref(cs), int(chi), float(cutoff),
                                      C.c_void_p(trace.data_ptr()), _stream_ptr(stream), C.byref(h)))
    return MPSBatch(h.value), trace


def autotune(batch: MPSBatch, precision="fp64", sample: int = 64, stream=None) -> dict:
    """Time every Gram kernel configuration of ``precision`` on the symmetric
    Gram of the first ``sample`` MPS of ``batch`` and keep the fastest for
    later Gram calls on batches with the same pad bucket."""
    r = _Tune()
    _check(_load().mps_gram_autotune(batch.handle, Precision.of(precision), int(sample), _stream_ptr(stream),
                                     C.byref(r)))
    return {f: getattr(r, f) for f, _ in _Tune._fields_}


def autotune_reset() -> None:
    """Back to the default Gram kernel configurations."""
    _check(_load().mps_gram_tune_reset())


def _check_out(out, na: int, nb: int, what: str = "out"):
    """A caller-supplied K block must be a CUDA float64 matrix with unit column
    stride that holds na x nb entries: the kernels write K[i * ldk + j]
    through its pointer with ldk = out.stride(0)."""
    import torch
    if not isinstance(out, torch.Tensor) or out.dim() != 2:
        raise ValueError(f"{what} must be a 2-D torch tensor")
    if out.dtype != torch.float64:
        raise ValueError(f"{what} must be float64 (got {out.dtype})")
    if out.shape[0] < na or out.shape[1] < nb:
        raise ValueError(f"{what} of shape {tuple(out.shape)} cannot hold {na} x {nb} entries")
    if nb > 1 and out.stride(1) != 1:
        raise ValueError(f"{what} must have unit column stride (got strides {out.stride()})")
    if na > 1 and out.stride(0) < nb:
        raise ValueError(f"{what} row stride {out.stride(0)} is below the {nb} columns written")
    if not out.is_cuda:
        raise ValueError(f"{what} must live on the GPU")


def _ldk(out, nb: int) -> int:
    return max(int(out.stride(0)), nb, 1)


def _stats_arg(stats):
    return C.byref(stats) if stats is not None else None


def _stats_dict(st) -> dict:
    return {f: getattr(st, f) for f, _ in _GramStats._fields_}


def gram(a: MPSBatch, b: Optional[MPSBatch] = None, precision="fp64", out=None, stream=None,
         stats: Optional[dict] = None):
    """K[i, j] = |<a_i|b_j>|^2 as a CUDA float64 tensor (symmetric when b is None).
    With a dict ``stats`` the call waits for the kernel and fills the dict
    with its statistics (entries, tiles, workgroups, configuration,
    algorithmic flops, kernel_ms)."""
    import torch
    na = a.n
    nb = na if b is None else b.n
    if out is None:
        out = torch.empty((na, nb), dtype=torch.float64, device="cuda")
    _check_out(out, na, nb)
    st = _GramStats() if stats is not None else None
    _check(_load().mps_gram(a.handle, None if b is None else b.handle, Precision.of(precision),
                            C.c_void_p(out.data_ptr()), _ldk(out, nb), _stream_ptr(stream), _stats_arg(st)))
    if st is not None:
        stats.update(_stats_dict(st))
    return out


def gram_block(a: MPSBatch, a0: int, na: int, b: MPSBatch, b0: int, nb: int, precision="fp64",
               upper_only: bool = False, out=None, stream=None, stats: Optional[dict] = None):
    import torch
    if out is None:
        out = torch.zeros((na, nb), dtype=torch.float64, device="cuda")
    _check_out(out, na, nb)
    st = _GramStats() if stats is not None else None
    _check(_load().mps_gram_block(a.handle, a0, na, b.handle, b0, nb, int(bool(upper_only)),
                                  Precision.of(precision), C.c_void_p(out.data_ptr()), _ldk(out, nb),
                                  _stream_ptr(stream), _stats_arg(st)))
    if st is not None:
        stats.update(_stats_dict(st))
    return out


def gram_block_noalloc(a: MPSBatch, a0: int, na: int, b: MPSBatch, b0: int, nb: int, out, precision="fp64",
                       upper_only: bool = False, stream=None):
    """mps_gram_block_noalloc: gram_block into the caller's ``out`` with no
    device allocation (the batches must already be packed in ``precision``;
    the work queue lives in the library's static per-device scratch)."""
    _check_out(out, na, nb)
    _check(_load().mps_gram_block_noalloc(a.handle, a0, na, b.handle, b0, nb, int(bool(upper_only)),
                                          Precision.of(precision), C.c_void_p(out.data_ptr()), _ldk(out, nb),
                                          _stream_ptr(stream)))
    return out


def gram_multi(jobs, precision="fp64", stream=None, stats: Optional[dict] = None):
    """jobs: list of dicts {a, b, a0, na, b0, nb, upper_only, out} -> one persistent launch."""
    arr = (_Job * len(jobs))()
    for k, j in enumerate(jobs):
        _check_out(j["out"], j["na"], j["nb"], f"jobs[{k}]['out']")
        arr[k].a = j["a"].handle.value
        arr[k].b = j["b"].handle.value
        arr[k].a0, arr[k].na = j.get("a0", 0), j["na"]
        arr[k].b0, arr[k].nb = j.get("b0", 0), j["nb"]
        arr[k].upper_only = int(bool(j.get("upper_only", False)))
        arr[k].reserved = 0
        arr[k].K_dev = j["out"].data_ptr()
        arr[k].ldk = _ldk(j["out"], j["nb"])
    st = _GramStats() if stats is not None else None
    _check(_load().mps_gram_multi(arr, len(jobs), Precision.of(precision), _stream_ptr(stream), _stats_arg(st)))
    if st is not None:
        stats.update(_stats_dict(st))
