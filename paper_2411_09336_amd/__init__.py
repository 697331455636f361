"""MI355X-native quantum-kernel Gram matrices from matrix product states.

The compute path is the HIP library ``libqkmps.so`` (C ABI declared in
``include/qkmps.h``); this package is a thin ctypes binding over it.  PyTorch
tensors are used only to hold device memory and to name HIP streams.

Importing the package does not load the library; the first call does, and it
raises ``RuntimeError`` if the library has not been built
(``python -m paper_2411_09336_amd.build``).
"""
from .api import (  # noqa: F401
    CircuitSpec, MPSBatch, QKError, Precision, autotune, autotune_reset, circuit_compile, gram, gram_block,
    gram_block_noalloc, gram_multi, import_batch, init, library_path, load_batch, simulate, simulate_trace, version,
)
