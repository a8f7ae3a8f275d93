"""MI355X-native stabilizer-tableau (Clifford) simulation.

The product path is libcliff.so (HIP kernels for gfx950 behind a C ABI,
declared in include/cliff.h); this package is its Python binding plus the
plumbing that gives it device memory and streams through PyTorch.
"""
from ._binding import *  # noqa: F401,F403
from ._binding import CliffError, LIB_PATH, exported_symbols  # noqa: F401
from .device import Context, DeviceTableau  # noqa: F401
