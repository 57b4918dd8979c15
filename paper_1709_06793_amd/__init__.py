"""MI355X-native stencil-scaling operator library (HIP kernels behind a C ABI).

The compute path is libhhg.so (include/hhg.h); `hhg` is its ctypes binding.
"""
from . import hhg  # noqa: F401
from .hhg import Context, HHGError  # noqa: F401
