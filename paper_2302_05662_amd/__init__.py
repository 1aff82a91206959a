"""MI355X-native SpMV with learned format selection (Auto-SpMV's run-time mode).

The compute path is libspmv.so (HIP kernels for gfx950, C ABI in
include/spmv.h); ``spmv`` is its ctypes binding with the same function names.
"""
from .spmv import *  # noqa: F401,F403
from .spmv import Handle, SpmvError, arrays_to_host, declared_functions, device_tensor  # noqa: F401
