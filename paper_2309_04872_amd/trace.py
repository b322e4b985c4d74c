"""Optional roctx ranges around the binding's calls, for rocprofv3
--marker-trace: set LBW_ROCTX=1 before importing the package. Off by
default, and then a range costs one branch."""
from __future__ import annotations

import contextlib
import ctypes
import os

ENABLED = os.environ.get("LBW_ROCTX") == "1"
_LIB = None


def _roctx():
    global _LIB
    if _LIB is None:
        # rocprofv3 records the ranges of the profiler SDK's roctx library;
        # the older roctracer one is only the fallback.
        lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
        try:
            L = ctypes.CDLL(os.path.join(lib, "librocprofiler-sdk-roctx.so"))
        except OSError:
            L = ctypes.CDLL(os.path.join(lib, "libroctx64.so"))
        L.roctxRangePushA.argtypes = [ctypes.c_char_p]
        L.roctxRangePushA.restype = ctypes.c_int
        L.roctxRangePop.restype = ctypes.c_int
        _LIB = L
    return _LIB


@contextlib.contextmanager
def marker(name: str):
    """A roctx range named ``name`` around the block when enabled."""
    if not ENABLED:
        yield
        return
    L = _roctx()
    L.roctxRangePushA(name.encode())
    try:
        yield
    finally:
        L.roctxRangePop()
