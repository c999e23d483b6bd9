"""roctx ranges for timelines of the serving loop.

The paper reads its runs off a timeline of communication and computation;
here rocprofv3 (``--marker-trace``) records, beside the kernel trace, one range
per request (admission to observed completion, named with its length and
path) and one per step or launch (enqueue to observed completion).

Off by default: set ``MI355SORT_MARKERS=1`` (or call ``enable(True)``).  When
off, or when ROCm's roctx library cannot be loaded, every call does nothing;
markers never change what is computed.
"""
from __future__ import annotations

import ctypes
import os

_enabled = os.environ.get("MI355SORT_MARKERS", "0") not in ("", "0")
_lib = None  # None: not loaded yet; False: unavailable


def _load():
    global _lib
    if _lib is None:
        _lib = False
        root = os.environ.get("ROCM_PATH", "/opt/rocm")
        for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so", "libroctx64.so"):
            try:
                lib = ctypes.CDLL(os.path.join(root, "lib", name))
            except OSError:
                continue
            lib.roctxRangeStartA.argtypes = [ctypes.c_char_p]
            lib.roctxRangeStartA.restype = ctypes.c_uint64
            lib.roctxRangeStop.argtypes = [ctypes.c_uint64]
            lib.roctxRangeStop.restype = None
            lib.roctxMarkA.argtypes = [ctypes.c_char_p]
            lib.roctxMarkA.restype = None
            _lib = lib
            break
    return _lib or None


def enable(on: bool = True) -> None:
    global _enabled
    _enabled = bool(on)


def enabled() -> bool:
    return _enabled and _load() is not None


def start(message: str) -> int:
    """Open a range that may end on any thread; returns its id (0 when off)."""
    if not _enabled:
        return 0
    lib = _load()
    return int(lib.roctxRangeStartA(message.encode())) if lib else 0


def stop(range_id: int) -> None:
    if _enabled and range_id:
        lib = _load()
        if lib:
            lib.roctxRangeStop(range_id)


def mark(message: str) -> None:
    if _enabled:
        lib = _load()
        if lib:
            lib.roctxMarkA(message.encode())
