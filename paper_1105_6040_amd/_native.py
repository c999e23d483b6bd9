"""ctypes binding of ``libmi355sort.so`` (the C ABI in ``include/mi355sort.h``).

Argument marshalling only: every step of every sort runs in the library's HIP
kernels.  PyTorch provides device memory (outputs and workspace come from its
caching allocator) and the current stream, whose handle is passed through.
If the shared library is missing the calls raise; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MI355SORT_LIB", os.path.join(HERE, "libmi355sort.so"))

# ms_status
MS_OK, MS_EINVAL, MS_ENOMEM, MS_EDEVICE, MS_ENOTSUP = 0, 1, 2, 3, 4
STATUS_NAMES = {0: "MS_OK", 1: "MS_EINVAL", 2: "MS_ENOMEM", 3: "MS_EDEVICE", 4: "MS_ENOTSUP"}
# ms_key_type
MS_KEY_I32, MS_KEY_U32, MS_KEY_U64 = 0, 1, 2
# ms_op
MS_OP_SORT_KEYS, MS_OP_SORT_PAIRS, MS_OP_SORT_SEGMENTED, MS_OP_MERGE_RUNS, MS_OP_MERGE_SPLIT = 0, 1, 2, 3, 4
MS_OP_SORT_STEP = 5
# continuous batching (sort_step)
MS_STEP_MAX_REQUESTS = 1024
MS_STEP_REQUEST_BYTES = 56

EXPORTS = ("ms_workspace_size", "sort_keys", "sort_pairs", "part_offsets", "sort_segmented", "merge_runs",
           "merge_split", "ms_step_plan", "sort_step", "ms_hbm_probe", "sort_keys_noalloc", "ms_last_error",
           "ms_timing_enable", "ms_timing_reset", "ms_timing_read", "ms_tune_set", "ms_tune_get")
# ms_tune_param
MS_TUNE_PASS_THREADS = 0
MS_TUNE_SEG_BLOCKS = 1
MS_TUNE_HIST_BLOCKS = 2
MS_TUNE_SMALL_SORT = 3
MS_TUNE_SEG_PASS_THREADS = 4
MS_TUNE_SEG_PASSES = 5

_lib = None
_lock = threading.Lock()


class NativeLibraryError(RuntimeError):
    """The HIP library is missing or failed to load."""


class SortError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise NativeLibraryError(
                f"{LIB_PATH} not found: build it with `python -m paper_1105_6040_amd.build` "
                "(or __graft_entry__.build()); there is no CPU fallback")
        try:
            L = ctypes.CDLL(LIB_PATH)
        except OSError as e:
            raise NativeLibraryError(f"cannot load {LIB_PATH}: {e}") from e
        vp, u64, i32, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
        L.ms_workspace_size.argtypes = [i32, i32, i32, u64, u64, ctypes.POINTER(sz)]
        L.sort_keys.argtypes = [vp, vp, u64, i32, vp, sz, vp]
        L.sort_pairs.argtypes = [vp, vp, vp, vp, u64, i32, vp, sz, vp]
        L.part_offsets.argtypes = [u64, u64, vp, vp]
        L.sort_keys_noalloc.argtypes = [vp, vp, u64, i32, vp]
        L.ms_step_plan.argtypes = [i32, i32, u64, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(sz)]
        L.sort_step.argtypes = [vp, u64, i32, i32, vp, sz, vp]
        L.ms_hbm_probe.argtypes = [i32, vp, vp, sz, vp]
        L.sort_segmented.argtypes = [vp, vp, vp, vp, vp, u64, u64, i32, vp, sz, vp]
        L.merge_runs.argtypes = [vp, vp, vp, vp, vp, u64, u64, i32, vp, sz, vp]
        L.merge_split.argtypes = [vp, vp, vp, vp, u64, u64, i32, vp, sz, vp]
        for fn in ("ms_workspace_size", "sort_keys", "sort_pairs", "part_offsets", "sort_segmented", "merge_runs",
                   "merge_split", "ms_step_plan", "sort_step", "ms_hbm_probe", "sort_keys_noalloc",
                   "ms_timing_enable", "ms_timing_reset"):
            getattr(L, fn).restype = i32
        L.ms_last_error.argtypes = []
        L.ms_last_error.restype = ctypes.c_char_p
        L.ms_timing_enable.argtypes = [i32]
        L.ms_timing_reset.argtypes = []
        L.ms_timing_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double), i32]
        L.ms_timing_read.restype = i32
        L.ms_tune_set.argtypes = [i32, ctypes.c_int64]
        L.ms_tune_set.restype = i32
        L.ms_tune_get.argtypes = [i32]
        L.ms_tune_get.restype = ctypes.c_int64
        _lib = L
        return L


def last_error() -> str:
    return lib().ms_last_error().decode(errors="replace")


def check(status: int, what: str) -> None:
    if status != MS_OK:
        raise SortError(status, f"{what}: {last_error()}")


def workspace_size(op: int, kt: int, has_values: bool, n_total: int, num_segments: int = 0) -> int:
    out = ctypes.c_size_t(0)
    check(lib().ms_workspace_size(op, kt, int(bool(has_values)), n_total, num_segments, ctypes.byref(out)),
          "ms_workspace_size")
    return out.value


def step_plan(kt: int, has_values: bool, n: int):
    """(phases, per-request work bytes) of a sort_step request of n keys."""
    ph = ctypes.c_uint32(0)
    wb = ctypes.c_size_t(0)
    check(lib().ms_step_plan(kt, int(bool(has_values)), n, ctypes.byref(ph), ctypes.byref(wb)), "ms_step_plan")
    return int(ph.value), int(wb.value)


def _step_request_dtype():
    import numpy as np
    return np.dtype([("keys_in", np.uint64), ("vals_in", np.uint64), ("keys_out", np.uint64),
                     ("vals_out", np.uint64), ("work", np.uint64), ("n", np.uint64), ("phase", np.uint32),
                     ("reserved", np.uint32)])


def __getattr__(name):
    # STEP_REQUEST_DTYPE: the NumPy layout of ms_step_request (NumPy imported lazily)
    if name == "STEP_REQUEST_DTYPE":
        return _step_request_dtype()
    raise AttributeError(name)


def tune_set(param: int, value: int) -> None:
    check(lib().ms_tune_set(param, int(value)), "ms_tune_set")


def tune_get(param: int) -> int:
    return int(lib().ms_tune_get(param))


def timing_enable(on: bool) -> None:
    check(lib().ms_timing_enable(int(bool(on))), "ms_timing_enable")


def timing_reset() -> None:
    check(lib().ms_timing_reset(), "ms_timing_reset")


def timing_read(max_entries: int = 64) -> dict:
    """{kernel name: (launches, total ms)} recorded since the last reset."""
    names = ctypes.create_string_buffer(64 * max_entries)
    counts = (ctypes.c_uint64 * max_entries)()
    ms = (ctypes.c_double * max_entries)()
    k = lib().ms_timing_read(names, counts, ms, max_entries)
    out = {}
    for i in range(min(k, max_entries)):
        name = names.raw[64 * i: 64 * (i + 1)].split(b"\0", 1)[0].decode()
        out[name] = (int(counts[i]), float(ms[i]))
    return out
