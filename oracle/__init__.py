"""CPU oracle for the paper's scatter / sort / merge method -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package.  The GPU library never does, and the oracle imports
nothing from it: the two share no code.  The arithmetic lives in ``oracle.c``
(plain C, compiled with gcc into ``liboracle.so`` next to it); this module only
marshals NumPy arrays through ctypes.

Every function returns the stable ascending sort the paper's method reaches
(El-Nashar 2011, Section 3.2, Figures 1-3): keys in the key type's natural order
(signed for int32, unsigned for uint32 / uint64), equal keys in their original
order, values travelling with their keys.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_DEFAULT = os.path.join(_HERE, "liboracle.so")

# key type codes used by oracle.c
KT_CODES = {np.dtype(np.int32): 0, np.dtype(np.uint32): 1, np.dtype(np.uint64): 2}

_lib = None


def build(out: str = _LIB_DEFAULT, src: str = _SRC, extra_flags=()) -> str:
    """Compile oracle.c with gcc into a shared object; returns its path."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", *extra_flags,
           src, "-o", out + ".tmp", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ORACLE_LIB", _LIB_DEFAULT)
    if path == _LIB_DEFAULT and (not os.path.exists(path)
                                 or os.path.getmtime(path) < os.path.getmtime(_SRC)):
        build(path)
    lib = ctypes.CDLL(path)
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    for name in ("oracle_sort", "oracle_bubble"):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int, vp, vp, vp, vp, u64]
        fn.restype = ctypes.c_int
    for name in ("oracle_sort_segmented", "oracle_merge_runs"):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp, u64]
        fn.restype = ctypes.c_int
    for name in ("oracle_paper_method", "oracle_merge_split", "oracle_paper_method_threads"):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int, vp, vp, vp, vp, u64, u64]
        fn.restype = ctypes.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    pass


def _kt(keys: np.ndarray) -> int:
    try:
        return KT_CODES[keys.dtype]
    except KeyError:
        raise TypeError(f"oracle: unsupported key dtype {keys.dtype}") from None


def _prep(keys, vals):
    keys = np.ascontiguousarray(keys)
    if keys.ndim != 1:
        raise ValueError("oracle: keys must be 1-D")
    kt = _kt(keys)
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
        if vals.shape != keys.shape:
            raise ValueError("oracle: values must match keys in length")
    kout = np.empty_like(keys)
    vout = None if vals is None else np.empty_like(vals)
    return kt, keys, vals, kout, vout


def _p(a):
    return None if a is None else a.ctypes.data


def _check(rc: int, what: str):
    if rc == -2:
        raise OracleError(f"{what}: precondition violated (offsets or unsorted run)")
    if rc != 0:
        raise OracleError(f"{what}: failed with code {rc}")


def _ret(kout, vout):
    return kout if vout is None else (kout, vout)


def sort(keys, vals=None):
    """Stable ascending sort (Figure 3 merge sort).  Returns keys, or (keys, vals)."""
    kt, keys, vals, kout, vout = _prep(keys, vals)
    _check(_load().oracle_sort(kt, _p(keys), _p(vals), _p(kout), _p(vout), keys.size),
           "oracle_sort")
    return _ret(kout, vout)


def bubble(keys, vals=None):
    """Figure 2's bubble sort (strict '>' exchange).  O(n^2): tiny inputs only."""
    kt, keys, vals, kout, vout = _prep(keys, vals)
    _check(_load().oracle_bubble(kt, _p(keys), _p(vals), _p(kout), _p(vout), keys.size),
           "oracle_bubble")
    return _ret(kout, vout)


def _offsets(offsets):
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    if off.ndim != 1 or off.size < 1:
        raise ValueError("oracle: offsets must be 1-D with at least one entry")
    return off


def sort_segmented(keys, offsets, vals=None):
    """Every segment [off[s], off[s+1]) sorted on its own."""
    kt, keys, vals, kout, vout = _prep(keys, vals)
    off = _offsets(offsets)
    if int(off[-1]) != keys.size:
        raise ValueError("oracle: offsets[-1] must equal len(keys)")
    _check(_load().oracle_sort_segmented(kt, _p(keys), _p(vals), _p(kout), _p(vout),
                                         off.ctypes.data, off.size - 1), "oracle_sort_segmented")
    return _ret(kout, vout)


def merge_runs(keys, offsets, vals=None):
    """Master merge (Section 3.2.2) of adjacent sorted runs [off[r], off[r+1])."""
    kt, keys, vals, kout, vout = _prep(keys, vals)
    off = _offsets(offsets)
    if off.size < 2:
        raise ValueError("oracle: merge_runs needs at least one run")
    if int(off[-1]) != keys.size:
        raise ValueError("oracle: offsets[-1] must equal len(keys)")
    _check(_load().oracle_merge_runs(kt, _p(keys), _p(vals), _p(kout), _p(vout),
                                     off.ctypes.data, off.size - 1), "oracle_merge_runs")
    return _ret(kout, vout)


def paper_method(keys, p, vals=None):
    """Figure 1 with the Section 3.2.2 master merge: p parts, each sorted, merged."""
    kt, keys, vals, kout, vout = _prep(keys, vals)
    _check(_load().oracle_paper_method(kt, _p(keys), _p(vals), _p(kout), _p(vout),
                                       keys.size, int(p)), "oracle_paper_method")
    return _ret(kout, vout)


def paper_method_threads(keys, p, vals=None):
    """As paper_method, with each part sorted on its own thread (timing only)."""
    kt, keys, vals, kout, vout = _prep(keys, vals)
    _check(_load().oracle_paper_method_threads(kt, _p(keys), _p(vals), _p(kout), _p(vout),
                                               keys.size, int(p)), "oracle_paper_method_threads")
    return _ret(kout, vout)


def merge_split(keys, p, vals=None):
    """Figure 1's merge phase read as odd/even transposition merge-split over p parts."""
    kt, keys, vals, kout, vout = _prep(keys, vals)
    _check(_load().oracle_merge_split(kt, _p(keys), _p(vals), _p(kout), _p(vout),
                                      keys.size, int(p)), "oracle_merge_split")
    return _ret(kout, vout)


def part_offsets(n: int, p: int) -> np.ndarray:
    """Part boundaries of the scatter phase: part i = [floor(i*n/p), floor((i+1)*n/p))."""
    return np.array([(i * n) // p for i in range(p + 1)], dtype=np.uint64)
