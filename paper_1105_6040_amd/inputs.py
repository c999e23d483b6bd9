"""Seeded synthetic inputs for the sort workloads.

This module only draws and lays out input data; it contains none of the
sorting arithmetic, so both the GPU library's tests and the CPU oracle can be
fed from it.  Every generator is deterministic in (workload id, seed): the
NumPy PCG64 stream is ``default_rng([workload_id, seed])``.

The paper gives no distribution ("arbitrary data", Section 4, Experiment 2) and
never states the key type (only an ``int`` swap temporary, Figure 2), so the
workloads follow the benchmark configurations:

* ``paper_small``   100,000 int32 uniform in [0, 2^31), p = 4 equal parts
* ``keys_2p28``     2^28 int32: uniform in [0, 2^31), the same draw sorted
                    ascending, or heavy duplicates uniform in [0, 1023]
* ``pairs_2p26``    2^26 (uint64 key uniform in [0, 2^64), uint32 value = index)
* ``segments``      50,000 segments, lengths log-uniform in [16, 10^6]
* ``serving``       Poisson arrivals of (uint32, uint32) requests, lengths
                    log-uniform in [10^3, 10^7]
"""
from __future__ import annotations

import numpy as np

WORKLOAD_IDS = {"paper_small": 1, "keys_2p28": 2, "pairs_2p26": 3, "segments": 4, "serving": 5,
                "process_sweep": 6, "unit": 9}

DTYPES = {"i32": np.int32, "u32": np.uint32, "u64": np.uint64}


def rng(workload: str, seed: int) -> np.random.Generator:
    return np.random.default_rng([WORKLOAD_IDS[workload], int(seed)])


# --------------------------------------------------------------------------- unit cases
def keys(dtype, n: int, dist: str = "uniform", seed: int = 0) -> np.ndarray:
    """Keys of one dtype ('i32'|'u32'|'u64' or a NumPy dtype) and distribution.

    dist: uniform (whole type range), pos31 (uniform in [0, 2^31)), small
    (uniform in [0, 1023]), bits16 (whole range masked to 16 low bits), equal,
    sorted (uniform drawn then laid out ascending), reverse (strictly
    descending distinct values), few (4 distinct values), extremes (the type's
    minimum, maximum, 0 and -1 / all-ones mixed).
    """
    dt = np.dtype(DTYPES.get(dtype, dtype))
    g = rng("unit", seed * 1000003 + n)
    info = np.iinfo(dt)
    if dist in ("uniform", "sorted"):
        x = g.integers(info.min, info.max, n, dtype=dt, endpoint=True)
        if dist == "sorted":
            x = np.sort(x, kind="stable")
        return x
    if dist == "pos31":
        return g.integers(0, 2**31, n, dtype=dt)
    if dist == "small":
        return g.integers(0, 1024, n, dtype=dt)
    if dist == "bits16":
        return (g.integers(info.min, info.max, n, dtype=dt, endpoint=True) & dt.type(0xFFFF)).astype(dt)
    if dist == "equal":
        return np.full(n, dt.type(g.integers(0, 1 << 20)), dtype=dt)
    if dist == "reverse":
        return _descending(dt, n)
    if dist == "few":
        vals = g.integers(info.min, info.max, 4, dtype=dt, endpoint=True)
        return vals[g.integers(0, 4, n)]
    if dist == "extremes":
        pool = np.array(sorted({int(info.min), int(info.max), 0, int(info.max) // 2,
                                -1 if dt.kind == "i" else int(info.max) - 1}), dtype=object)
        pool = np.array([int(v) for v in pool], dtype=dt)
        return pool[g.integers(0, pool.size, n)]
    raise ValueError(f"unknown distribution {dist!r}")


def _descending(dt: np.dtype, n: int) -> np.ndarray:
    """n strictly descending distinct values of dtype dt spread over its range."""
    info = np.iinfo(dt)
    span = int(info.max) - int(info.min)
    step = max(1, span // max(n, 1))
    if dt == np.uint64:
        return np.uint64(info.max) - np.arange(n, dtype=np.uint64) * np.uint64(step)
    return (int(info.max) - np.arange(n, dtype=np.int64) * step).astype(dt)


# --------------------------------------------------------------------------- workloads
def paper_small(seed: int = 0):
    """100,000 int32 keys uniform in [0, 2^31) and p = 4 (the paper's method, small)."""
    g = rng("paper_small", seed)
    return g.integers(0, 2**31, 100_000, dtype=np.int32), 4


def process_sweep_keys(n: int, seed: int = 0) -> np.ndarray:
    """n int32 keys uniform in [0, 2^31): the lists of the process-count sweep
    (the paper's Experiment 1 sorts 2*10^5 and 6*10^6 items)."""
    g = np.random.default_rng([WORKLOAD_IDS["process_sweep"], int(n), int(seed)])
    return g.integers(0, 2**31, n, dtype=np.int32)


def keys_2p28(dist: str = "uniform", seed: int = 0, n: int = 2**28) -> np.ndarray:
    """2^28 int32 keys: 'uniform' in [0, 2^31), 'sorted' (that draw ascending), 'dup' in [0, 1023]."""
    g = rng("keys_2p28", seed)
    if dist == "dup":
        return g.integers(0, 1024, n, dtype=np.int32)
    x = g.integers(0, 2**31, n, dtype=np.int32)
    if dist == "sorted":
        x.sort(kind="stable")
    elif dist != "uniform":
        raise ValueError(dist)
    return x


def pairs_2p26(seed: int = 0, n: int = 2**26):
    """2^26 pairs: uint64 keys uniform in [0, 2^64), uint32 values = original index."""
    g = rng("pairs_2p26", seed)
    k = g.integers(0, 2**64, n, dtype=np.uint64, endpoint=False)
    return k, np.arange(n, dtype=np.uint32)


def loguniform_lengths(g: np.random.Generator, count: int, lo: int, hi: int) -> np.ndarray:
    """Integer lengths L = floor(exp(ln lo + u (ln(hi+1) - ln lo))) clipped to [lo, hi], u ~ U[0,1)."""
    u = g.random(count)
    L = np.floor(np.exp(np.log(lo) + u * (np.log(hi + 1.0) - np.log(lo)))).astype(np.int64)
    return np.clip(L, lo, hi)


def segment_lengths(seed: int = 0, nseg: int = 50_000, lo: int = 16, hi: int = 1_000_000) -> np.ndarray:
    return loguniform_lengths(rng("segments", seed), nseg, lo, hi)


def offsets_from_lengths(lengths) -> np.ndarray:
    off = np.zeros(len(lengths) + 1, dtype=np.uint64)
    np.cumsum(np.asarray(lengths, dtype=np.uint64), out=off[1:])
    return off


def segment_keys(total: int, seed: int = 0) -> np.ndarray:
    """Keys for the segmented workload: int32 uniform in [0, 2^31)."""
    g = np.random.default_rng([WORKLOAD_IDS["segments"], int(seed), 1])
    return g.integers(0, 2**31, total, dtype=np.int32)


def serving_trace(seed: int = 0, nreq: int = 2200, lo: int = 1000, hi: int = 10_000_000,
                  rate_per_s: float = 1000.0):
    """Arrival times (s, Poisson with the given rate) and request lengths."""
    g = rng("serving", seed)
    lengths = loguniform_lengths(g, nreq, lo, hi)
    gaps = g.exponential(1.0 / rate_per_s, nreq)
    return np.cumsum(gaps) - gaps[0], lengths


def serving_payload(length: int, req_id: int, seed: int = 0):
    """One request: uint32 keys uniform in [0, 2^32), uint32 values = index."""
    g = np.random.default_rng([WORKLOAD_IDS["serving"], int(seed), 2, int(req_id)])
    return g.integers(0, 2**32, int(length), dtype=np.uint32), np.arange(int(length), dtype=np.uint32)
