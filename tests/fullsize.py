"""Full-size parity against the oracle on the host's cores.

The oracle is single-threaded C; these helpers only spread independent oracle
calls over host threads (ctypes releases the GIL for the duration of a foreign
call) and stream device results to the host in chunks, so that lists of 2^28
keys and the 50,000-segment workload (4.56e9 keys) are compared with the
oracle element by element in tens of seconds.  No sorting arithmetic lives
here: every expected value is an oracle call's output.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import sys

import numpy as np
import torch

import oracle

# The host's share of cores for one GPU.
THREADS = max(1, min(16, os.cpu_count() or 1))


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def oracle_whole(keys: np.ndarray, vals: np.ndarray | None = None, parts: int = THREADS):
    """The oracle's stable sort of a whole list, through the method itself:
    `parts` contiguous parts each sorted on its own host thread, then the
    master merge (Figure 1 with Section 3.2.2; pinned equal to the plain
    oracle sort on the CPU)."""
    return oracle.paper_method_threads(keys, parts, vals)


def _chunks_of_segments(off: np.ndarray, target: int):
    """Consecutive groups of whole segments of about `target` keys each:
    list of (first segment, end segment)."""
    out, s, nseg = [], 0, off.size - 1
    while s < nseg:
        want = int(off[s]) + target
        e = int(np.searchsorted(off, want, side="right")) - 1
        e = max(e, s + 1)
        e = min(e, nseg)
        out.append((s, e))
        s = e
    return out


def compare_segments(k_dev: torch.Tensor, out_dev: torch.Tensor, off: np.ndarray,
                     v_dev: torch.Tensor | None = None, vout_dev: torch.Tensor | None = None,
                     chunk_keys: int = 1 << 27, big_segment: int = 1 << 26) -> int:
    """Every segment of a device sort_segmented result against the oracle,
    element by element.  Chunks of whole segments are copied to the host and
    sorted by the oracle on THREADS threads; a segment of at least
    `big_segment` keys is sorted by oracle_whole on its own.  Returns the
    number of segments compared."""
    nseg = off.size - 1
    off64 = off.astype(np.int64)
    done = 0
    pool = cf.ThreadPoolExecutor(max_workers=THREADS)
    try:
        for (s0, s1) in _chunks_of_segments(off, chunk_keys):
            a, b = int(off64[s0]), int(off64[s1])
            kin = k_dev[a:b].cpu().numpy()
            got = out_dev[a:b].cpu().numpy()
            vin = v_dev[a:b].cpu().numpy() if v_dev is not None else None
            vgot = vout_dev[a:b].cpu().numpy() if vout_dev is not None else None
            loc = off64[s0:s1 + 1] - a
            if s1 - s0 == 1 and b - a >= big_segment:
                exp = oracle_whole(kin, vin)
                ek, ev = exp if vin is not None else (exp, None)
                assert np.array_equal(got, ek), f"segment {s0} differs from the oracle"
                if vin is not None:
                    assert np.array_equal(vgot, ev), f"segment {s0} values differ from the oracle"
                done += 1
                continue
            # Split the chunk into THREADS groups of whole segments.
            groups = _chunks_of_segments(loc.astype(np.uint64), max(1, (b - a) // THREADS + 1))

            def run(g):
                g0, g1 = g
                x, y = int(loc[g0]), int(loc[g1])
                sub = (loc[g0:g1 + 1] - x).astype(np.uint64)
                if vin is None:
                    return g, oracle.sort_segmented(kin[x:y], sub), None
                ek, ev = oracle.sort_segmented(kin[x:y], sub, vin[x:y])
                return g, ek, ev

            for (g0, g1), ek, ev in pool.map(run, groups):
                x, y = int(loc[g0]), int(loc[g1])
                if not np.array_equal(got[x:y], ek):
                    bad = next(s for s in range(g0, g1)
                               if not np.array_equal(got[loc[s]:loc[s + 1]], ek[loc[s] - x:loc[s + 1] - x]))
                    raise AssertionError(f"segment {s0 + bad} differs from the oracle")
                if ev is not None:
                    assert np.array_equal(vgot[x:y], ev), f"values of segments {s0 + g0}..{s0 + g1} differ"
            done += s1 - s0
    finally:
        pool.shutdown()
    assert done == nseg
    return done
