"""Autotuner for the sort library's launch parameters.

Results never depend on these parameters, only speed.  For a workload class
the tuner times every candidate on synthetic data of that shape (HIP events,
median of a few repetitions), keeps the fastest, applies it with
ms_tune_set, and remembers it in a JSON cache keyed by device name and
workload class so later runs start from the known best.

Tuned per class:
  whole-list sorts  digit-pass tile (threads x 16 keys) and histogram grid
  segmented sorts   the one-launch persistent kernel (workgroup count, and
                    whether segments of at most 64 keys are ordered by a
                    comparison network -- bitonic, one wave -- or by radix
                    passes) and, for segments averaging more than 8,192
                    keys, the whole-device segment passes (pass tile: 512
                    or 1,024 threads x 16 keys; a launch per phase, or every
                    phase in one persistent launch) as further candidates
  serving           the continuous-batching server's bound on steps queued
                    on the device ahead of the one running

The radix width is fixed at 8 bits (each digit ordered by two 4-bit splits),
so it is not a tuning dimension.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time
from typing import Callable, Dict, Iterable, List, Optional, Tuple

from . import _native as N

DEFAULT_CACHE = os.environ.get("MI355SORT_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "mi355sort", "tune.json"))

PASS_THREADS = (256, 512, 1024)
HIST_BLOCKS = (128, 256, 512, 1024)
SEG_BLOCKS = (256, 512, 1024, 2048)
SMALL_SORT = (64, 0)
SEG_PASS_THREADS = (512, 1024)
# sort_segmented runs whole-device digit passes when there are several
# segments averaging more than this many keys (mi355sort.h): a launch per
# phase from SEG_PASS_MIN_AVERAGE, the one-launch work queue from
# SEG_QUEUE_MIN_AVERAGE.
SEG_PASS_MIN_AVERAGE = 8192
SEG_QUEUE_MIN_AVERAGE = 1024
SERVE_STEPS_INFLIGHT = (1, 2, 3)
# Continuous-batching server: requests above this many pairs take a launch of
# their own beside the steps (None: every request is batched), and how many of
# those launches may run at once.
SERVE_DIRECT_ABOVE = (None, 10_000, 30_000, 100_000, 300_000, 1_000_000)
SERVE_DIRECT_INFLIGHT = (2, 4)


def serving_candidates():
    """(steps queued ahead, direct threshold, direct launches in flight)."""
    out = []
    for si in SERVE_STEPS_INFLIGHT:
        for above in SERVE_DIRECT_ABOVE:
            for dinf in (SERVE_DIRECT_INFLIGHT if above is not None else SERVE_DIRECT_INFLIGHT[:1]):
                out.append((si, above, dinf))
    return out


def uses_segment_passes(n: int, nseg: int, mode: int = 1) -> bool:
    """Whether sort_segmented of n keys in nseg segments takes the
    whole-device segment passes (else the persistent kernel) when
    MS_TUNE_SEG_PASSES is `mode` (1: a launch per phase, 2: one launch)."""
    if nseg <= 1 or mode == 0:
        return False
    return n > (SEG_PASS_MIN_AVERAGE if mode == 1 else SEG_QUEUE_MIN_AVERAGE) * nseg


def size_class(n: int) -> int:
    """Workload size class: floor(log2 n), or 0 for n < 2."""
    return int(math.floor(math.log2(n))) if n >= 2 else 0


class Tuner:
    def __init__(self, cache_path: Optional[str] = DEFAULT_CACHE, reps: int = 5):
        self.cache_path = cache_path
        self.reps = reps
        self.cache: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            try:
                self.cache = json.load(open(cache_path))
            except (OSError, ValueError):
                self.cache = {}

    # -- helpers ---------------------------------------------------------------
    def _device(self) -> str:
        import torch
        return torch.cuda.get_device_name(0).replace(" ", "_")

    def _save(self) -> None:
        if not self.cache_path:
            return
        os.makedirs(os.path.dirname(self.cache_path), exist_ok=True)
        tmp = self.cache_path + ".tmp"
        json.dump(self.cache, open(tmp, "w"), indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    def _time(self, fn: Callable[[], None]) -> float:
        """Median milliseconds of `reps` runs after one warm-up."""
        import torch
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(self.reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        times.sort()
        return times[len(times) // 2]

    def _search(self, key: str, space: Iterable[Tuple], apply: Callable[[Tuple], None],
                run: Callable[[], None], force: bool) -> dict:
        if not force and key in self.cache:
            rec = self.cache[key]
            apply(tuple(rec["params"]))
            return rec
        trials = []
        for params in space:
            apply(params)
            trials.append((self._time(run), params))
        trials.sort()
        best_ms, best = trials[0]
        apply(best)
        rec = {"params": list(best), "ms": round(best_ms, 4),
               "trials": [[list(p), round(t, 4)] for t, p in trials]}
        self.cache[key] = rec
        self._save()
        return rec

    # -- workload classes --------------------------------------------------------
    def tune_sort(self, keys, vals=None, force: bool = False) -> dict:
        """Tune the whole-list sort for tensors shaped like `keys` (and `vals`)."""
        import torch

        from . import api
        kt = api.key_type(keys)
        n = keys.numel()
        key = f"{self._device()}|sort|kt{kt}|v{int(vals is not None)}|c{size_class(n)}"
        out = torch.empty_like(keys)
        vout = None if vals is None else torch.empty_like(vals)
        op = N.MS_OP_SORT_PAIRS if vals is not None else N.MS_OP_SORT_KEYS
        ws = torch.empty(max(1, N.workspace_size(op, kt, vals is not None, n)), dtype=torch.uint8,
                         device=keys.device)

        def apply(p):
            N.tune_set(N.MS_TUNE_PASS_THREADS, p[0])
            N.tune_set(N.MS_TUNE_HIST_BLOCKS, p[1])

        def run():
            if vals is None:
                api.sort_keys(keys, out=out, ws=ws)
            else:
                api.sort_pairs(keys, vals, out, vout, ws=ws)

        return self._search(key, itertools.product(PASS_THREADS, HIST_BLOCKS), apply, run, force)

    def tune_segmented(self, keys, offsets, vals=None, force: bool = False) -> dict:
        import torch

        from . import api
        kt = api.key_type(keys)
        n, nseg = keys.numel(), offsets.numel() - 1
        key = f"{self._device()}|segmented|kt{kt}|v{int(vals is not None)}|c{size_class(n)}|s{size_class(nseg)}"
        out = torch.empty_like(keys)
        vout = None if vals is None else torch.empty_like(vals)
        # Sized with the one-launch queue selected: the largest of the forms.
        saved = N.tune_get(N.MS_TUNE_SEG_PASSES)
        N.tune_set(N.MS_TUNE_SEG_PASSES, 2)
        try:
            nbytes = N.workspace_size(N.MS_OP_SORT_SEGMENTED, kt, vals is not None, n, nseg)
        finally:
            N.tune_set(N.MS_TUNE_SEG_PASSES, saved)
        ws = torch.empty(max(1, nbytes), dtype=torch.uint8, device=keys.device)

        def run():
            api.sort_segmented(keys, offsets, vals, out, vout, ws=ws)

        # (segment passes on, pass threads, persistent workgroups, small-segment network)
        persistent = [(0, SEG_PASS_THREADS[0], b, m) for b, m in itertools.product(SEG_BLOCKS, SMALL_SORT)]
        space = persistent
        if uses_segment_passes(n, nseg, 1):
            space = [(1, t, 0, SMALL_SORT[0]) for t in SEG_PASS_THREADS] + space
        if uses_segment_passes(n, nseg, 2):
            space = [(2, SEG_PASS_THREADS[0], 0, SMALL_SORT[0])] + space

        def apply(p):
            N.tune_set(N.MS_TUNE_SEG_PASSES, p[0])
            N.tune_set(N.MS_TUNE_SEG_PASS_THREADS, p[1])
            N.tune_set(N.MS_TUNE_SEG_BLOCKS, p[2])
            N.tune_set(N.MS_TUNE_SMALL_SORT, p[3])

        return self._search(key + "|v4", space, apply, run, force)

    def tune_serving(self, run_server: Callable[[tuple], "object"], force: bool = False,
                     candidates: Optional[Iterable[tuple]] = None) -> dict:
        """Pick the continuous-batching server's parameters (steps queued
        ahead, direct threshold, direct launches in flight) with the lowest
        p99 latency; run_server(params) must run a short trace (not the one
        that is reported) and return ServeStats."""
        key = f"{self._device()}|serving|steps_direct"
        if not force and key in self.cache:
            return self.cache[key]
        trials = []
        for c in (serving_candidates() if candidates is None else candidates):
            st = run_server(tuple(c))
            trials.append((st.p99_ms, st.p50_ms, list(c)))
        trials.sort(key=lambda t: (t[0], t[1]))
        rec = {"params": trials[0][2], "p99_ms": round(trials[0][0], 4),
               "trials": [[c, round(p99, 4), round(p50, 4)] for p99, p50, c in trials]}
        self.cache[key] = rec
        self._save()
        return rec
