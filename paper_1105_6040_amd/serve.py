"""Serving loop: sort requests admitted by free HBM, batched on the device.

Requests are (uint32 key, uint32 value) arrays of different lengths arriving
over time.  Their payloads are staged on the device in arrival order, one
contiguous pool, so any run of consecutive requests is one contiguous range
that a single segmented launch can sort (each request a segment).  The
scheduler loop, in real time:

  * admits arrivals into a FIFO queue;
  * retires finished work (HIP events on the launch streams), recording each
    request's latency (arrival to observed completion) and releasing its
    workspace reservation;
  * launches while the number of launches in flight is below `max_inflight`
    and the workspace the next launch needs fits in the HBM budget: a run of
    consecutive short requests at the head of the queue (each at most
    `large_threshold` pairs, together at most `max_batch_pairs`) becomes one
    sort_segmented launch; a long request at the head is launched alone as
    sort_pairs (its digit passes spread over every CU).  Launches go round
    robin over several streams, so work admitted while other work runs
    overlaps with it on the device.

The baseline server launches every request on its own (sort_pairs), with the
same admission and streams.  Latency percentiles are nearest-rank.

The scheduler is independent of the device: an Executor does the launches.
``GpuExecutor`` drives the HIP library; ``FakeExecutor`` (tests) completes
requests on the CPU after a simulated duration.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Dict, List, Optional, Sequence


@dataclasses.dataclass
class Request:
    rid: int
    n: int
    arrival: float          # seconds from the start of the trace
    offset: int = 0         # first pair of this request in the pool
    launched: float = math.nan
    done: float = math.nan
    path: str = ""          # "batch" or "single"

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def percentile(xs: Sequence[float], q: float) -> float:
    """Nearest-rank percentile (q in (0, 100])."""
    s = sorted(xs)
    if not s:
        return math.nan
    k = max(1, math.ceil(q * len(s) / 100.0))
    return s[min(k, len(s)) - 1]


class Executor:
    """Launches work and reports completion; subclasses talk to a device."""

    def workspace_bytes(self, pairs: int, segments: int) -> int:
        raise NotImplementedError

    def launch(self, reqs: List[Request], stream_slot: int):
        """Start sorting `reqs` (consecutive in the pool); returns a handle."""
        raise NotImplementedError

    def finished(self, handle) -> bool:
        raise NotImplementedError

    def release(self, handle) -> None:
        pass

    def join(self) -> None:
        """Order the caller's later work after every launch (device executors)."""


@dataclasses.dataclass
class ServeStats:
    latencies_ms: List[float]
    pairs: int
    wall_s: float
    launches: int
    max_inflight_seen: int
    budget_waits: int
    max_reserved_bytes: int = 0

    @property
    def p50_ms(self) -> float:
        return percentile(self.latencies_ms, 50)

    @property
    def p99_ms(self) -> float:
        return percentile(self.latencies_ms, 99)

    @property
    def gkeys_per_s(self) -> float:
        return self.pairs / self.wall_s / 1e9 if self.wall_s > 0 else math.nan

    def as_dict(self) -> Dict[str, float]:
        return {"requests": len(self.latencies_ms), "p50_ms": round(self.p50_ms, 4), "p99_ms": round(self.p99_ms, 4),
                "GKeys_per_s": round(self.gkeys_per_s, 4), "launches": self.launches,
                "wall_s": round(self.wall_s, 4), "max_inflight": self.max_inflight_seen,
                "budget_waits": self.budget_waits, "max_reserved_bytes": self.max_reserved_bytes}


class Server:
    def __init__(self, executor: Executor, budget_bytes: int, batching: bool = True,
                 large_threshold: int = 1 << 18, max_batch_pairs: int = 1 << 24, max_inflight: int = 4,
                 streams: int = 2, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.batching = batching
        self.large_threshold = large_threshold
        self.max_batch_pairs = max_batch_pairs
        self.max_inflight = max_inflight
        self.streams = streams
        self.clock = clock

    def _next_unit(self, queue: "collections.deque[Request]") -> List[Request]:
        head = queue[0]
        if not self.batching or head.n > self.large_threshold:
            return [head]
        unit, total = [], 0
        for r in queue:
            if r.n > self.large_threshold or total + r.n > self.max_batch_pairs:
                break
            if unit and r.rid != unit[-1].rid + 1:
                break  # only consecutive requests share a contiguous range
            unit.append(r)
            total += r.n
        return unit or [head]

    def run(self, reqs: List[Request]) -> ServeStats:
        reqs = sorted(reqs, key=lambda r: r.arrival)
        queue: "collections.deque[Request]" = collections.deque()
        inflight = []  # (handle, units, reserved)
        used = 0
        i = 0
        done = 0
        launches = 0
        max_seen = 0
        max_used = 0
        waits = 0
        slot = 0
        t0 = self.clock()
        while done < len(reqs):
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                queue.append(reqs[i])
                i += 1
            still = []
            for h, unit, reserved in inflight:
                if self.ex.finished(h):
                    t = self.clock() - t0
                    for r in unit:
                        r.done = t
                    done += len(unit)
                    used -= reserved
                    self.ex.release(h)
                else:
                    still.append((h, unit, reserved))
            inflight = still
            progressed = False
            while queue and len(inflight) < self.max_inflight:
                unit = self._next_unit(queue)
                need = self.ex.workspace_bytes(sum(r.n for r in unit), len(unit))
                if used + need > self.budget and inflight:
                    waits += 1
                    break  # wait for memory to free up
                t = self.clock() - t0
                for r in unit:
                    queue.popleft()
                    r.launched = t
                    r.path = "batch" if len(unit) > 1 else "single"
                h = self.ex.launch(unit, slot % self.streams)
                slot += 1
                launches += 1
                used += need
                max_used = max(max_used, used)
                inflight.append((h, unit, need))
                max_seen = max(max_seen, len(inflight))
                progressed = True
            if not progressed and not inflight and i < len(reqs):
                # idle until the next arrival
                wait = reqs[i].arrival - (self.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
        self.ex.join()
        wall = max(r.done for r in reqs) - min(r.arrival for r in reqs)
        return ServeStats([r.latency * 1e3 for r in reqs], sum(r.n for r in reqs), wall, launches, max_seen, waits,
                          max_used)


def make_requests(arrivals, lengths) -> List[Request]:
    reqs, off = [], 0
    for rid, (a, n) in enumerate(zip(arrivals, lengths)):
        reqs.append(Request(rid=rid, n=int(n), arrival=float(a), offset=off))
        off += int(n)
    return reqs


class FakeExecutor(Executor):
    """CPU stand-in: a launch finishes after `cost(pairs, launches)` seconds.
    `sort_fn(keys, vals) -> (keys, vals)` (e.g. the oracle) produces results
    so tests can compare each request alone and in a batch."""

    def __init__(self, keys, vals, sort_fn, seconds_per_pair=1e-9, launch_overhead=20e-6,
                 ws_bytes_per_pair=8, clock=time.perf_counter):
        self.keys, self.vals = keys, vals
        self.out_k = keys.copy()
        self.out_v = vals.copy()
        self.sort_fn = sort_fn
        self.spp = seconds_per_pair
        self.overhead = launch_overhead
        self.ws_per_pair = ws_bytes_per_pair
        self.clock = clock
        self.max_reserved_seen = 0

    def workspace_bytes(self, pairs: int, segments: int) -> int:
        return pairs * self.ws_per_pair + 256 * segments

    def launch(self, reqs, stream_slot):
        for r in reqs:
            a, b = r.offset, r.offset + r.n
            k, v = self.sort_fn(self.keys[a:b], self.vals[a:b])
            self.out_k[a:b], self.out_v[a:b] = k, v
        return self.clock() + self.overhead + self.spp * sum(r.n for r in reqs)

    def finished(self, handle) -> bool:
        return self.clock() >= handle


class GpuExecutor(Executor):
    """Launches on the HIP library.  keys/vals: uint32 device tensors holding
    every request's payload in arrival order; results go to out_k/out_v at
    the same positions."""

    def __init__(self, keys, vals, out_k, out_v, streams: int = 2):
        import torch

        from . import _native as N
        self.torch, self.N = torch, N
        self.keys, self.vals, self.out_k, self.out_v = keys, vals, out_k, out_v
        self.device = keys.device
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        # The payload and output buffers were produced on the caller's stream;
        # the launch streams do not synchronise with it by themselves.
        caller = torch.cuda.current_stream(self.device)
        for st in self.streams:
            st.wait_stream(caller)

    def join(self) -> None:
        """Make the caller's stream wait for everything launched so far."""
        caller = self.torch.cuda.current_stream(self.device)
        for st in self.streams:
            caller.wait_stream(st)

    def workspace_bytes(self, pairs: int, segments: int) -> int:
        N = self.N
        if segments == 1:
            return N.workspace_size(N.MS_OP_SORT_PAIRS, N.MS_KEY_U32, True, pairs)
        return N.workspace_size(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_U32, True, pairs, segments)

    def launch(self, reqs, stream_slot):
        torch, N = self.torch, self.N
        from . import api
        s = self.streams[stream_slot % len(self.streams)]
        a = reqs[0].offset
        b = reqs[-1].offset + reqs[-1].n
        with torch.cuda.stream(s):
            kin, vin = self.keys[a:b], self.vals[a:b]
            kout, vout = self.out_k[a:b], self.out_v[a:b]
            if len(reqs) == 1:
                ws = torch.empty(max(1, self.workspace_bytes(b - a, 1)), dtype=torch.uint8, device=self.device)
                api.sort_pairs(kin, vin, kout, vout, ws=ws)
                off = None
            else:
                bounds = [r.offset - a for r in reqs] + [b - a]
                off = torch.tensor(bounds, dtype=torch.int64).to(self.device, non_blocking=True)
                ws = torch.empty(max(1, self.workspace_bytes(b - a, len(reqs))), dtype=torch.uint8,
                                 device=self.device)
                api.sort_segmented(kin, off, vin, kout, vout, ws=ws)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, ws, off)

    def finished(self, handle) -> bool:
        return handle[0].query()
