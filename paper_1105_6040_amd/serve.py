"""Serving loop: sort requests admitted by free HBM and batched on the device.

Requests are (uint32 key, uint32 value) arrays of different lengths arriving
over time; their payloads and result buffers are resident on the device.
Two servers share the request model and the statistics:

``StepServer`` -- continuous batching.  The device runs one *step* at a time,
  one launch of the library's ``sort_step`` over every active request, each
  advancing by one phase (a request of at most one LDS tile is sorted in its
  only phase; a longer one has a histogram phase and one phase per 8-bit
  digit pass).  At every step boundary the loop, in real time:

  * admits arrivals into a FIFO queue;
  * retires the requests whose last phase ran in a step the device has
    finished (recording latency from arrival to observed completion) and
    releases their per-request state;
  * admits queued requests while their per-request state (``work``: digit
    histograms, look-back rows and ping-pong buffers, sized by the library)
    fits in the HBM budget and a slot is free -- they join the next step at
    phase 0, alongside requests in the middle of their passes;
  * enqueues the next step while fewer than ``max_steps_inflight`` steps are
    queued on the device (steps of one request run in stream order, so the
    host never waits for a step before queueing the next one).

  Optionally (``direct`` + ``direct_above``) requests longer than a threshold
  skip the steps: each is one launch of its whole sort on streams of its own,
  admitted by the same HBM budget from a queue of its own, and runs on the
  device beside the steps.  A step then lasts as long as the phases of the
  short requests in it, not of the longest one admitted.

``Server`` -- the baseline: one launch per request (sort_pairs), the same
  admission by workspace bytes, launches round robin over a few streams.

Latency percentiles are nearest-rank.  The schedulers do not depend on the
device: an executor does the launches.  ``GpuStepExecutor`` / ``GpuExecutor``
drive the HIP library; ``FakeStepExecutor`` / ``FakeExecutor`` (tests)
complete work on the CPU after a simulated duration.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Dict, List, Sequence

from . import markers


@dataclasses.dataclass
class Request:
    rid: int
    n: int
    arrival: float          # seconds from the start of the trace
    offset: int = 0         # first pair of this request in the pool
    launched: float = math.nan
    done: float = math.nan
    path: str = ""          # "step" (continuous batching) or "single"
    phases: int = 0         # step phases (StepServer)
    phase: int = 0          # next phase to run (StepServer)
    work: object = None     # executor's per-request state (StepServer)
    work_bytes: int = 0
    marker: int = 0         # roctx range of the request (markers.py)

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


@dataclasses.dataclass
class ServeStats:
    latencies_ms: List[float]
    pairs: int
    wall_s: float
    launches: int
    max_inflight_seen: int
    budget_waits: int
    max_reserved_bytes: int = 0
    max_active: int = 0

    @property
    def p50_ms(self) -> float:
        return percentile(self.latencies_ms, 50)

    @property
    def p99_ms(self) -> float:
        return percentile(self.latencies_ms, 99)

    @property
    def gkeys_per_s(self) -> float:
        return self.pairs / self.wall_s / 1e9 if self.wall_s > 0 else math.nan

    @property
    def requests_per_s(self) -> float:
        return len(self.latencies_ms) / self.wall_s if self.wall_s > 0 else math.nan

    def as_dict(self) -> Dict[str, float]:
        return {"requests": len(self.latencies_ms), "p50_ms": round(self.p50_ms, 4), "p99_ms": round(self.p99_ms, 4),
                "GKeys_per_s": round(self.gkeys_per_s, 4), "req_per_s": round(self.requests_per_s, 1),
                "launches": self.launches, "wall_s": round(self.wall_s, 4), "max_inflight": self.max_inflight_seen,
                "max_active": self.max_active, "budget_waits": self.budget_waits,
                "max_reserved_bytes": self.max_reserved_bytes}


def _stats(reqs: List[Request], launches: int, max_seen: int, waits: int, max_used: int,
           max_active: int = 0) -> ServeStats:
    wall = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return ServeStats([r.latency * 1e3 for r in reqs], sum(r.n for r in reqs), wall, launches, max_seen, waits,
                      max_used, max_active)


def make_requests(arrivals, lengths) -> List[Request]:
    reqs, off = [], 0
    for rid, (a, n) in enumerate(zip(arrivals, lengths)):
        reqs.append(Request(rid=rid, n=int(n), arrival=float(a), offset=off))
        off += int(n)
    return reqs


# =========================================================================== continuous batching
class StepExecutor:
    """Runs steps of the continuous-batching server on a device."""

    max_requests_per_step = 1024

    def plan(self, n: int):
        """(phases, work bytes) of a request of n pairs."""
        raise NotImplementedError

    def admit(self, r: Request) -> None:
        """Allocate r.work (r.work_bytes bytes of per-request state)."""

    def step(self, batch: List[Request]):
        """Enqueue one step: every request of `batch` runs its phase r.phase.
        Returns a handle for finished()."""
        raise NotImplementedError

    def finished(self, handle) -> bool:
        raise NotImplementedError

    def release(self, r: Request) -> None:
        r.work = None

    def join(self) -> None:
        """Order the caller's later work after every step (device executors)."""


class StepServer:
    def __init__(self, executor: StepExecutor, budget_bytes: int, max_active: int = 1024,
                 max_steps_inflight: int = 2, clock=time.perf_counter, direct: "Executor" = None,
                 direct_above: int = None, direct_inflight: int = 2):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = min(int(max_active), executor.max_requests_per_step)
        self.max_steps_inflight = int(max_steps_inflight)
        self.clock = clock
        # Requests of more than `direct_above` pairs skip the steps: each is
        # one launch of its whole sort on the `direct` executor's streams,
        # running beside the steps (at most `direct_inflight` at once).
        self.direct = direct if direct_above is not None else None
        self.direct_above = direct_above
        self.direct_inflight = max(1, int(direct_inflight))

    def run(self, reqs: List[Request]) -> ServeStats:
        reqs = sorted(reqs, key=lambda r: r.arrival)
        dx = self.direct
        for r in reqs:
            if dx is not None and r.n > self.direct_above:
                r.path = "single"
                r.phases, r.work_bytes = 0, dx.workspace_bytes(r.n)
            else:
                r.path = "step"
                r.phases, r.work_bytes = self.ex.plan(r.n)
            r.phase = 0
        queue: "collections.deque[Request]" = collections.deque()   # waiting for steps
        dqueue: "collections.deque[Request]" = collections.deque()  # waiting for a launch of their own
        active: List[Request] = []
        inflight: "collections.deque" = collections.deque()  # (handle, requests finishing in that step, marker)
        dinflight: List[tuple] = []                          # (handle, request) of direct launches
        used = i = done = steps = waits = max_used = max_seen = max_act = dlaunches = slot = 0
        t0 = self.clock()
        while done < len(reqs):
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                (dqueue if reqs[i].path == "single" else queue).append(reqs[i])
                i += 1
            # Retire, in step order, what the device has finished.
            while inflight and self.ex.finished(inflight[0][0]):
                _, fin, mk = inflight.popleft()
                t = self.clock() - t0
                markers.stop(mk)
                for r in fin:
                    r.done = t
                    used -= r.work_bytes
                    self.ex.release(r)
                    markers.stop(r.marker)
                done += len(fin)
            if dinflight:
                still = []
                for h, r in dinflight:
                    if dx.finished(h):
                        r.done = self.clock() - t0
                        used -= r.work_bytes
                        dx.release(h)
                        markers.stop(r.marker)
                        done += 1
                    else:
                        still.append((h, r))
                dinflight = still
            # Admit into free slots and memory; an empty device always takes
            # the head request (so that a request above the budget still runs).
            blocked = False
            while queue and len(active) < self.max_active:
                r = queue[0]
                if used + r.work_bytes > self.budget and (active or inflight or dinflight):
                    blocked = True
                    break
                queue.popleft()
                self.ex.admit(r)
                used += r.work_bytes
                max_used = max(max_used, used)
                r.launched = self.clock() - t0
                r.marker = markers.start(f"request {r.rid} n={r.n} step")
                active.append(r)
            while dqueue and len(dinflight) < self.direct_inflight:
                r = dqueue[0]
                if used + r.work_bytes > self.budget and (active or inflight or dinflight):
                    blocked = True
                    break
                dqueue.popleft()
                used += r.work_bytes
                max_used = max(max_used, used)
                r.launched = self.clock() - t0
                r.marker = markers.start(f"request {r.rid} n={r.n} single")
                dinflight.append((dx.launch(r, slot), r))
                slot += 1
                dlaunches += 1
            if blocked:
                waits += 1
            if active and len(inflight) < self.max_steps_inflight:
                mk = markers.start(f"step {steps} requests={len(active)}")
                h = self.ex.step(active)
                steps += 1
                fin, keep = [], []
                for r in active:
                    r.phase += 1
                    (fin if r.phase >= r.phases else keep).append(r)
                inflight.append((h, fin, mk))
                max_seen = max(max_seen, len(inflight))
                max_act = max(max_act, len(active))
                active = keep
                continue
            if not (active or inflight or dinflight or queue or dqueue) and i < len(reqs):
                wait = reqs[i].arrival - (self.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.0005))
        self.ex.join()
        if dx is not None:
            dx.join()
        return _stats(reqs, steps + dlaunches, max_seen, waits, max_used, max_act)


class FakeStepExecutor(StepExecutor):
    """CPU stand-in for the step engine: a request of at most `small` pairs
    has one phase, a longer one 5 (histogram + four 8-bit digit passes); a
    step finishes `overhead + seconds_per_pair * pairs in it` after it is
    enqueued, steps run one after another.  `sort_fn(keys, vals)` (e.g. the
    oracle) writes a request's result when its last phase is enqueued."""

    def __init__(self, keys, vals, sort_fn, seconds_per_pair=1e-9, step_overhead=20e-6, small=8192,
                 clock=time.perf_counter):
        self.keys, self.vals = keys, vals
        self.out_k = keys.copy()
        self.out_v = vals.copy()
        self.sort_fn = sort_fn
        self.spp = seconds_per_pair
        self.overhead = step_overhead
        self.small = small
        self.clock = clock
        self.device_free_at = 0.0
        self.phase_log: List[List[tuple]] = []   # per step: (rid, phase)

    def plan(self, n):
        phases = 0 if n == 0 else (1 if n <= self.small else 5)
        return phases, (0 if n <= self.small else 8 * n + 4096)

    def step(self, batch):
        self.phase_log.append([(r.rid, r.phase) for r in batch])
        for r in batch:
            if r.phase == r.phases - 1:
                a, b = r.offset, r.offset + r.n
                k, v = self.sort_fn(self.keys[a:b], self.vals[a:b])
                self.out_k[a:b], self.out_v[a:b] = k, v
        start = max(self.clock(), self.device_free_at)
        self.device_free_at = start + self.overhead + self.spp * sum(r.n for r in batch)
        return self.device_free_at

    def finished(self, handle) -> bool:
        return self.clock() >= handle


class GpuStepExecutor(StepExecutor):
    """Steps on the HIP library (sort_step).  keys/vals: uint32 device tensors
    holding every request's payload in arrival order; results go to
    out_k/out_v at the same positions.  Each step's descriptor table is
    written into a pinned host slot and copied to a device slot on the step
    stream; `ring` slots are reused round robin (a slot is rewritten only
    after the step that read it has retired, which the server's bound on
    steps in flight guarantees)."""

    def __init__(self, keys, vals, out_k, out_v, ring: int = 8):
        import numpy as np
        import torch

        from . import _native as N
        self.np, self.torch, self.N = np, torch, N
        self.keys, self.vals, self.out_k, self.out_v = keys, vals, out_k, out_v
        self.device = keys.device
        self.stream = torch.cuda.Stream(device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self.max_requests_per_step = N.MS_STEP_MAX_REQUESTS
        rec = N.MS_STEP_REQUEST_BYTES
        self.ring = ring
        self.host = torch.empty((ring, self.max_requests_per_step * rec), dtype=torch.uint8, pin_memory=True)
        self.table = torch.empty((ring, self.max_requests_per_step * rec), dtype=torch.uint8, device=self.device)
        self.host_rec = self.host.numpy().view(N.STEP_REQUEST_DTYPE)
        self.ws = torch.empty(max(1, N.workspace_size(N.MS_OP_SORT_STEP, N.MS_KEY_U32, True, 0,
                                                      self.max_requests_per_step)),
                              dtype=torch.uint8, device=self.device)
        self.slot = 0
        self.k_base, self.v_base = keys.data_ptr(), vals.data_ptr()
        self.ok_base, self.ov_base = out_k.data_ptr(), out_v.data_ptr()
        self.events = []

    def plan(self, n):
        return self.N.step_plan(self.N.MS_KEY_U32, True, n)

    def admit(self, r):
        if r.work_bytes:
            with self.torch.cuda.stream(self.stream):
                r.work = self.torch.empty(r.work_bytes, dtype=self.torch.uint8, device=self.device)

    def step(self, batch):
        np, torch, N = self.np, self.torch, self.N
        s = self.slot
        self.slot = (s + 1) % self.ring
        m = len(batch)
        rec = self.host_rec[s][:m]
        off = np.fromiter((r.offset for r in batch), dtype=np.uint64, count=m) * np.uint64(4)
        rec["keys_in"] = off + np.uint64(self.k_base)
        rec["vals_in"] = off + np.uint64(self.v_base)
        rec["keys_out"] = off + np.uint64(self.ok_base)
        rec["vals_out"] = off + np.uint64(self.ov_base)
        rec["work"] = np.fromiter((r.work.data_ptr() if r.work is not None else 0 for r in batch), dtype=np.uint64,
                                  count=m)
        rec["n"] = np.fromiter((r.n for r in batch), dtype=np.uint64, count=m)
        rec["phase"] = np.fromiter((r.phase for r in batch), dtype=np.uint32, count=m)
        rec["reserved"] = 0
        nbytes = m * N.MS_STEP_REQUEST_BYTES
        with torch.cuda.stream(self.stream):
            self.table[s, :nbytes].copy_(self.host[s, :nbytes], non_blocking=True)
            N.check(N.lib().sort_step(self.table[s].data_ptr(), m, N.MS_KEY_U32, 1, self.ws.data_ptr(),
                                      self.ws.numel(), self.stream.cuda_stream), "sort_step")
            ev = torch.cuda.Event()
            ev.record(self.stream)
        return ev

    def finished(self, handle) -> bool:
        return handle.query()

    def release(self, r):
        # The caching allocator reuses the block only for work queued after
        # this point on the step stream, i.e. after the request's last step.
        if r.work is not None:
            r.work.record_stream(self.stream)
        r.work = None

    def join(self) -> None:
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)


# =========================================================================== one launch per request
class Executor:
    """Launches whole requests and reports completion (baseline server)."""

    def workspace_bytes(self, pairs: int) -> int:
        raise NotImplementedError

    def launch(self, r: Request, stream_slot: int):
        raise NotImplementedError

    def finished(self, handle) -> bool:
        raise NotImplementedError

    def release(self, handle) -> None:
        pass

    def join(self) -> None:
        """Order the caller's later work after every launch (device executors)."""


class Server:
    """One launch per request, admitted by workspace bytes, round robin over streams."""

    def __init__(self, executor: Executor, budget_bytes: int, max_inflight: int = 4, streams: int = 2,
                 clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.streams = streams
        self.clock = clock

    def run(self, reqs: List[Request]) -> ServeStats:
        reqs = sorted(reqs, key=lambda r: r.arrival)
        queue: "collections.deque[Request]" = collections.deque()
        inflight = []  # (handle, request, reserved)
        used = i = done = launches = max_seen = max_used = waits = slot = 0
        t0 = self.clock()
        while done < len(reqs):
            now = self.clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                queue.append(reqs[i])
                i += 1
            still = []
            for h, r, reserved in inflight:
                if self.ex.finished(h):
                    r.done = self.clock() - t0
                    done += 1
                    used -= reserved
                    self.ex.release(h)
                    markers.stop(r.marker)
                else:
                    still.append((h, r, reserved))
            inflight = still
            progressed = False
            while queue and len(inflight) < self.max_inflight:
                r = queue[0]
                need = self.ex.workspace_bytes(r.n)
                if used + need > self.budget and inflight:
                    waits += 1
                    break  # wait for memory to free up
                queue.popleft()
                r.launched = self.clock() - t0
                r.path = "single"
                r.marker = markers.start(f"request {r.rid} n={r.n} single")
                h = self.ex.launch(r, slot % self.streams)
                slot += 1
                launches += 1
                used += need
                max_used = max(max_used, used)
                inflight.append((h, r, need))
                max_seen = max(max_seen, len(inflight))
                progressed = True
            if not progressed and not inflight and i < len(reqs):
                wait = reqs[i].arrival - (self.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.0005))
        self.ex.join()
        return _stats(reqs, launches, max_seen, waits, max_used)


class FakeExecutor(Executor):
    """CPU stand-in: a launch finishes after `overhead + seconds_per_pair * n`.
    `sort_fn(keys, vals) -> (keys, vals)` (e.g. the oracle) produces results."""

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

    def workspace_bytes(self, pairs: int) -> int:
        return pairs * self.ws_per_pair + 256

    def launch(self, r, stream_slot):
        a, b = r.offset, r.offset + r.n
        k, v = self.sort_fn(self.keys[a:b], self.vals[a:b])
        self.out_k[a:b], self.out_v[a:b] = k, v
        return self.clock() + self.overhead + self.spp * r.n

    def finished(self, handle) -> bool:
        return self.clock() >= handle


class GpuExecutor(Executor):
    """One sort_pairs per request on the HIP library.  keys/vals: uint32
    device tensors holding every request's payload in arrival order; results
    go to out_k/out_v at the same positions."""

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

    def workspace_bytes(self, pairs: int) -> int:
        N = self.N
        return N.workspace_size(N.MS_OP_SORT_PAIRS, N.MS_KEY_U32, True, pairs)

    def launch(self, r, stream_slot):
        torch = self.torch
        from . import api
        s = self.streams[stream_slot % len(self.streams)]
        a, b = r.offset, r.offset + r.n
        with torch.cuda.stream(s):
            ws = torch.empty(max(1, self.workspace_bytes(b - a)), dtype=torch.uint8, device=self.device)
            api.sort_pairs(self.keys[a:b], self.vals[a:b], self.out_k[a:b], self.out_v[a:b], ws=ws)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, ws)

    def finished(self, handle) -> bool:
        return handle[0].query()
