"""Benchmark of the MI355X sort library (one GPU).

Headline: a stable key-only sort of 2^28 int32 keys drawn uniformly from
[0, 2^31) (the paper's "sort phase" for one whole list), inputs resident in
HBM before the clock starts.  One step = one full sort_keys call.  Prints ONE
JSON line:

  value        GKeys/s over the timed steps (n * steps / elapsed)
  roofline     the dominant kernel (the onesweep digit pass): algorithmic
               bytes per launch (read + write of every key: 2 * n * 4 B)
               divided by its mean duration from HIP events recorded on its
               own stream during the timed steps, against 8 TB/s
  cpu_baseline the CPU oracle (plain merge sort, one thread) timed on a
               bounded sample of the same keys; cpu_baseline_paper_method_threads
               the oracle's paper method with its parts sorted on host threads
  extra        the other workloads: sorted and heavy-duplicate 2^28 int32,
               2^26 (uint64, uint32) pairs, the paper's 10^5-key p = 4 method,
               and a copy-kernel HBM probe

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra] [--no-cpu] [--no-tune]
       python bench.py --psweep    (the process-count sweep instead of the headline)
       python bench.py --memory    (device bytes against list size; no GPU needed)

--no-tune runs the library's default launch parameters instead of timing
candidates first (profiling runs use it, so that only the measured kernels
appear in the trace).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "GKeys/s at 2^28 int32 vs HBM roofline; p50/p99 latency of batched sorts"
DOMINANT = "onesweep_pass"
PMC_FILE = os.path.join(ROOT, "profiles", "onesweep_pass_2p28_i32_pmc.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1105_6040_amd", "csrc", "radix.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    """Nearest-rank percentile."""
    s = sorted(xs)
    k = max(1, int(-(-q * len(s) // 100)))
    return s[min(k, len(s)) - 1]


def time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in evs]
    return wall, per


def source_hash(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def traffic_from_profile(n_launch_bytes):
    """HBM bytes per onesweep launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    try:
        rec = json.load(open(PMC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != source_hash(KERNEL_SRC):
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(keys_np, budget_s=12.0, chunk=1 << 22):
    import oracle
    done = 0
    t0 = time.perf_counter()
    chunks = 0
    while True:
        a = keys_np[chunks * chunk:(chunks + 1) * chunk]
        if a.size == 0:
            break
        oracle.sort(a)
        done += a.size
        chunks += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": round(done / el / 1e9, 6), "unit": "GKeys/s", "cores": 1, "kind": "oracle",
            "sample": f"{chunks} chunk(s) of {chunk} keys (2^22) of the same 2^28 int32 input, each "
                      f"sorted by the single-threaded oracle merge sort; {el:.1f} s"}


def cpu_baseline_threads(keys_np, budget_s=12.0):
    """The oracle's paper method with its parts sorted on host threads (p =
    the threads used, at most 16: the host cores one GPU gets), then merged by
    the master merge, on the largest power-of-two prefix of the same keys that
    stays within the budget."""
    import oracle
    p = max(1, min(16, os.cpu_count() or 1))
    n = 1 << 20
    el = 0.0
    while True:
        t0 = time.perf_counter()
        oracle.paper_method_threads(keys_np[:n], p)
        el = time.perf_counter() - t0
        if el * 2.2 > budget_s or 2 * n > keys_np.size:
            break
        n *= 2
    return {"value": round(n / el / 1e9, 6), "unit": "GKeys/s", "cores": p, "kind": "oracle",
            "sample": f"the first {n} keys of the same 2^28 int32 input: {p} parts sorted on {p} threads by "
                      f"the oracle merge sort, then the master merge; {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--psweep", action="store_true",
                    help="instead of the headline: the process-count sweep (paper's method, p = 1..64)")
    ap.add_argument("--memory", action="store_true",
                    help="instead of the headline: device bytes against list size (no GPU needed)")
    ap.add_argument("--segments", action="store_true",
                    help="instead of the headline: the 50,000-segment batched sort alone, after a 1 GiB "
                         "device copy (the copy calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (no multi-GPU path is built)",
              file=sys.stderr)
        sys.exit(2)

    if args.memory:
        print(json.dumps(memory_table()), flush=True)
        return

    import numpy as np
    import torch

    from paper_1105_6040_amd import _native as N
    from paper_1105_6040_amd import api, inputs

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.psweep:
        print(json.dumps(process_sweep(dev, stream)), flush=True)
        return
    if args.segments:
        a = torch.zeros(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        _, cper = time_steps(lambda: b.copy_(a), 5, 2, stream)
        del a, b
        res = segments_workload(dev, stream)
        res["copy_probe_GBps"] = round(2 * (1 << 28) * 4 / (sorted(cper)[len(cper) // 2] * 1e-3) / 1e9, 1)
        print(json.dumps({"segments_50k": res}), flush=True)
        return
    n = 1 << 28
    log("generating 2^28 int32 uniform keys")
    keys_np = inputs.keys_2p28("uniform", seed=0)
    keys = torch.from_numpy(keys_np).to(dev)
    out = torch.empty_like(keys)
    ws = torch.empty(N.workspace_size(N.MS_OP_SORT_KEYS, N.MS_KEY_I32, False, n), dtype=torch.uint8, device=dev)
    run = lambda: api.sort_keys(keys, out=out, ws=ws)  # noqa: E731

    # HBM probe: a plain device copy of the 1 GiB key array (1 GiB read + 1 GiB
    # written).  Its duration gives achievable bandwidth; under rocprofv3 its
    # byte counters calibrate those of the sort kernels.
    log("copy probe")
    _, cper = time_steps(lambda: out.copy_(keys), 5, 2, stream)
    copy_probe = {"bytes_per_launch": 2 * n * 4, "ms_median": round(sorted(cper)[len(cper) // 2], 4),
                  "GBps": round(2 * n * 4 / (sorted(cper)[len(cper) // 2] * 1e-3) / 1e9, 1)}

    from paper_1105_6040_amd import tune
    if args.no_tune:
        tuned = {"params": [N.tune_get(N.MS_TUNE_PASS_THREADS), N.tune_get(N.MS_TUNE_HIST_BLOCKS)], "trials": []}
    else:
        log("autotuning the headline sort")
        tuned = tune.Tuner(cache_path=None, reps=3).tune_sort(keys)
    log("timing headline")
    N.timing_reset()
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    N.timing_enable(True)
    N.timing_reset()
    wall, per = time_steps(run, args.steps, 0, stream)
    N.timing_enable(False)
    kt = N.timing_read()
    N.timing_reset()
    ms_per_step = wall * 1e3 / args.steps
    value = n * args.steps / wall / 1e9

    launches, total_ms = kt.get(DOMINANT, (0, 0.0))
    mean_ms = total_ms / max(launches, 1)
    alg_bytes = 2 * n * 4  # every key read once and written once per digit pass
    achieved = alg_bytes / (mean_ms * 1e-3) / 1e9 if launches else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4) if achieved else None,
                "traffic": traffic_from_profile(alg_bytes), "kernel": DOMINANT,
                "mean_launch_ms": round(mean_ms, 4), "launches": launches,
                "algorithmic_bytes_per_launch": alg_bytes}
    kernel_ms = {k: round(v[1] / max(v[0], 1), 4) for k, v in kt.items()}

    # correctness spot check of the timed output (sortedness)
    o = out[: 1 << 20].cpu().numpy()
    assert np.all(o[:-1] <= o[1:])

    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "GKeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": "stable key-only sort of 2^28 int32 keys uniform in [0, 2^31), 1 GPU",
                   "n": n, "key": "int32", "distribution": "uniform [0, 2^31)", "seed": 0,
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(percentile(per, 50), 4), "p99": round(percentile(per, 99), 4)},
        "roofline": roofline,
        "kernel_mean_ms": kernel_ms,
        "hbm_copy_probe": copy_probe,
        "tuning": {"pass_threads": tuned["params"][0], "hist_blocks": tuned["params"][1],
                   "trials_ms": tuned["trials"]},
    }
    del out, ws
    torch.cuda.empty_cache()

    if not args.no_extra:
        result["extra"] = extra_workloads(args, dev, stream, keys, keys_np)
    if not args.no_cpu:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(keys_np)
        log("cpu baseline, paper method on threads")
        result["cpu_baseline_paper_method_threads"] = cpu_baseline_threads(keys_np)
    print(json.dumps(result), flush=True)


def extra_workloads(args, dev, stream, keys_u, keys_u_np):
    import numpy as np
    import torch

    from paper_1105_6040_amd import _native as N
    from paper_1105_6040_amd import api, inputs

    ex = {}
    steps = max(5, args.steps // 2)

    for dist in ("sorted", "dup"):
        log(f"2^28 int32 {dist}")
        k_np = inputs.keys_2p28(dist, seed=0)
        k = torch.from_numpy(k_np).to(dev)
        o = torch.empty_like(k)
        ws = torch.empty(N.workspace_size(0, 0, False, k.numel()), dtype=torch.uint8, device=dev)
        wall, per = time_steps(lambda: api.sort_keys(k, out=o, ws=ws), steps, 2, stream)
        ex[f"keys_2p28_{dist}"] = {"GKeys_per_s": round(k.numel() * steps / wall / 1e9, 3),
                                   "ms_median": round(sorted(per)[len(per) // 2], 4)}
        del k, o, ws

    log("2^26 u64/u32 pairs")
    pk_np, pv_np = inputs.pairs_2p26(seed=0)
    pk, pv = torch.from_numpy(pk_np).to(dev), torch.from_numpy(pv_np).to(dev)
    ok, ov = torch.empty_like(pk), torch.empty_like(pv)
    ws = torch.empty(N.workspace_size(1, 2, True, pk.numel()), dtype=torch.uint8, device=dev)
    N.timing_enable(True)
    N.timing_reset()
    wall, per = time_steps(lambda: api.sort_pairs(pk, pv, ok, ov, ws=ws), steps, 2, stream)
    N.timing_enable(False)
    kt = N.timing_read()
    N.timing_reset()
    c, t = kt.get(DOMINANT, (0, 0.0))
    pass_ms = t / max(c, 1)
    ex["pairs_2p26_u64_u32"] = {"GPairs_per_s": round(pk.numel() * steps / wall / 1e9, 3),
                                "ms_median": round(sorted(per)[len(per) // 2], 4),
                                "onesweep_pass_GBps": round(2 * pk.numel() * 12 / (pass_ms * 1e-3) / 1e9, 1)
                                if c else None}
    del pk, pv, ok, ov, ws

    log("paper method 10^5, p = 4")
    k_np, p = inputs.paper_small(0)
    k, toff = torch.from_numpy(k_np).to(dev), api.part_offsets(k_np.size, p, dev)
    s_out, m_out = torch.empty_like(k), torch.empty_like(k)

    def paper():
        api.sort_segmented(k, toff, keys_out=s_out)
        api.merge_runs(s_out, toff, keys_out=m_out)
    wall, per = time_steps(paper, 100, 10, stream)
    ex["paper_small_p4"] = {"us_median": round(sorted(per)[len(per) // 2] * 1e3, 1),
                            "us_p99": round(percentile(per, 99) * 1e3, 1)}
    # The paper's method (parts sorted, then merged) must give the whole-list sort.
    assert torch.equal(m_out, api.sort_keys(k)), "paper method differs from sort_keys"
    # The same two calls captured once in a HIP graph and replayed back to back
    # (no allocation, memset or host wait inside a call, so they capture).
    ws_s = torch.empty(max(1, N.workspace_size(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, k.numel(), p)),
                       dtype=torch.uint8, device=dev)
    ws_m = torch.empty(max(1, N.workspace_size(N.MS_OP_MERGE_RUNS, N.MS_KEY_I32, False, k.numel(), p)),
                       dtype=torch.uint8, device=dev)

    def paper_ws():
        api.sort_segmented(k, toff, keys_out=s_out, ws=ws_s)
        api.merge_runs(s_out, toff, keys_out=m_out, ws=ws_m)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        paper_ws()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        paper_ws()
    m_out.zero_()
    wall_g, per_g = time_steps(graph.replay, 100, 10, stream)
    assert torch.equal(m_out, api.sort_keys(k)), "graph replay of the paper method differs from sort_keys"
    ex["paper_small_p4"]["graph_replay_us_median"] = round(sorted(per_g)[len(per_g) // 2] * 1e3, 1)
    ex["paper_small_p4"]["graph_replay_us_p99"] = round(percentile(per_g, 99) * 1e3, 1)
    del graph, ws_s, ws_m
    del k, toff, s_out, m_out

    ex["segments_50k"] = segments_workload(dev, stream)
    ex["serving"] = serving_workload(dev)
    return ex


def memory_table():
    """The paper's Experiment 2 on the GPU: device bytes the sort takes as the
    list grows, with two parts (its two processes).  Per call: the keys in,
    the keys out and the workspace the library asks for (ms_workspace_size);
    the paper's method (two parts sorted, then merged) also holds the sorted
    parts between its two calls.  Table 2's list sizes: 5..10 x 10^4 and
    2.5..5 x 10^6 int32 keys."""
    from paper_1105_6040_amd import _native as N

    K = 4
    rows = []
    for n in [k * 10**4 for k in range(5, 11)] + [k * 5 * 10**5 for k in range(5, 11)]:
        ws_sort = N.workspace_size(N.MS_OP_SORT_KEYS, N.MS_KEY_I32, False, n)
        ws_seg = N.workspace_size(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, n, 2)
        ws_merge = N.workspace_size(N.MS_OP_MERGE_RUNS, N.MS_KEY_I32, False, n, 2)
        whole = 2 * n * K + ws_sort
        method = 3 * n * K + max(ws_seg, ws_merge)  # keys, sorted parts, merged output; one workspace reused
        rows.append({"n": n, "sort_keys_bytes": whole, "sort_keys_workspace": ws_sort,
                     "paper_method_p2_bytes": method, "sort_segmented_workspace": ws_seg,
                     "merge_runs_workspace": ws_merge})
    big = [r for r in rows if r["n"] >= 2_500_000]
    slope = lambda key: (big[-1][key] - big[0][key]) / (big[-1]["n"] - big[0]["n"])  # noqa: E731
    return {"experiment": "device memory against list size (paper's Experiment 2, Table 2 sizes), int32 keys",
            "unit": "bytes", "rows": rows,
            "bytes_per_key_2p5e6_to_5e6": {"sort_keys": round(slope("sort_keys_bytes"), 3),
                                            "paper_method_p2": round(slope("paper_method_p2_bytes"), 3)}}


def process_sweep(dev, stream, reps=20, warmup=5):
    """The paper's Experiment 1 on the GPU: a list of n int32 keys (2*10^5 and
    6*10^6, Table 1's sizes) split into p = 1, 2, 4, ..., 64 contiguous parts,
    each part sorted (sort_segmented, one launch for all parts), then the p
    sorted parts merged (merge_runs: merge-path rounds), and the same merge
    by Figure 1's odd/even merge-split schedule (merge_split: p phases).
    Median of `reps` HIP-event-timed runs per phase; every result must equal
    sort_keys on the whole list."""
    import numpy as np
    import torch

    from paper_1105_6040_amd import api, inputs

    rows = []
    for n in (200_000, 6_000_000):
        log(f"process sweep n={n}")
        k = torch.from_numpy(inputs.process_sweep_keys(n, 0)).to(dev)
        ref = api.sort_keys(k)
        s_out, m_out = torch.empty_like(k), torch.empty_like(k)
        _, whole = time_steps(lambda: api.sort_keys(k, out=s_out), reps, warmup, stream)
        for p in (1, 2, 4, 8, 16, 32, 64):
            off = api.part_offsets(n, p, dev)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            sort_ms, merge_ms = [], []
            for it in range(warmup + reps):
                ev[0].record(stream)
                api.sort_segmented(k, off, keys_out=s_out)
                ev[1].record(stream)
                api.merge_runs(s_out, off, keys_out=m_out)
                ev[2].record(stream)
                torch.cuda.synchronize()
                if it >= warmup:
                    sort_ms.append(ev[0].elapsed_time(ev[1]))
                    merge_ms.append(ev[1].elapsed_time(ev[2]))
            assert torch.equal(m_out, ref), f"paper method differs from sort_keys at n={n}, p={p}"
            # The same merge phase by Figure 1's own schedule (p merge-split phases).
            _, split = time_steps(lambda: api.merge_split(s_out, p, keys_out=m_out), reps, warmup, stream)
            assert torch.equal(m_out, ref), f"merge-split differs from sort_keys at n={n}, p={p}"
            med = lambda xs: sorted(xs)[len(xs) // 2]  # noqa: E731
            rows.append({"n": n, "p": p, "sort_phase_us": round(med(sort_ms) * 1e3, 1),
                         "merge_phase_us": round(med(merge_ms) * 1e3, 1),
                         "total_us": round(med([a + b for a, b in zip(sort_ms, merge_ms)]) * 1e3, 1),
                         "merge_split_phase_us": round(med(split) * 1e3, 1),
                         "sort_keys_whole_list_us": round(med(whole) * 1e3, 1)})
            log(rows[-1])
        del k, ref, s_out, m_out
    return {"experiment": "process-count sweep (paper's Experiment 1, Table 1 sizes)", "unit": "us",
            "data": "synthetic int32 uniform [0, 2^31), seed 0", "rows": rows}


def segments_workload(dev, stream, seed=0):
    """50,000 segments, lengths log-uniform in [16, 10^6] (about 4.5e9 int32
    keys, uniform in [0, 2^31), drawn on the device from a seeded generator),
    one sort_segmented call."""
    import numpy as np
    import torch

    from paper_1105_6040_amd import _native as N
    from paper_1105_6040_amd import api, inputs

    log("segments: 50,000 log-uniform [16, 1e6]")
    lengths = inputs.segment_lengths(seed)
    off = inputs.offsets_from_lengths(lengths)
    n = int(off[-1])
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    k = torch.randint(0, 2**31, (n,), dtype=torch.int32, device=dev, generator=g)
    toff = torch.from_numpy(off).to(dev)
    out = torch.empty_like(k)
    ws = torch.empty(N.workspace_size(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, n, lengths.size),
                     dtype=torch.uint8, device=dev)
    from paper_1105_6040_amd import tune
    tuned = tune.Tuner(cache_path=None, reps=1).tune_segmented(k, toff)
    wall, per = time_steps(lambda: api.sort_segmented(k, toff, keys_out=out, ws=ws), 3, 1, stream)
    ms = sorted(per)[len(per) // 2]
    passes, threads, blocks, small = tuned["params"]
    if passes and tune.uses_segment_passes(n, lengths.size):
        choice = {"path": "segment passes", "pass_threads": threads}
    else:
        choice = {"path": "one persistent launch", "seg_blocks": blocks or 1024, "small_segment_network": bool(small)}
    one_launch = min(t for p, t in tuned["trials"] if p[0] == 0)
    res = {"segments": int(lengths.size), "keys": n, "ms_median": round(ms, 3), "tuned": choice,
           "one_persistent_launch_best_ms": one_launch,
           "tuning_trials_ms": tuned["trials"],
           "GKeys_per_s": round(n / (ms * 1e-3) / 1e9, 3),
           "GBps_at_36B_per_key": round(n * 36 / (ms * 1e-3) / 1e9, 1)}
    del k, out, ws, toff
    torch.cuda.empty_cache()
    return res


def serving_workload(dev, nreq=1000, seed=0):
    """Serving stream: requests of (uint32 key, uint32 value) pairs, lengths
    log-uniform in [1e3, 1e7], keys uniform, payloads staged on the device
    before the clock.  The one-launch-per-request server's saturation rate C
    is measured with every request arriving at once; both servers then run
    the same Poisson trace at 0.8 C."""
    import torch

    from paper_1105_6040_amd import inputs, serve

    log(f"serving: {nreq} requests")
    arr, lengths = inputs.serving_trace(seed=seed, nreq=nreq, rate_per_s=1.0)
    total = int(sum(int(x) for x in lengths))
    g = torch.Generator(device=dev)
    g.manual_seed(seed + 5)
    keys = torch.randint(-2**31, 2**31, (total,), dtype=torch.int32, device=dev, generator=g).view(torch.uint32)
    vals = torch.arange(total, dtype=torch.int32, device=dev).view(torch.uint32)
    ok, ov = torch.empty_like(keys), torch.empty_like(vals)
    free, _ = torch.cuda.mem_get_info(dev)
    budget = max(1 << 30, free - (16 << 30))

    def serve_once(batching, arrivals=None, threshold=1 << 18):
        a = arrivals if arrivals is not None else [0.0] * nreq
        reqs = serve.make_requests(a, lengths)
        ex = serve.GpuExecutor(keys, vals, ok, ov, streams=2)
        srv = serve.Server(ex, budget_bytes=budget, batching=batching, large_threshold=threshold,
                           max_batch_pairs=1 << 24, max_inflight=4, streams=2)
        st = srv.run(reqs)
        torch.cuda.synchronize()
        return st

    serve_once(False)  # warm-up
    sat = serve_once(False)
    cap = nreq / sat.wall_s
    rate = 0.8 * cap
    g2 = inputs.rng("serving", seed + 1)
    gaps = g2.exponential(1.0 / rate, nreq)
    arrivals = list(gaps.cumsum() - gaps[0])
    from paper_1105_6040_amd import tune
    tuned = tune.Tuner(cache_path=None).tune_serving(lambda t: serve_once(True, arrivals, t))
    threshold = tuned["params"][0]
    per_req = serve_once(False, arrivals)
    batched = serve_once(True, arrivals, threshold)
    return {"requests": nreq, "pairs": total, "per_request_capacity_req_per_s": round(cap, 1),
            "rate_req_per_s": round(rate, 1), "batch_threshold_pairs": threshold,
            "threshold_trials_p99_p50_ms": tuned["trials"],
            "one_launch_per_request": per_req.as_dict(), "batched": batched.as_dict()}


if __name__ == "__main__":
    main()
