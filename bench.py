"""Benchmark of the MI355X sort library (one GPU).

Headline: a stable key-only sort of 2^28 int32 keys drawn uniformly from
[0, 2^31) (the paper's "sort phase" for one whole list), inputs resident in
HBM before the clock starts.  One step = one full sort_keys call.  Prints ONE
JSON line:

  value        GKeys/s over the timed steps (n * steps / elapsed), timed
               with no instrumentation inside the library
  roofline     the dominant kernel (the onesweep digit pass): algorithmic
               bytes per launch (read + write of every key: 2 * n * 4 B)
               divided by its mean duration from HIP events recorded on its
               own stream around every launch during a second timed region
               of the same steps, against 8 TB/s; `traffic` is the HBM bytes
               rocprofv3 counted for it (profiles/), when taken on the
               current kernel source
  hbm_probe    the library's own streaming read / write / copy kernels over
               1 GiB: the practical ceiling beside the 8 TB/s peak
  cpu_baseline the CPU oracle (plain merge sort, one thread) on a bounded
               sample of the same keys; cpu_baselines the oracle timed for
               every configuration, with the host's core count and model
  extra        the other workloads: sorted and heavy-duplicate 2^28 int32,
               2^26 (uint64, uint32) pairs, the paper's 10^5-key p = 4
               method, the 50,000-segment batched sort on each of its paths,
               and the serving stream (continuous batching against one launch
               per request)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra] [--no-cpu] [--no-tune]
       python bench.py --psweep    (the process-count sweep instead of the headline)
       python bench.py --memory    (device bytes against list size: measured on a
                                    GPU, the workspace arithmetic without one)
       python bench.py --segments  (the 50,000-segment batched sort alone)
       python bench.py --serving   (the serving stream alone)

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
CPU_THREADS = 16  # the host cores one GPU gets


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    """Nearest-rank percentile."""
    s = sorted(xs)
    k = max(1, int(-(-q * len(s) // 100)))
    return s[min(k, len(s)) - 1]


def median(xs):
    return sorted(xs)[len(xs) // 2]


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


def host_info():
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": model,
            "threads_used": CPU_THREADS}


# ============================================================================ HBM probe
def hbm_probe(dev, stream, nbytes=1 << 30, reps=5):
    """The library's streaming kernels (ms_hbm_probe) over `nbytes`: GB/s by
    HIP events, median of `reps` launches; a copy counts its bytes read plus
    written."""
    import torch

    from paper_1105_6040_amd import _native as N

    a = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    a.fill_(7)
    b = torch.empty_like(a)
    out = {}
    names = {0: "read", 1: "write", 2: "copy", 3: "read_nt", 4: "write_nt", 5: "copy_nt"}
    for kind, name in names.items():
        def run():
            N.check(N.lib().ms_hbm_probe(kind, a.data_ptr(), b.data_ptr(), nbytes, stream.cuda_stream),
                    "ms_hbm_probe")
        _, per = time_steps(run, reps, 2, stream)
        moved = 2 * nbytes if kind in (2, 5) else nbytes
        ms = median(per)
        out[name] = {"GBps": round(moved / (ms * 1e-3) / 1e9, 1), "ms_median": round(ms, 4), "bytes": moved}
    del a, b
    torch.cuda.empty_cache()
    best_copy = max(out["copy"]["GBps"], out["copy_nt"]["GBps"])
    out["peak_GBps"] = HBM_PEAK_GBPS
    out["copy_frac_of_peak"] = round(best_copy / HBM_PEAK_GBPS, 4)
    return out


# ============================================================================ CPU baselines
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


def cpu_baselines(keys_np):
    """The oracle timed for every configuration on the host's cores (bounded
    samples; rates scale to the configuration's unit)."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    from paper_1105_6040_amd import inputs

    res = {"host": host_info()}
    p = CPU_THREADS
    # C1: the paper's method on 10^5 keys, p = 4: whole workload, single thread.
    k1, p1 = inputs.paper_small(0)
    t0 = time.perf_counter()
    oracle.paper_method(k1, p1)
    el = time.perf_counter() - t0
    res["paper_small_p4"] = {"us": round(el * 1e6, 1), "cores": 1, "sample": "the whole 10^5-key workload"}
    # C2-uniform: the whole 2^28 list by the method on host threads.
    t0 = time.perf_counter()
    oracle.paper_method_threads(keys_np, p)
    el = time.perf_counter() - t0
    res["keys_2p28_uniform"] = {"GKeys_per_s": round(keys_np.size / el / 1e9, 6), "s": round(el, 2), "cores": p,
                                "sample": f"the whole 2^28 list: {p} parts on {p} threads, then the master merge"}
    # C2-sorted / C2-dup: 2^24-key prefixes, single thread.
    for dist in ("sorted", "dup"):
        k = inputs.keys_2p28(dist, seed=0)[: 1 << 24]
        t0 = time.perf_counter()
        oracle.sort(k)
        el = time.perf_counter() - t0
        res[f"keys_2p28_{dist}"] = {"GKeys_per_s": round(k.size / el / 1e9, 6), "s": round(el, 2), "cores": 1,
                                    "sample": "the first 2^24 keys of the input, single-threaded oracle"}
    # C3: 2^26 pairs by the method on host threads.
    pk, pv = inputs.pairs_2p26(seed=0)
    t0 = time.perf_counter()
    oracle.paper_method_threads(pk, p, pv)
    el = time.perf_counter() - t0
    res["pairs_2p26_u64_u32"] = {"GPairs_per_s": round(pk.size / el / 1e9, 6), "s": round(el, 2), "cores": p,
                                 "sample": f"all 2^26 pairs: {p} parts on {p} threads, then the master merge"}
    # C4: segments of the workload spread over host threads (the first
    # segments up to ~2^28 keys).
    lengths = inputs.segment_lengths(0)
    off = inputs.offsets_from_lengths(lengths)
    m = int(np.searchsorted(off, 1 << 28, side="right")) - 1
    total = int(off[m])
    g = np.random.default_rng(0)
    keys = g.integers(0, 2**31, total, dtype=np.int32)
    groups = np.array_split(np.arange(m), p)

    def run(gr):
        if gr.size == 0:
            return 0
        a, b = int(off[gr[0]]), int(off[gr[-1] + 1])
        oracle.sort_segmented(keys[a:b], (off[gr[0]:gr[-1] + 2] - off[gr[0]]).astype(np.uint64))
        return b - a

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=p) as ex:
        done = sum(ex.map(run, groups))
    el = time.perf_counter() - t0
    res["segments_50k"] = {"GKeys_per_s": round(done / el / 1e9, 6), "s": round(el, 2), "cores": p,
                           "sample": f"the first {m} of the 50,000 segments ({done} keys), spread over {p} threads"}
    return res


# ============================================================================ main
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
                    help="instead of the headline: device bytes against list size")
    ap.add_argument("--segments", action="store_true",
                    help="instead of the headline: the 50,000-segment batched sort alone")
    ap.add_argument("--serving", action="store_true", help="instead of the headline: the serving stream alone")
    ap.add_argument("--segments-hi", type=int, default=None,
                    help="with --segments: only the workload with lengths log-uniform in [16, this]")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="measured requests of the serving stream (after 200 warm-up ones)")
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
        his = (1_000_000, 19_023) if args.segments_hi is None else (args.segments_hi,)
        names = {1_000_000: "segments_50k", 19_023: "segments_50k_hi19023"}
        print(json.dumps({names.get(hi, f"segments_50k_hi{hi}"): segments_workload(dev, stream, tune_it=not args.no_tune,
                                                                                    hi=hi) for hi in his}),
              flush=True)
        return
    if args.serving:
        print(json.dumps({"serving": serving_workload(dev, nreq=args.serving_requests,
                                                      tune_it=not args.no_tune)}), flush=True)
        return
    n = 1 << 28
    log("generating 2^28 int32 uniform keys")
    keys_np = inputs.keys_2p28("uniform", seed=0)
    keys = torch.from_numpy(keys_np).to(dev)
    out = torch.empty_like(keys)
    ws = torch.empty(N.workspace_size(N.MS_OP_SORT_KEYS, N.MS_KEY_I32, False, n), dtype=torch.uint8, device=dev)
    run = lambda: api.sort_keys(keys, out=out, ws=ws)  # noqa: E731

    log("HBM probe kernels")
    probe = hbm_probe(dev, stream)

    from paper_1105_6040_amd import tune
    if args.no_tune:
        tuned = {"params": [N.tune_get(N.MS_TUNE_PASS_THREADS), N.tune_get(N.MS_TUNE_HIST_BLOCKS)], "trials": []}
    else:
        log("autotuning the headline sort")
        tuned = tune.Tuner(cache_path=None, reps=3).tune_sort(keys)
    log("timing headline")
    N.timing_enable(False)
    wall, per = time_steps(run, args.steps, args.warmup, stream)
    ms_per_step = wall * 1e3 / args.steps
    value = n * args.steps / wall / 1e9
    # The same steps again with a HIP event pair around every launch inside
    # the library: per-kernel mean durations for the roofline.
    N.timing_reset()
    N.timing_enable(True)
    wall_i, _ = time_steps(run, args.steps, 0, stream)
    N.timing_enable(False)
    kt = N.timing_read()
    N.timing_reset()

    launches, total_ms = kt.get(DOMINANT, (0, 0.0))
    mean_ms = total_ms / max(launches, 1)
    alg_bytes = 2 * n * 4  # every key read once and written once per digit pass
    achieved = alg_bytes / (mean_ms * 1e-3) / 1e9 if launches else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1) if achieved else None, "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4) if achieved else None,
                "traffic": traffic_from_profile(alg_bytes), "kernel": DOMINANT,
                "mean_launch_ms": round(mean_ms, 4), "launches": launches,
                "algorithmic_bytes_per_launch": alg_bytes,
                "frac_of_probe_copy": round(achieved / max(probe["copy"]["GBps"], probe["copy_nt"]["GBps"]), 4)
                if achieved else None}
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
        "ms_per_step_with_kernel_events": round(wall_i * 1e3 / args.steps, 4),
        "roofline": roofline,
        "kernel_mean_ms": kernel_ms,
        "hbm_probe": probe,
        "tuning": {"pass_threads": tuned["params"][0], "hist_blocks": tuned["params"][1],
                   "trials_ms": tuned["trials"]},
    }
    del out, ws
    torch.cuda.empty_cache()

    if not args.no_extra:
        result["extra"] = extra_workloads(args, dev, stream)
    if not args.no_cpu:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(keys_np)
        log("cpu baselines per configuration")
        result["cpu_baselines"] = cpu_baselines(keys_np)
    print(json.dumps(result), flush=True)


def extra_workloads(args, dev, stream):
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
                                   "ms_median": round(median(per), 4)}
        del k, o, ws

    log("2^26 u64/u32 pairs")
    pk_np, pv_np = inputs.pairs_2p26(seed=0)
    pk, pv = torch.from_numpy(pk_np).to(dev), torch.from_numpy(pv_np).to(dev)
    ok, ov = torch.empty_like(pk), torch.empty_like(pv)
    ws = torch.empty(N.workspace_size(1, 2, True, pk.numel()), dtype=torch.uint8, device=dev)
    wall, per = time_steps(lambda: api.sort_pairs(pk, pv, ok, ov, ws=ws), steps, 2, stream)
    N.timing_reset()
    N.timing_enable(True)
    time_steps(lambda: api.sort_pairs(pk, pv, ok, ov, ws=ws), steps, 0, stream)
    N.timing_enable(False)
    kt = N.timing_read()
    N.timing_reset()
    c, t = kt.get(DOMINANT, (0, 0.0))
    pass_ms = t / max(c, 1)
    ex["pairs_2p26_u64_u32"] = {"GPairs_per_s": round(pk.numel() * steps / wall / 1e9, 3),
                                "ms_median": round(median(per), 4),
                                "onesweep_pass_GBps": round(2 * pk.numel() * 12 / (pass_ms * 1e-3) / 1e9, 1)
                                if c else None}
    del pk, pv, ok, ov, ws

    ex["paper_small_p4"] = paper_small_workload(dev, stream)
    ex["segments_50k"] = segments_workload(dev, stream, tune_it=not args.no_tune)
    # The batched configuration's stated total (~2^27 keys) with its segment
    # count: lengths log-uniform in [16, 19,023].
    ex["segments_50k_hi19023"] = segments_workload(dev, stream, tune_it=not args.no_tune, hi=19_023)
    ex["serving"] = serving_workload(dev, nreq=args.serving_requests, tune_it=not args.no_tune)
    return ex


def paper_small_workload(dev, stream):
    """The paper's method on 10^5 int32 keys with p = 4: part_offsets,
    sort_segmented over the parts, merge_runs over the sorted parts; eager and
    replayed from a HIP graph."""
    import torch

    from paper_1105_6040_amd import _native as N
    from paper_1105_6040_amd import api, inputs

    log("paper method 10^5, p = 4")
    k_np, p = inputs.paper_small(0)
    k, toff = torch.from_numpy(k_np).to(dev), api.part_offsets(k_np.size, p, dev)
    s_out, m_out = torch.empty_like(k), torch.empty_like(k)
    ws_s = torch.empty(max(1, N.workspace_size(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, k.numel(), p)),
                       dtype=torch.uint8, device=dev)
    ws_m = torch.empty(max(1, N.workspace_size(N.MS_OP_MERGE_RUNS, N.MS_KEY_I32, False, k.numel(), p)),
                       dtype=torch.uint8, device=dev)

    def paper():
        api.sort_segmented(k, toff, keys_out=s_out, ws=ws_s)
        api.merge_runs(s_out, toff, keys_out=m_out, ws=ws_m)
    _, per = time_steps(paper, 100, 10, stream)
    res = {"us_median": round(median(per) * 1e3, 1), "us_p99": round(percentile(per, 99) * 1e3, 1)}
    # The paper's method (parts sorted, then merged) must give the whole-list sort.
    assert torch.equal(m_out, api.sort_keys(k)), "paper method differs from sort_keys"
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        paper()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        paper()
    m_out.zero_()
    _, per_g = time_steps(graph.replay, 100, 10, stream)
    assert torch.equal(m_out, api.sort_keys(k)), "graph replay of the paper method differs from sort_keys"
    res["graph_replay_us_median"] = round(median(per_g) * 1e3, 1)
    res["graph_replay_us_p99"] = round(percentile(per_g, 99) * 1e3, 1)
    N.timing_reset()
    N.timing_enable(True)
    time_steps(paper, 20, 0, stream)
    N.timing_enable(False)
    res["kernel_mean_us"] = {kk: round(v[1] / max(v[0], 1) * 1e3, 1) for kk, v in N.timing_read().items()}
    N.timing_reset()
    return res


def memory_table():
    """The paper's Experiment 2 on the GPU: device bytes the sort takes as the
    list grows, for sort_keys, sort_pairs and the paper's method with two
    parts (its two processes).  With a GPU: measured -- the rise of torch's
    allocated bytes over the inputs during each call (outputs and workspace),
    beside the workspace arithmetic (ms_workspace_size); without one, the
    arithmetic alone.  Table 2's list sizes: 5..10 x 10^4 and 2.5..5 x 10^6."""
    from paper_1105_6040_amd import _native as N

    K = 4
    try:
        import torch
        gpu = torch.cuda.is_available()
    except Exception:
        gpu = False
    rows = []
    for n in [k * 10**4 for k in range(5, 11)] + [k * 5 * 10**5 for k in range(5, 11)]:
        ws_sort = N.workspace_size(N.MS_OP_SORT_KEYS, N.MS_KEY_I32, False, n)
        ws_pairs = N.workspace_size(N.MS_OP_SORT_PAIRS, N.MS_KEY_I32, True, n)
        ws_seg = N.workspace_size(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, n, 2)
        ws_merge = N.workspace_size(N.MS_OP_MERGE_RUNS, N.MS_KEY_I32, False, n, 2)
        row = {"n": n,
               "sort_keys_bytes": 2 * n * K + ws_sort, "sort_keys_workspace": ws_sort,
               "sort_pairs_bytes": 2 * n * (K + 4) + ws_pairs, "sort_pairs_workspace": ws_pairs,
               # keys, sorted parts, merged output; one workspace at a time
               "paper_method_p2_bytes": 3 * n * K + max(ws_seg, ws_merge),
               "sort_segmented_workspace": ws_seg, "merge_runs_workspace": ws_merge}
        if gpu:
            row.update(_measure_memory(n))
        rows.append(row)
    big = [r for r in rows if r["n"] >= 2_500_000]
    slope = lambda key: round((big[-1][key] - big[0][key]) / (big[-1]["n"] - big[0]["n"]), 3)  # noqa: E731
    slopes = {k[: -len("_bytes")]: slope(k) for k in rows[0] if k.endswith("_bytes")}
    return {"experiment": "device memory against list size (paper's Experiment 2, Table 2 sizes), int32 keys",
            "unit": "bytes", "measured_on_gpu": gpu, "rows": rows, "bytes_per_key_2p5e6_to_5e6": slopes}


def _measure_memory(n):
    """Peak device bytes each call allocates beyond its inputs (torch's
    allocator statistics around the call; inputs allocated before)."""
    import torch

    from paper_1105_6040_amd import api, inputs

    dev = torch.device("cuda:0")
    out = {}
    k = torch.from_numpy(inputs.process_sweep_keys(n, 0)).to(dev)
    v = torch.arange(n, dtype=torch.int32, device=dev).view(torch.uint32)

    def peak(fn):
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        base = torch.cuda.memory_allocated(dev)
        torch.cuda.reset_peak_memory_stats(dev)
        res = fn()
        torch.cuda.synchronize()
        p = torch.cuda.max_memory_allocated(dev) - base
        del res
        return p

    out["measured_sort_keys_bytes"] = peak(lambda: api.sort_keys(k)) + n * 4  # + the keys in
    out["measured_sort_pairs_bytes"] = peak(lambda: api.sort_pairs(k, v)) + n * 8

    def method():
        off = api.part_offsets(n, 2, dev)
        s = api.sort_segmented(k, off)
        return api.merge_runs(s, off)
    out["measured_paper_method_p2_bytes"] = peak(method) + n * 4
    del k, v
    return out


def process_sweep(dev, stream, reps=20, warmup=5):
    """The paper's Experiment 1 on the GPU: a list of n int32 keys (2*10^5 and
    6*10^6, Table 1's sizes) split into p = 1, 2, 4, ..., 64 contiguous parts,
    each part sorted (sort_segmented, one launch for all parts), then the p
    sorted parts merged (merge_runs: merge-path rounds), and the same merge
    by Figure 1's odd/even merge-split schedule (merge_split: p phases).
    Median of `reps` HIP-event-timed runs per phase; every result must equal
    sort_keys on the whole list."""
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
            rows.append({"n": n, "p": p, "sort_phase_us": round(median(sort_ms) * 1e3, 1),
                         "merge_phase_us": round(median(merge_ms) * 1e3, 1),
                         "total_us": round(median([a + b for a, b in zip(sort_ms, merge_ms)]) * 1e3, 1),
                         "merge_split_phase_us": round(median(split) * 1e3, 1),
                         "sort_keys_whole_list_us": round(median(whole) * 1e3, 1)})
            log(rows[-1])
        del k, ref, s_out, m_out
    return {"experiment": "process-count sweep (paper's Experiment 1, Table 1 sizes)", "unit": "us",
            "data": "synthetic int32 uniform [0, 2^31), seed 0", "rows": rows}


def segments_workload(dev, stream, seed=0, tune_it=True, hi=1_000_000):
    """50,000 segments, lengths log-uniform in [16, hi] (hi = 10^6: about
    4.5e9 int32 keys; hi = 19,023: about 2^27, the total the batched
    configuration states), keys uniform in [0, 2^31) drawn on the device from
    a seeded generator, one sort_segmented call on each path that applies:
    the work queue (one persistent launch for every phase; segments
    averaging more than 1,024 keys), the segment passes (a launch per phase;
    more than 8,192) and the persistent kernel with one workgroup per
    segment."""
    import torch

    from paper_1105_6040_amd import _native as N
    from paper_1105_6040_amd import api, inputs, tune

    log(f"segments: 50,000 log-uniform [16, {hi}]")
    lengths = inputs.segment_lengths(seed, hi=hi)
    off = inputs.offsets_from_lengths(lengths)
    n = int(off[-1])
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    k = torch.randint(0, 2**31, (n,), dtype=torch.int32, device=dev, generator=g)
    toff = torch.from_numpy(off).to(dev)
    out = torch.empty_like(k)
    saved = N.tune_get(N.MS_TUNE_SEG_PASSES)
    N.tune_set(N.MS_TUNE_SEG_PASSES, 2)  # sized for every path
    ws = torch.empty(N.workspace_size(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, n, lengths.size),
                     dtype=torch.uint8, device=dev)
    N.tune_set(N.MS_TUNE_SEG_PASSES, saved)
    run = lambda: api.sort_segmented(k, toff, keys_out=out, ws=ws)  # noqa: E731
    paths = {}
    nseg = int(lengths.size)
    modes = [(m, name) for m, name in ((2, "work_queue_one_launch"), (1, "segment_passes"))
             if tune.uses_segment_passes(n, nseg, m)] + [(0, "persistent_one_wg_per_segment")]
    for mode, name in modes:
        N.tune_set(N.MS_TUNE_SEG_PASSES, mode)
        _, per = time_steps(run, 3, 1, stream)
        N.timing_reset()
        N.timing_enable(True)
        time_steps(run, 1, 0, stream)
        N.timing_enable(False)
        kt = N.timing_read()
        N.timing_reset()
        ms = median(per)
        paths[name] = {"ms_median": round(ms, 3), "GKeys_per_s": round(n / (ms * 1e-3) / 1e9, 3),
                       "launches_per_call": sum(c for c, _ in kt.values()),
                       "kernel_ms": {kk: round(v[1], 3) for kk, v in kt.items()}}
        log(name, paths[name]["ms_median"])
    N.tune_set(N.MS_TUNE_SEG_PASSES, saved)
    res = {"segments": int(lengths.size), "keys": n, "paths": paths}
    if tune_it:
        tuned = tune.Tuner(cache_path=None, reps=1).tune_segmented(k, toff)
        res["tuned"] = {"params": tuned["params"], "trials_ms": tuned["trials"]}
        _, per = time_steps(run, 3, 1, stream)
    else:
        _, per = time_steps(run, 3, 1, stream)
    ms = median(per)
    res.update({"ms_median": round(ms, 3), "path": {0: "persistent", 1: "segment passes", 2: "work queue"}[
        N.tune_get(N.MS_TUNE_SEG_PASSES)], "GKeys_per_s": round(n / (ms * 1e-3) / 1e9, 3),
        "GBps_at_36B_per_key": round(n * 36 / (ms * 1e-3) / 1e9, 1)})
    if "work_queue_one_launch" in paths:
        q = paths["work_queue_one_launch"]["ms_median"]
        res["work_queue_GBps_at_36B_per_key"] = round(n * 36 / (q * 1e-3) / 1e9, 1)
    del k, out, ws, toff
    torch.cuda.empty_cache()
    return res


def serving_workload(dev, nreq=2000, warm=200, seed=0, tune_it=True):
    """Serving stream: requests of (uint32 key, uint32 value) pairs, lengths
    log-uniform in [1e3, 1e7], keys uniform, payloads staged on the device
    before the clock.  Each server's closed-loop capacity is measured with
    every request arriving at once; both then run the same Poisson trace at
    0.8 x the one-launch-per-request server's capacity (warm + nreq requests,
    the first `warm` excluded from the figures).  The continuous-batching
    server's parameters (steps queued ahead; the length above which a request
    takes a launch of its own beside the steps, and how many such launches run
    at once) are tuned on a Poisson trace of another seed at the same rate
    (without tuning: 2 steps ahead, requests above 10^6 pairs on launches of
    their own, 2 of those at once)."""
    import numpy as np
    import torch

    from paper_1105_6040_amd import inputs, serve, tune

    total_req = warm + nreq
    log(f"serving: {warm} + {nreq} requests")
    _, lengths = inputs.serving_trace(seed=seed, nreq=total_req, rate_per_s=1.0)
    total = int(sum(int(x) for x in lengths))
    g = torch.Generator(device=dev)
    g.manual_seed(seed + 5)
    keys = torch.randint(-2**31, 2**31, (total,), dtype=torch.int32, device=dev, generator=g).view(torch.uint32)
    vals = torch.arange(total, dtype=torch.int32, device=dev).view(torch.uint32)
    ok, ov = torch.empty_like(keys), torch.empty_like(vals)
    free, _ = torch.cuda.mem_get_info(dev)
    budget = max(1 << 30, free - (16 << 30))

    def run(kind, arrivals, params=(2, None, 2), lens=lengths):
        reqs = serve.make_requests(arrivals, lens)
        if kind == "step":
            steps_inflight, above, dinf = params
            ex = serve.GpuStepExecutor(keys, vals, ok, ov)
            dx = serve.GpuExecutor(keys, vals, ok, ov, streams=2) if above is not None else None
            srv = serve.StepServer(ex, budget_bytes=budget, max_steps_inflight=steps_inflight, direct=dx,
                                   direct_above=above, direct_inflight=dinf)
        else:
            ex = serve.GpuExecutor(keys, vals, ok, ov, streams=2)
            srv = serve.Server(ex, budget_bytes=budget, max_inflight=4, streams=2)
        st = srv.run(reqs)
        torch.cuda.synchronize()
        return st, reqs

    def summary(st, reqs):
        m = [r for r in reqs if r.rid >= warm]
        lat = [r.latency * 1e3 for r in m]
        wall = max(r.done for r in m) - min(r.arrival for r in m)
        pairs = sum(r.n for r in m)
        return {"requests": len(m), "p50_ms": round(percentile(lat, 50), 4), "p99_ms": round(percentile(lat, 99), 4),
                "GKeys_per_s": round(pairs / wall / 1e9, 3), "req_per_s": round(len(m) / wall, 1),
                "launches": st.launches, "max_active": st.max_active, "max_inflight": st.max_inflight_seen,
                "budget_waits": st.budget_waits, "max_reserved_bytes": st.max_reserved_bytes}

    at_once = [0.0] * total_req
    run("single", at_once)  # warm-up of both paths
    run("step", at_once, (2, 100_000, 2))
    cap = {"one_launch_per_request": summary(*run("single", at_once))}
    rate = 0.8 * cap["one_launch_per_request"]["req_per_s"]

    def poisson(s):
        g2 = inputs.rng("serving", s)
        gaps = g2.exponential(1.0 / rate, total_req)
        return list(gaps.cumsum() - gaps[0])

    # Tune on a trace of another seed (its own lengths too) at the same rate.
    _, tl = inputs.serving_trace(seed=seed + 1, nreq=total_req, rate_per_s=1.0)
    tl = np.minimum(tl, lengths)  # fits the staged pool request by request
    tune_arrivals = poisson(seed + 101)
    if tune_it:
        tuned = tune.Tuner(cache_path=None).tune_serving(lambda c: run("step", tune_arrivals, c, tl)[0])
    else:
        tuned = {"params": [2, 1_000_000, 2], "trials": []}
    best = tuple(tuned["params"])
    cap["continuous_batching"] = summary(*run("step", at_once, best))
    cap["continuous_batching_steps_only"] = summary(*run("step", at_once, (best[0], None, 2)))
    arrivals = poisson(seed + 1)
    per_req = summary(*run("single", arrivals))
    batched = summary(*run("step", arrivals, best))
    steps_only = summary(*run("step", arrivals, (best[0], None, 2)))
    return {"requests_measured": nreq, "warmup_requests": warm, "pairs_staged": total,
            "closed_loop_capacity": cap, "rate_req_per_s": round(rate, 1),
            "continuous_batching_params": {"steps_inflight": best[0], "direct_above_pairs": best[1],
                                           "direct_inflight": best[2]},
            "tuning_trials_params_p99_p50_ms": tuned["trials"],
            "one_launch_per_request": per_req, "continuous_batching": batched,
            "continuous_batching_steps_only": steps_only}


if __name__ == "__main__":
    main()
