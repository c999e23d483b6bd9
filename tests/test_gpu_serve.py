"""Serving on the GPU.  The step engine (sort_step, continuous batching)
through the C ABI, and both servers over a request stream: every request's
result equals the oracle's stable sort of it, and is the same alone (one
sort_pairs call) and in the mix (tolerance 0: integer work), with and without
an HBM budget that makes admission wait."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1105_6040_amd import _native as N
from paper_1105_6040_amd import api, inputs, serve

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _key_np(kt):
    return {N.MS_KEY_I32: np.int32, N.MS_KEY_U32: np.uint32, N.MS_KEY_U64: np.uint64}[kt]


@pytest.mark.parametrize("kt,pairs", [(N.MS_KEY_U32, True), (N.MS_KEY_I32, False), (N.MS_KEY_U64, True),
                                      (N.MS_KEY_U32, False)])
def test_sort_step_mixed_phases(kt, pairs):
    """Requests of one-tile and multi-tile lengths join the step loop at
    different steps, so most steps mix phases (histogram, digit passes,
    whole one-tile sorts); each result against the oracle."""
    g = np.random.default_rng(11 + kt)
    lengths = [20000, 5, 8192, 8193, 1, 300001, 700, 16384, 4096, 4097, 65536 * 3 + 17, 0, 1 << 20]
    arrive = [0, 0, 1, 1, 2, 2, 5, 7, 3, 3, 4, 4, 6]
    dt = _key_np(kt)
    info = np.iinfo(dt)
    kin = [g.integers(info.min, info.max, n, dtype=dt, endpoint=True) for n in lengths]
    kin[7] &= dt(0xFFF)  # many ties
    vin = [g.integers(0, 2**32, n, dtype=np.uint32) for n in lengths]
    dk = [torch.from_numpy(k).cuda() for k in kin]
    dv = [torch.from_numpy(v).cuda() for v in vin]
    ok = [torch.empty_like(k) for k in dk]
    ov = [torch.empty_like(v) for v in dv]
    plans = [N.step_plan(kt, pairs, n) for n in lengths]
    work = [torch.full((max(1, wb),), 0x5A, dtype=torch.uint8, device="cuda") for _, wb in plans]  # garbage
    ws = torch.empty(N.workspace_size(N.MS_OP_SORT_STEP, kt, pairs, 0, N.MS_STEP_MAX_REQUESTS), dtype=torch.uint8,
                     device="cuda")
    phase = [0] * len(lengths)
    rec_t = N.STEP_REQUEST_DTYPE
    steps = 0
    for step in range(100):
        idx = [i for i in range(len(lengths)) if arrive[i] <= step and phase[i] < plans[i][0]]
        if not idx:
            if all(phase[i] >= plans[i][0] for i in range(len(lengths))):
                break
            continue
        tab = np.zeros(len(idx), dtype=rec_t)
        for row, i in enumerate(idx):
            tab[row] = (dk[i].data_ptr(), dv[i].data_ptr() if pairs else 0, ok[i].data_ptr(),
                        ov[i].data_ptr() if pairs else 0, work[i].data_ptr() if plans[i][1] else 0, lengths[i],
                        phase[i], 0)
            phase[i] += 1
        dtab = torch.from_numpy(tab.view(np.uint8)).cuda()
        N.check(N.lib().sort_step(dtab.data_ptr(), len(idx), kt, int(pairs), ws.data_ptr(), ws.numel(),
                                  torch.cuda.current_stream().cuda_stream), "sort_step")
        steps += 1
        torch.cuda.synchronize()
    say(f"sort_step kt={kt} pairs={pairs}: {steps} steps")
    for i, n in enumerate(lengths):
        if pairs:
            ek, ev = oracle.sort(kin[i], vin[i])
            assert np.array_equal(ok[i].cpu().numpy(), ek), (i, n)
            assert np.array_equal(ov[i].cpu().numpy(), ev), (i, n)
        elif n:
            assert np.array_equal(ok[i].cpu().numpy(), oracle.sort(kin[i])), (i, n)


def staged(nreq=160, lo=1000, hi=300_000, rate=4000.0, seed=7):
    arr, lengths = inputs.serving_trace(seed=seed, nreq=nreq, lo=lo, hi=hi, rate_per_s=rate)
    reqs = serve.make_requests(arr, lengths)
    total = sum(r.n for r in reqs)
    g = np.random.default_rng(seed)
    keys = g.integers(0, 2**32, total, dtype=np.uint32)
    keys[: total // 3] &= np.uint32(0xFFF)  # many ties in the first third of the pool
    vals = np.arange(total, dtype=np.uint32)
    return reqs, keys, vals


def _check_every_request(reqs, keys, vals, tk, tv, out_k, out_v, alone=True):
    for r in reqs:
        a, b = r.offset, r.offset + r.n
        ek, ev = oracle.sort(keys[a:b], vals[a:b])
        assert np.array_equal(out_k[a:b], ek) and np.array_equal(out_v[a:b], ev), (r.rid, r.n, r.path)
        if alone:
            ak, av = api.sort_pairs(tk[a:b], tv[a:b])
            torch.cuda.synchronize()
            assert np.array_equal(ak.cpu().numpy(), ek) and np.array_equal(av.cpu().numpy(), ev), r.rid


@pytest.mark.parametrize("server", ["step", "step_direct", "one_launch"])
def test_serving_results_alone_and_in_the_mix(server):
    reqs, keys, vals = staged()
    dev = torch.device("cuda:0")
    tk, tv = torch.from_numpy(keys).to(dev), torch.from_numpy(vals).to(dev)
    ok, ov = torch.zeros_like(tk), torch.zeros_like(tv)
    say(f"serving {len(reqs)} requests, server={server}")
    if server == "step":
        ex = serve.GpuStepExecutor(tk, tv, ok, ov)
        stats = serve.StepServer(ex, budget_bytes=1 << 34).run(reqs)
        assert stats.launches < 5 * len(reqs)
        assert stats.max_active > 1
    elif server == "step_direct":
        # Long requests as launches of their own beside the steps of the rest.
        ex = serve.GpuStepExecutor(tk, tv, ok, ov)
        dx = serve.GpuExecutor(tk, tv, ok, ov, streams=2)
        stats = serve.StepServer(ex, budget_bytes=1 << 34, direct=dx, direct_above=30_000, direct_inflight=4).run(reqs)
        paths = {r.path for r in reqs}
        assert paths == {"step", "single"}, paths
        assert all((r.path == "single") == (r.n > 30_000) for r in reqs)
        assert stats.max_active > 1
    else:
        ex = serve.GpuExecutor(tk, tv, ok, ov, streams=2)
        stats = serve.Server(ex, budget_bytes=1 << 34).run(reqs)
        assert stats.launches == len(reqs)
    torch.cuda.synchronize()
    assert len(stats.latencies_ms) == len(reqs)
    say("comparing every request with the oracle and with its own sort_pairs call")
    _check_every_request(reqs, keys, vals, tk, tv, ok.cpu().numpy(), ov.cpu().numpy())


@pytest.mark.parametrize("server", ["step", "step_direct", "one_launch"])
def test_serving_under_an_hbm_cap(server):
    """Everything arrives at once and the budget holds about three requests'
    state: admission waits for memory, results are unchanged."""
    reqs, keys, vals = staged(nreq=120, rate=1e7, seed=8)
    dev = torch.device("cuda:0")
    tk, tv = torch.from_numpy(keys).to(dev), torch.from_numpy(vals).to(dev)
    ok, ov = torch.zeros_like(tk), torch.zeros_like(tv)
    big = max(r.n for r in reqs)
    if server == "step":
        budget = 3 * N.step_plan(N.MS_KEY_U32, True, big)[1]
        ex = serve.GpuStepExecutor(tk, tv, ok, ov)
        stats = serve.StepServer(ex, budget_bytes=budget).run(reqs)
    elif server == "step_direct":
        budget = 3 * max(N.step_plan(N.MS_KEY_U32, True, big)[1],
                         N.workspace_size(N.MS_OP_SORT_PAIRS, N.MS_KEY_U32, True, big))
        ex = serve.GpuStepExecutor(tk, tv, ok, ov)
        dx = serve.GpuExecutor(tk, tv, ok, ov, streams=2)
        stats = serve.StepServer(ex, budget_bytes=budget, direct=dx, direct_above=30_000,
                                 direct_inflight=4).run(reqs)
    else:
        budget = 3 * N.workspace_size(N.MS_OP_SORT_PAIRS, N.MS_KEY_U32, True, big)
        ex = serve.GpuExecutor(tk, tv, ok, ov, streams=2)
        stats = serve.Server(ex, budget_bytes=budget, max_inflight=8).run(reqs)
    torch.cuda.synchronize()
    say(f"{server}: budget {budget} B, {stats.budget_waits} waits, peak reserved {stats.max_reserved_bytes} B")
    assert stats.budget_waits > 0
    assert stats.max_reserved_bytes <= budget
    _check_every_request(reqs, keys, vals, tk, tv, ok.cpu().numpy(), ov.cpu().numpy(), alone=False)


def test_hbm_probe_kernels():
    """The bandwidth probe's copy and write kernels move the bytes they claim."""
    n = (1 << 24) + 4
    src = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    s = torch.cuda.current_stream().cuda_stream
    N.check(N.lib().ms_hbm_probe(2, src.data_ptr(), dst.data_ptr(), n * 4, s), "copy")
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    N.check(N.lib().ms_hbm_probe(5, dst.data_ptr(), src.data_ptr(), n * 4, s), "copy nt")
    N.check(N.lib().ms_hbm_probe(4, None, dst.data_ptr(), n * 4, s), "write nt")
    sink = torch.zeros(4096, dtype=torch.int32, device="cuda")
    N.check(N.lib().ms_hbm_probe(0, src.data_ptr(), sink.data_ptr(), n * 4, s), "read")
    torch.cuda.synchronize()
    w = dst.view(torch.int32).cpu().numpy().view(np.uint32)
    assert np.array_equal(w.reshape(-1, 4)[:, 0], np.full(n // 4, 0x9e3779b9, np.uint32))
    assert N.lib().ms_hbm_probe(0, src.data_ptr(), sink.data_ptr(), 17, s) == N.MS_EINVAL
