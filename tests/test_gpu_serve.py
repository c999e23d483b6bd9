"""Serving on the GPU: every request's result is the same alone and in the
mix (tolerance 0: integer work), and matches the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1105_6040_amd import api, inputs, serve

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def staged(nreq=160, lo=1000, hi=300_000, rate=4000.0, seed=7):
    arr, lengths = inputs.serving_trace(seed=seed, nreq=nreq, lo=lo, hi=hi, rate_per_s=rate)
    reqs = serve.make_requests(arr, lengths)
    total = sum(r.n for r in reqs)
    g = np.random.default_rng(seed)
    keys = g.integers(0, 2**32, total, dtype=np.uint32)
    keys[: total // 3] &= np.uint32(0xFFF)  # many ties in the first third of the pool
    vals = np.arange(total, dtype=np.uint32)
    return reqs, keys, vals


@pytest.mark.parametrize("batching", [True, False])
def test_serving_results_alone_and_in_the_mix(batching):
    reqs, keys, vals = staged()
    dev = torch.device("cuda:0")
    tk, tv = torch.from_numpy(keys).to(dev), torch.from_numpy(vals).to(dev)
    ok, ov = torch.zeros_like(tk), torch.zeros_like(tv)
    ex = serve.GpuExecutor(tk, tv, ok, ov, streams=2)
    say(f"serving {len(reqs)} requests, batching={batching}")
    stats = serve.Server(ex, budget_bytes=1 << 32, batching=batching, large_threshold=1 << 16,
                         max_batch_pairs=1 << 22, max_inflight=4, streams=2).run(reqs)
    torch.cuda.synchronize()
    assert len(stats.latencies_ms) == len(reqs)
    if batching:
        assert stats.launches < len(reqs)
    out_k, out_v = ok.cpu().numpy(), ov.cpu().numpy()
    say("comparing every request with its own sort_pairs call")
    for r in reqs:
        a, b = r.offset, r.offset + r.n
        ak, av = api.sort_pairs(tk[a:b], tv[a:b])
        torch.cuda.synchronize()
        ak, av = ak.cpu().numpy(), av.cpu().numpy()
        if not (np.array_equal(out_k[a:b], ak) and np.array_equal(out_v[a:b], av)):
            ek, ev = oracle.sort(keys[a:b], vals[a:b])
            bad = np.nonzero((out_k[a:b] != ek) | (out_v[a:b] != ev))[0]
            say(f"request {r.rid} n={r.n} path={r.path}: served==oracle {bad.size == 0}, "
                f"alone==oracle {np.array_equal(ak, ek) and np.array_equal(av, ev)}, "
                f"served mismatches {bad.size} first {bad[:8].tolist()} "
                f"served keys sorted {bool(np.all(out_k[a:b][1:] >= out_k[a:b][:-1]))}")
            if bad.size:
                i = int(bad[0])
                say(f"  at {i}: served {out_k[a+i]}/{out_v[a+i]} oracle {ek[i]}/{ev[i]}")
        assert np.array_equal(out_k[a:b], ak), r.rid
        assert np.array_equal(out_v[a:b], av), r.rid
    for r in reqs[::16]:
        a, b = r.offset, r.offset + r.n
        ek, ev = oracle.sort(keys[a:b], vals[a:b])
        assert np.array_equal(out_k[a:b], ek) and np.array_equal(out_v[a:b], ev), r.rid
