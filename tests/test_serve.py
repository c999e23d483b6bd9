"""Serving loop logic on the CPU with a fake executor (no GPU)."""
import numpy as np
import pytest

import oracle
from paper_1105_6040_amd import inputs, serve


def test_percentile_nearest_rank():
    xs = list(range(1, 101))
    assert serve.percentile(xs, 50) == 50
    assert serve.percentile(xs, 99) == 99
    assert serve.percentile(xs, 100) == 100
    assert serve.percentile([7.0], 99) == 7.0
    assert serve.percentile([3, 1, 2], 50) == 2


def _trace(nreq=150, lo=10, hi=6000, rate=20000.0, seed=3):
    arr, lengths = inputs.serving_trace(seed=seed, nreq=nreq, lo=lo, hi=hi, rate_per_s=rate)
    reqs = serve.make_requests(arr, lengths)
    total = sum(r.n for r in reqs)
    g = np.random.default_rng(seed)
    keys = g.integers(0, 2**32, total, dtype=np.uint32)
    vals = np.arange(total, dtype=np.uint32)
    return reqs, keys, vals


def _oracle_sort(k, v):
    return oracle.sort(k, v)


@pytest.mark.parametrize("batching", [True, False])
def test_every_request_sorted_alone_and_in_the_mix(batching):
    reqs, keys, vals = _trace()
    ex = serve.FakeExecutor(keys, vals, _oracle_sort)
    stats = serve.Server(ex, budget_bytes=1 << 30, batching=batching, large_threshold=3000,
                         max_batch_pairs=20000).run(reqs)
    assert len(stats.latencies_ms) == len(reqs)
    for r in reqs:
        a, b = r.offset, r.offset + r.n
        ek, ev = oracle.sort(keys[a:b], vals[a:b])
        assert np.array_equal(ex.out_k[a:b], ek) and np.array_equal(ex.out_v[a:b], ev)
        assert r.done >= r.launched >= r.arrival
    if batching:
        assert stats.launches < len(reqs)
        assert any(r.path == "batch" for r in reqs)
        assert all(r.path == "single" for r in reqs if r.n > 3000)
    else:
        assert stats.launches == len(reqs)


def test_fifo_launch_order():
    reqs, keys, vals = _trace(nreq=80)
    ex = serve.FakeExecutor(keys, vals, _oracle_sort)
    serve.Server(ex, budget_bytes=1 << 30, batching=True, large_threshold=3000).run(reqs)
    launched = [r.launched for r in sorted(reqs, key=lambda r: r.arrival)]
    assert all(a <= b for a, b in zip(launched, launched[1:]))


def test_admission_respects_the_hbm_budget():
    reqs, keys, vals = _trace(nreq=120, rate=1e6)  # everything arrives at once
    ex = serve.FakeExecutor(keys, vals, _oracle_sort, seconds_per_pair=2e-8)
    budget = 20000 * ex.ws_per_pair  # room for two or three launches at a time
    stats = serve.Server(ex, budget_bytes=budget, batching=True, large_threshold=3000, max_batch_pairs=8000,
                         max_inflight=8).run(reqs)
    biggest_unit = max(ex.workspace_bytes(r.n, 1) for r in reqs)
    assert stats.max_reserved_bytes <= max(budget, biggest_unit)
    assert stats.budget_waits > 0


def test_consecutive_only_batches():
    reqs = serve.make_requests([0.0] * 6, [10, 10, 5000, 10, 10, 10])
    srv = serve.Server(serve.FakeExecutor(np.zeros(5050, np.uint32), np.zeros(5050, np.uint32), _oracle_sort),
                       budget_bytes=1 << 30, large_threshold=1000)
    import collections
    q = collections.deque(reqs)
    assert [r.rid for r in srv._next_unit(q)] == [0, 1]
    q.popleft(); q.popleft()
    assert [r.rid for r in srv._next_unit(q)] == [2]
    q.popleft()
    assert [r.rid for r in srv._next_unit(q)] == [3, 4, 5]
