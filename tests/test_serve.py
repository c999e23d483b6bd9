"""Serving loop logic on the CPU with fake executors (no GPU)."""
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


def _trace(nreq=150, lo=10, hi=60000, rate=20000.0, seed=3):
    arr, lengths = inputs.serving_trace(seed=seed, nreq=nreq, lo=lo, hi=hi, rate_per_s=rate)
    reqs = serve.make_requests(arr, lengths)
    total = sum(r.n for r in reqs)
    g = np.random.default_rng(seed)
    keys = g.integers(0, 2**32, total, dtype=np.uint32)
    vals = np.arange(total, dtype=np.uint32)
    return reqs, keys, vals


def _oracle_sort(k, v):
    return oracle.sort(k, v)


def _check_results(reqs, ex, keys, vals):
    for r in reqs:
        a, b = r.offset, r.offset + r.n
        ek, ev = oracle.sort(keys[a:b], vals[a:b])
        assert np.array_equal(ex.out_k[a:b], ek) and np.array_equal(ex.out_v[a:b], ev), r.rid
        assert r.done >= r.launched >= r.arrival


def test_step_server_sorts_every_request():
    reqs, keys, vals = _trace()
    ex = serve.FakeStepExecutor(keys, vals, _oracle_sort, small=5000)
    stats = serve.StepServer(ex, budget_bytes=1 << 30).run(reqs)
    assert len(stats.latencies_ms) == len(reqs)
    _check_results(reqs, ex, keys, vals)
    assert all(r.path == "step" for r in reqs)
    assert stats.launches < 5 * len(reqs)


def test_step_server_runs_every_phase_once_in_order():
    """Each request appears in consecutive steps, phase 0, 1, ... its last,
    once each: requests join at a pass boundary and leave after their last."""
    reqs, keys, vals = _trace(nreq=60, rate=5e4)
    ex = serve.FakeStepExecutor(keys, vals, _oracle_sort, small=5000)
    serve.StepServer(ex, budget_bytes=1 << 30, max_steps_inflight=3).run(reqs)
    seen = {}
    for k, step in enumerate(ex.phase_log):
        for rid, ph in step:
            seen.setdefault(rid, []).append((k, ph))
    for r in reqs:
        steps = seen[r.rid]
        assert [ph for _, ph in steps] == list(range(r.phases)), r.rid
        assert [k for k, _ in steps] == list(range(steps[0][0], steps[0][0] + r.phases)), r.rid
    # the batch really mixes phases
    assert any(len({ph for _, ph in step}) > 1 for step in ex.phase_log)


def test_step_server_admits_by_the_hbm_budget():
    reqs, keys, vals = _trace(nreq=120, rate=1e6)  # everything arrives at once
    ex = serve.FakeStepExecutor(keys, vals, _oracle_sort, seconds_per_pair=2e-8, small=5000)
    budget = 3 * 8 * 60000
    stats = serve.StepServer(ex, budget_bytes=budget).run(reqs)
    biggest = max(ex.plan(r.n)[1] for r in reqs)
    assert stats.max_reserved_bytes <= max(budget, biggest)
    assert stats.budget_waits > 0
    _check_results(reqs, ex, keys, vals)


def test_step_server_slot_limit():
    reqs, keys, vals = _trace(nreq=100, rate=1e6)
    ex = serve.FakeStepExecutor(keys, vals, _oracle_sort, small=5000)
    stats = serve.StepServer(ex, budget_bytes=1 << 40, max_active=7).run(reqs)
    assert stats.max_active <= 7
    assert max(len(s) for s in ex.phase_log) <= 7
    _check_results(reqs, ex, keys, vals)


def test_one_launch_per_request_server():
    reqs, keys, vals = _trace()
    ex = serve.FakeExecutor(keys, vals, _oracle_sort)
    stats = serve.Server(ex, budget_bytes=1 << 30).run(reqs)
    assert stats.launches == len(reqs)
    _check_results(reqs, ex, keys, vals)
    launched = [r.launched for r in sorted(reqs, key=lambda r: r.arrival)]
    assert all(a <= b for a, b in zip(launched, launched[1:]))


def test_one_launch_server_respects_the_budget():
    reqs, keys, vals = _trace(nreq=120, rate=1e6)
    ex = serve.FakeExecutor(keys, vals, _oracle_sort, seconds_per_pair=2e-8)
    budget = 20000 * ex.ws_per_pair
    stats = serve.Server(ex, budget_bytes=budget, max_inflight=8).run(reqs)
    biggest = max(ex.workspace_bytes(r.n) for r in reqs)
    assert stats.max_reserved_bytes <= max(budget, biggest)
    assert stats.budget_waits > 0


def test_step_server_gives_long_requests_a_launch_of_their_own():
    """Requests above the threshold run as one launch each beside the steps;
    the rest are batched; every result is the oracle's."""
    reqs, keys, vals = _trace(nreq=150, rate=5e4)
    ex = serve.FakeStepExecutor(keys, vals, _oracle_sort, small=5000)
    dx = serve.FakeExecutor(keys, vals, _oracle_sort)
    dx.out_k, dx.out_v = ex.out_k, ex.out_v  # one output pool for both paths
    stats = serve.StepServer(ex, budget_bytes=1 << 30, direct=dx, direct_above=20000).run(reqs)
    _check_results(reqs, ex, keys, vals)
    for r in reqs:
        assert r.path == ("single" if r.n > 20000 else "step"), (r.rid, r.n, r.path)
    long_ids = {r.rid for r in reqs if r.n > 20000}
    assert long_ids and len(long_ids) < len(reqs)
    assert all(rid not in long_ids for step in ex.phase_log for rid, _ in step)
    assert stats.launches == len(ex.phase_log) + len(long_ids)


def test_step_server_with_direct_launches_respects_the_budget():
    reqs, keys, vals = _trace(nreq=120, rate=1e6)  # everything arrives at once
    ex = serve.FakeStepExecutor(keys, vals, _oracle_sort, seconds_per_pair=2e-8, small=5000)
    dx = serve.FakeExecutor(keys, vals, _oracle_sort, seconds_per_pair=2e-8)
    dx.out_k, dx.out_v = ex.out_k, ex.out_v
    budget = 3 * 8 * 60000
    stats = serve.StepServer(ex, budget_bytes=budget, direct=dx, direct_above=30000, direct_inflight=3).run(reqs)
    biggest = max(max(ex.plan(r.n)[1], dx.workspace_bytes(r.n)) for r in reqs)
    assert stats.max_reserved_bytes <= max(budget, biggest)
    assert stats.budget_waits > 0
    _check_results(reqs, ex, keys, vals)


def test_markers_cover_every_request_and_step(monkeypatch):
    """With markers on, every request and every step opens one roctx range
    and closes it once; results are unchanged."""
    from paper_1105_6040_amd import markers
    opened, closed = {}, []
    counter = iter(range(1, 1 << 30))

    def start(msg):
        i = next(counter)
        opened[i] = msg
        return i

    monkeypatch.setattr(markers, "start", start)
    monkeypatch.setattr(markers, "stop", lambda i: closed.append(i))
    reqs, keys, vals = _trace(nreq=80, rate=5e4)
    ex = serve.FakeStepExecutor(keys, vals, _oracle_sort, small=5000)
    dx = serve.FakeExecutor(keys, vals, _oracle_sort)
    dx.out_k, dx.out_v = ex.out_k, ex.out_v
    stats = serve.StepServer(ex, budget_bytes=1 << 30, direct=dx, direct_above=20000).run(reqs)
    _check_results(reqs, ex, keys, vals)
    assert sorted(closed) == sorted(opened)
    names = list(opened.values())
    assert sum(m.startswith("request ") for m in names) == len(reqs)
    assert sum(m.startswith("step ") for m in names) == len(ex.phase_log)
    assert sum(m.endswith(" single") for m in names) == sum(r.path == "single" for r in reqs)
    assert stats.launches == len(ex.phase_log) + sum(r.path == "single" for r in reqs)


def test_markers_call_the_roctx_library():
    from paper_1105_6040_amd import markers
    was = markers._enabled
    markers.enable(True)
    try:
        if not markers.enabled():
            pytest.skip("no roctx library on this machine")
        rid = markers.start("test range")
        markers.mark("test mark")
        markers.stop(rid)
    finally:
        markers.enable(was)
