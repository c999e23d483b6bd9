"""Autotuner logic that needs no GPU: size classes and the cached search."""
import json

from paper_1105_6040_amd import tune


def test_size_class():
    assert tune.size_class(1) == 0
    assert tune.size_class(2) == 1
    assert tune.size_class(2**28) == 28
    assert tune.size_class(2**28 + 5) == 28
    assert tune.size_class(2**28 - 1) == 27


def test_search_picks_fastest_and_caches(tmp_path, monkeypatch):
    path = str(tmp_path / "tune.json")
    t = tune.Tuner(cache_path=path, reps=1)
    applied = []
    fake_times = {(1,): 3.0, (2,): 1.0, (3,): 2.0}
    state = {}
    monkeypatch.setattr(t, "_time", lambda fn: fake_times[state["p"]])

    def apply(p):
        state["p"] = p
        applied.append(p)

    rec = t._search("k", [(1,), (2,), (3,)], apply, lambda: None, force=False)
    assert rec["params"] == [2] and applied[-1] == (2,)
    assert json.load(open(path))["k"]["params"] == [2]
    applied.clear()
    t2 = tune.Tuner(cache_path=path, reps=1)
    rec2 = t2._search("k", [(1,), (2,), (3,)], apply, lambda: 1 / 0, force=False)  # cached: no timing
    assert rec2["params"] == [2] and applied == [(2,)]


def test_serving_candidates_cover_every_combination_once():
    c = tune.serving_candidates()
    assert len(c) == len(set(c))
    for si in tune.SERVE_STEPS_INFLIGHT:
        assert (si, None, tune.SERVE_DIRECT_INFLIGHT[0]) in c
        for above in tune.SERVE_DIRECT_ABOVE:
            if above is not None:
                for dinf in tune.SERVE_DIRECT_INFLIGHT:
                    assert (si, above, dinf) in c
    assert sum(1 for x in c if x[1] is None) == len(tune.SERVE_STEPS_INFLIGHT)


def test_tune_serving_picks_lowest_p99_then_p50_and_caches(tmp_path, monkeypatch):
    class St:
        def __init__(self, p99, p50):
            self.p99_ms, self.p50_ms = p99, p50

    def fake(params):
        si, above, dinf = params
        seen.append(params)
        p99 = 1.0 if above is None else 0.5 + abs(above - 100_000) / 1e6  # best at 100k
        return St(p99, 0.3 - 0.01 * dinf + 0.001 * si)

    seen = []
    path = str(tmp_path / "tune.json")
    t = tune.Tuner(cache_path=path)
    monkeypatch.setattr(t, "_device", lambda: "fake")
    rec = t.tune_serving(fake)
    assert rec["params"] == [1, 100_000, 4]
    assert len(seen) == len(tune.serving_candidates())
    seen.clear()
    t2 = tune.Tuner(cache_path=path)
    monkeypatch.setattr(t2, "_device", lambda: "fake")
    assert t2.tune_serving(fake)["params"] == [1, 100_000, 4] and not seen  # cached
