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
