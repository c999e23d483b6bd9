"""The full-size comparison helper (tests/fullsize.py) on the CPU: it accepts
the oracle's own segmented result, walks every segment once whatever the
chunking, and rejects a result with one key moved or one value swapped."""
import numpy as np
import pytest
import torch

import oracle
from paper_1105_6040_amd import inputs
from tests import fullsize


def _case(seed, dt=np.int32):
    g = np.random.default_rng(seed)
    lengths = np.concatenate([g.integers(0, 50, 300), [0, 0, 5000, 1, 20000], g.integers(0, 3000, 40)])
    g.shuffle(lengths)
    off = inputs.offsets_from_lengths(lengths)
    k = g.integers(0, 1000, int(off[-1])).astype(dt)
    v = np.arange(k.size, dtype=np.uint32)
    return off, k, v


@pytest.mark.parametrize("chunk", [1, 777, 1 << 12, 1 << 20])
def test_accepts_the_oracle_result(chunk):
    off, k, v = _case(1)
    ek, ev = oracle.sort_segmented(k, off, v)
    t = torch.from_numpy
    n = fullsize.compare_segments(t(k), t(ek), off, t(v), t(ev), chunk_keys=chunk, big_segment=10_000)
    assert n == off.size - 1


@pytest.mark.parametrize("chunk", [1000, 1 << 20])
def test_rejects_a_wrong_key_or_value(chunk):
    off, k, v = _case(2)
    ek, ev = oracle.sort_segmented(k, off, v)
    t = torch.from_numpy
    bad = ek.copy()
    i = int(off[200]) + 1 if off[201] - off[200] > 1 else int(off[-1]) - 1
    bad[i] += 1
    with pytest.raises(AssertionError):
        fullsize.compare_segments(t(k), t(bad), off, chunk_keys=chunk, big_segment=10_000)
    # two equal keys in one segment with their values swapped: keys still
    # right, order of ties wrong
    badv = ev.copy()
    for s in range(off.size - 1):
        a, b = int(off[s]), int(off[s + 1])
        eq = np.flatnonzero(ek[a:b - 1] == ek[a + 1:b])
        if eq.size:
            j = a + int(eq[0])
            badv[j], badv[j + 1] = badv[j + 1], badv[j]
            break
    with pytest.raises(AssertionError):
        fullsize.compare_segments(t(k), t(ek), off, t(v), t(badv), chunk_keys=chunk, big_segment=10_000)


def test_oracle_whole_is_the_oracle_sort():
    g = np.random.default_rng(5)
    k = g.integers(0, 50, 100_003).astype(np.uint32)
    v = np.arange(k.size, dtype=np.uint32)
    ek, ev = fullsize.oracle_whole(k, v, parts=7)
    rk, rv = oracle.sort(k, v)
    assert np.array_equal(ek, rk) and np.array_equal(ev, rv)
