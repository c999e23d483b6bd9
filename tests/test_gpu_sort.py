"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Integer work, so the bar is bit-exact equality with the oracle's stable sort
on the same seeded inputs.  Sizes straddle the tile sizes (4,096 keys per
onesweep tile for 32-bit keys, 2,048 for 64-bit; 8,192 / 4,096 keys in one
LDS tile) and leave ragged tails.  Full-size configurations are compared with
the oracle element by element as well, the oracle run on the host's cores
(tests/fullsize.py).
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1105_6040_amd import _native as N
from paper_1105_6040_amd import api, inputs
from tests import fullsize
from tests.oracle_pins import certify_stable_sort

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 63, 64, 65, 1000, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 10000, 65537,
         100003, (1 << 20) + 17]
DISTS = ["uniform", "pos31", "small", "sorted", "reverse", "equal", "extremes", "few", "bits16"]
DTYPES = ["i32", "u32", "u64"]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", SIZES)
def test_sort_keys_parity(dt, n):
    for dist in DISTS:
        say(f"sort_keys {dt} n={n} {dist}")
        k = inputs.keys(dt, n, dist, seed=n)
        out = host(api.sort_keys(dev(k)))
        assert np.array_equal(out, oracle.sort(k)), (dt, n, dist)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", SIZES)
def test_sort_pairs_parity(dt, n):
    for dist in ("uniform", "small", "equal", "few", "bits16", "reverse"):
        say(f"sort_pairs {dt} n={n} {dist}")
        k = inputs.keys(dt, n, dist, seed=n + 1)
        v = np.arange(n, dtype=np.uint32)
        ko, vo = api.sort_pairs(dev(k), dev(v))
        ek, ev = oracle.sort(k, v)
        assert np.array_equal(host(ko), ek), (dt, n, dist)
        assert np.array_equal(host(vo), ev), (dt, n, dist)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", [5, 4097, 8193, 100003])
def test_in_place(dt, n):
    for dist in ("uniform", "small", "equal"):
        say(f"in-place {dt} n={n} {dist}")
        k = inputs.keys(dt, n, dist, seed=7)
        t = dev(k)
        api.sort_keys(t, out=t)
        assert np.array_equal(host(t), oracle.sort(k)), (dt, n, dist)
        v = np.arange(n, dtype=np.uint32)
        tk, tv = dev(k), dev(v)
        api.sort_pairs(tk, tv, keys_out=tk, vals_out=tv)
        ek, ev = oracle.sort(k, v)
        assert np.array_equal(host(tk), ek) and np.array_equal(host(tv), ev), (dt, n, dist)


@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_every_tile_size(threads):
    from paper_1105_6040_amd import _native as N
    old = N.tune_get(N.MS_TUNE_PASS_THREADS)
    N.tune_set(N.MS_TUNE_PASS_THREADS, threads)
    try:
        for dt in DTYPES:
            for n in (9000, 16383, 16385, 18599, 40000, 300_001):
                for dist in ("uniform", "small", "bits16"):
                    say(f"tile threads={threads} {dt} n={n} {dist}")
                    k = inputs.keys(dt, n, dist, seed=n + threads)
                    v = np.arange(n, dtype=np.uint32)
                    assert np.array_equal(host(api.sort_keys(dev(k))), oracle.sort(k)), (threads, dt, n, dist)
                    ko, vo = api.sort_pairs(dev(k), dev(v))
                    ek, ev = oracle.sort(k, v)
                    assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), (threads, dt, n, dist)
    finally:
        N.tune_set(N.MS_TUNE_PASS_THREADS, old)


@pytest.mark.parametrize("dt", ["i32", "u32"])
def test_single_block_histogram(dt):
    """The whole digit-histogram read done by one workgroup (each of its
    counters then sees every key of its lane class).  Nearly all keys are
    equal, so one bin of every digit position takes almost every key; the
    view starts one key in, so the unaligned head and the tail are counted
    too.  Closed form: each distinct key, ascending, repeated by its count."""
    from paper_1105_6040_amd import _native as N
    old = N.tune_get(N.MS_TUNE_HIST_BLOCKS)
    N.tune_set(N.MS_TUNE_HIST_BLOCKS, 1)
    try:
        n = (1 << 24) + 3
        g = np.random.default_rng(11)
        ty = np.int32 if dt == "i32" else np.uint32
        k = np.full(n, 0x5A5A5A5A, dtype=ty)
        k[g.integers(0, n, 1000)] = g.integers(-(2**31) if dt == "i32" else 0, 2**31, 1000).astype(ty)
        say(f"single-block histogram {dt}: sorting")
        out = host(api.sort_keys(dev(k)[1:]))
        vals, counts = np.unique(k[1:], return_counts=True)
        assert np.array_equal(out, np.repeat(vals, counts)), dt
    finally:
        N.tune_set(N.MS_TUNE_HIST_BLOCKS, old)


def test_repeat_determinism_low_bits():
    """The same pairs sorted 25 times give the oracle's answer every time
    (12-bit keys: two constant digit bytes, many ties)."""
    g = np.random.default_rng(7)
    k = (g.integers(0, 2**32, 18599, dtype=np.uint32) & np.uint32(0xFFF)).astype(np.uint32)
    v = np.arange(k.size, dtype=np.uint32)
    ek, ev = oracle.sort(k, v)
    tk, tv = dev(k), dev(v)
    for rep in range(25):
        ko, vo = api.sort_pairs(tk, tv)
        assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), rep


def test_unaligned_views():
    base = inputs.keys("i32", 300_001, "uniform", seed=3)
    t = dev(base)
    for start in (1, 2, 3):
        view = t[start:]
        out = host(api.sort_keys(view))
        assert np.array_equal(out, oracle.sort(base[start:])), start


def test_deterministic_repeat():
    k = inputs.keys("u32", 3_000_000, "few", seed=4)
    v = np.arange(k.size, dtype=np.uint32)
    tk, tv = dev(k), dev(v)
    a = [host(x) for x in api.sort_pairs(tk, tv)]
    b = [host(x) for x in api.sort_pairs(tk, tv)]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    certify_stable_sort(k, a[0], a[1])


@pytest.mark.parametrize("dt", DTYPES)
def test_sort_segmented_parity(dt):
    g = np.random.default_rng(21)
    for trial in range(3):
        lengths = np.concatenate([g.integers(0, 40, 60), g.integers(8000, 8400, 6), g.integers(0, 5000, 30),
                                  g.integers(9000, 70000, 5), [0, 1, 2]])
        g.shuffle(lengths)
        off = inputs.offsets_from_lengths(lengths)
        n = int(off[-1])
        for dist in ("uniform", "few"):
            say(f"sort_segmented {dt} trial={trial} n={n} nseg={lengths.size} {dist}")
            k = inputs.keys(dt, n, dist, seed=trial)
            v = np.arange(n, dtype=np.uint32)
            ko = api.sort_segmented(dev(k), dev(off))
            assert np.array_equal(host(ko), oracle.sort_segmented(k, off)), (dt, trial, dist)
            ko, vo = api.sort_segmented(dev(k), dev(off), dev(v))
            ek, ev = oracle.sort_segmented(k, off, v)
            assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), (dt, trial, dist)


LONG_SEGMENT_CASES = [
    [40000, 0, 20000, 1, 50000],                 # empty, one-key and partial-tile segments
    [16384, 16383, 16385, 8191, 8193, 8192, 200000],  # around the 8,192-key tile
    [(1 << 20) + 3, 1 << 19, 17, 0, 70000],
    [300000],                                    # one segment: the whole list
    [25000] * 4,                                 # the paper's 10^5-key, p = 4 parts
]


@pytest.mark.parametrize("dt", DTYPES)
def test_sort_segmented_long_segments(dt):
    """Segments averaging > 8,192 keys take whole-device digit passes (tiles
    cut from each segment's start, per-segment digit bases, a look-back that
    ends at the segment's first tile).  Keys and pairs against
    the oracle, also through a view one key into the buffer (unaligned
    tiles)."""
    for ci, lengths in enumerate(LONG_SEGMENT_CASES):
        off = inputs.offsets_from_lengths(np.array(lengths))
        n = int(off[-1])
        for dist in ("uniform", "few", "sorted"):
            say(f"long segments {dt} case={ci} n={n} nseg={len(lengths)} {dist}")
            k = inputs.keys(dt, n, dist, seed=ci)
            v = np.arange(n, dtype=np.uint32)
            assert np.array_equal(host(api.sort_segmented(dev(k), dev(off))), oracle.sort_segmented(k, off)), \
                (dt, ci, dist)
            ko, vo = api.sort_segmented(dev(k), dev(off), dev(v))
            ek, ev = oracle.sort_segmented(k, off, v)
            assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), (dt, ci, dist)
        buf = dev(np.concatenate([k[:1], k]))
        assert np.array_equal(host(api.sort_segmented(buf[1:], dev(off))), oracle.sort_segmented(k, off)), (dt, ci)


def test_sort_segmented_long_in_place():
    lengths = [70000, 1, 33000]
    off = inputs.offsets_from_lengths(np.array(lengths))
    k = inputs.keys("i32", int(off[-1]), "uniform", seed=3)
    v = np.arange(k.size, dtype=np.uint32)
    tk, tv = dev(k), dev(v)
    api.sort_segmented(tk, dev(off), tv, keys_out=tk, vals_out=tv)
    ek, ev = oracle.sort_segmented(k, off, v)
    assert np.array_equal(host(tk), ek) and np.array_equal(host(tv), ev)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("small", [64, 0])
def test_sort_segmented_tiny_segments(dt, small):
    """Segments of 1..80 keys: those of at most 64 go through the one-wave
    bitonic network (ordered by key, then input position) when
    MS_TUNE_SMALL_SORT is 64, through radix passes when it is 0; both give
    the oracle's stable sort, keys and pairs, tie-heavy and uniform keys."""
    from paper_1105_6040_amd import _native as N
    old = N.tune_get(N.MS_TUNE_SMALL_SORT)
    N.tune_set(N.MS_TUNE_SMALL_SORT, small)
    try:
        g = np.random.default_rng(64 + small)
        lengths = np.concatenate([g.integers(1, 81, 3000), [0, 64, 65, 1, 63]])
        g.shuffle(lengths)
        off = inputs.offsets_from_lengths(lengths)
        n = int(off[-1])
        for dist in ("few", "uniform", "extremes"):
            say(f"tiny segments {dt} small={small} n={n} {dist}")
            k = inputs.keys(dt, n, dist, seed=small)
            v = np.arange(n, dtype=np.uint32)
            assert np.array_equal(host(api.sort_segmented(dev(k), dev(off))), oracle.sort_segmented(k, off)), \
                (dt, small, dist)
            ko, vo = api.sort_segmented(dev(k), dev(off), dev(v))
            ek, ev = oracle.sort_segmented(k, off, v)
            assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), (dt, small, dist)
    finally:
        N.tune_set(N.MS_TUNE_SMALL_SORT, old)


def test_sort_segmented_in_place_and_edges():
    k = inputs.keys("i32", 50_000, "uniform", seed=5)
    off = np.array([0, 0, 10, 10, 20_000, 20_001, 50_000, 50_000], dtype=np.uint64)
    t = dev(k)
    api.sort_segmented(t, dev(off), keys_out=t)
    assert np.array_equal(host(t), oracle.sort_segmented(k, off))
    one = np.array([0, 50_000], dtype=np.uint64)
    assert np.array_equal(host(api.sort_segmented(dev(k), dev(one))), oracle.sort(k))


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("nruns", [1, 2, 3, 4, 5, 8, 13, 64])
def test_merge_runs_parity(dt, nruns):
    g = np.random.default_rng(nruns)
    for trial in range(2):
        lengths = g.integers(0, 30_000, nruns)
        if trial == 1 and nruns > 2:
            lengths[g.integers(0, nruns, 2)] = 0
        off = inputs.offsets_from_lengths(lengths)
        n = int(off[-1])
        say(f"merge_runs {dt} nruns={nruns} n={n} trial={trial}")
        k = inputs.keys(dt, n, "small" if trial else "uniform", seed=nruns)
        v = np.arange(n, dtype=np.uint32)
        rk, rv = oracle.sort_segmented(k, off, v)  # sorted runs (input construction)
        ko, vo = api.merge_runs(dev(rk), dev(off), dev(rv))
        ek, ev = oracle.merge_runs(rk, off, rv)
        assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), (dt, nruns, trial)


@pytest.mark.parametrize("dt", DTYPES)
def test_merge_runs_long_runs(dt):
    """Runs of hundreds of merge tiles (most tiles inside one pair: 64-way
    co-rank search, LDS merge), tie-heavy keys for the left-first rule, and a
    view one key into the buffer."""
    lengths = [1 << 20, (1 << 20) + 3, 77, 0, 300001]
    off = inputs.offsets_from_lengths(np.array(lengths))
    n = int(off[-1])
    for dist in ("few", "uniform"):
        say(f"merge_runs long {dt} n={n} {dist}")
        k = inputs.keys(dt, n, dist, seed=len(dist))
        v = np.arange(n, dtype=np.uint32)
        rk, rv = oracle.sort_segmented(k, off, v)  # sorted runs (input construction)
        ek, ev = oracle.merge_runs(rk, off, rv)
        ko, vo = api.merge_runs(dev(rk), dev(off), dev(rv))
        assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), (dt, dist)
        buf = dev(np.concatenate([rk[:1], rk]))
        assert np.array_equal(host(api.merge_runs(buf[1:], dev(off))), ek), (dt, dist)


@pytest.mark.parametrize("dt", DTYPES)
def test_merge_split_parity(dt):
    """Figure 1's odd/even merge-split schedule (p phases over p equal sorted
    parts) against the oracle's merge-split of the same list, and equal to
    merge_runs over the same parts (reading 5: every schedule gives the
    stable sort)."""
    for p in (1, 2, 3, 4, 5, 8, 16, 64):
        for s_len in (1000, 4097):
            n = p * s_len
            for dist in ("uniform", "few"):
                say(f"merge_split {dt} p={p} s={s_len} {dist}")
                k = inputs.keys(dt, n, dist, seed=p + s_len)
                v = np.arange(n, dtype=np.uint32)
                off = oracle.part_offsets(n, p)
                rk, rv = oracle.sort_segmented(k, off, v)  # sorted parts (input construction)
                ek, ev = oracle.merge_split(k, p, v)
                ko, vo = api.merge_split(dev(rk), p, dev(rv))
                assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), (dt, p, s_len, dist)
                mk = api.merge_runs(dev(rk), dev(off))
                assert np.array_equal(host(api.merge_split(dev(rk), p)), host(mk)), (dt, p, s_len, dist)


@pytest.mark.parametrize("dt", ["i32", "u64"])
def test_merge_long_lists(dt):
    """Lists of 2^22 keys and more merge with the larger tiles: merge_runs
    over uneven runs and merge_split over equal parts, pairs, tie-heavy keys,
    against the oracle."""
    lengths = [1 << 21, (1 << 21) + 3, 77, 0, 5, 300001]
    off = inputs.offsets_from_lengths(np.array(lengths))
    n = int(off[-1])
    say(f"long merge_runs {dt} n={n}")
    k = inputs.keys(dt, n, "few", seed=22)
    v = np.arange(n, dtype=np.uint32)
    rk, rv = oracle.sort_segmented(k, off, v)  # sorted runs (input construction)
    ek, ev = oracle.merge_runs(rk, off, rv)
    ko, vo = api.merge_runs(dev(rk), dev(off), dev(rv))
    assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), dt
    p = 4
    n2 = p * ((1 << 20) + 1)
    say(f"long merge_split {dt} n={n2}")
    k2 = inputs.keys(dt, n2, "uniform", seed=23)
    v2 = np.arange(n2, dtype=np.uint32)
    rk2, rv2 = oracle.sort_segmented(k2, oracle.part_offsets(n2, p), v2)
    ek2, ev2 = oracle.merge_split(k2, p, v2)
    ko2, vo2 = api.merge_split(dev(rk2), p, dev(rv2))
    assert np.array_equal(host(ko2), ek2) and np.array_equal(host(vo2), ev2), dt


@pytest.mark.parametrize("p,s_len", [(7, 1), (64, 1), (5, 2), (2, 1), (3, 3)])
def test_merge_split_tiny_parts(p, s_len):
    """Parts of one to three keys: every phase pairs single items (pairs
    against the oracle's merge-split, tie-heavy keys)."""
    n = p * s_len
    k = inputs.keys("i32", n, "few", seed=n)
    v = np.arange(n, dtype=np.uint32)
    rk, rv = oracle.sort_segmented(k, oracle.part_offsets(n, p), v)
    ek, ev = oracle.merge_split(k, p, v)
    ko, vo = api.merge_split(dev(rk), p, dev(rv))
    assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), (p, s_len)


def many_segment_lengths(nseg, nlong, seed):
    """nseg lengths averaging > 8,192: short ones (0 .. 9,000 keys, one tile
    or two, empty ones among them) with nlong long ones (40,000 .. 140,000)
    interleaved at random positions."""
    g = np.random.default_rng(seed)
    lengths = g.integers(0, 9001, nseg)
    lengths[g.integers(0, nseg, 7)] = 0
    lengths[g.integers(0, nseg, 7)] = 8192  # exactly one full tile
    lengths[g.choice(nseg, nlong, replace=False)] = g.integers(40000, 140001, nlong)
    return lengths


@pytest.mark.parametrize("threads", [512, 1024])
@pytest.mark.parametrize("nseg,nlong", [(1025, 60), (2048, 130), (2049, 130), (4700, 320)])
def test_sort_segmented_many_long_segments(nseg, nlong, threads):
    """Segment passes over thousands of segments: the tile table is planned in
    chunks of 2,048 segments (one, exactly one, just over one and three
    chunks here), one-tile segments are stored in place without histograms,
    the rest take per-segment bases and a look-back that ends at their first
    tile.  Keys with both pass tiles (16,384-key tiles apply to key-only
    32-bit sorts), and pairs, against the oracle."""
    lengths = many_segment_lengths(nseg, nlong, nseg)
    off = inputs.offsets_from_lengths(lengths)
    n = int(off[-1])
    assert n > 8192 * nseg  # the segment passes take it
    say(f"many long segments nseg={nseg} n={n} threads={threads}")
    from paper_1105_6040_amd import _native as N
    k = inputs.keys("i32", n, "uniform", seed=nseg)
    old = N.tune_get(N.MS_TUNE_SEG_PASS_THREADS)
    N.tune_set(N.MS_TUNE_SEG_PASS_THREADS, threads)
    try:
        ek = oracle.sort_segmented(k, off)
        assert np.array_equal(host(api.sort_segmented(dev(k), dev(off))), ek), (nseg, threads)
        if threads == 512:
            v = np.arange(n, dtype=np.uint32)
            ko, vo = api.sort_segmented(dev(k), dev(off), dev(v))
            ek, ev = oracle.sort_segmented(k, off, v)
            assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), nseg
    finally:
        N.tune_set(N.MS_TUNE_SEG_PASS_THREADS, old)


@pytest.mark.parametrize("dt", ["i32", "u32", "u64"])
@pytest.mark.parametrize("nseg,nlong", [(7, 5), (1025, 60), (2049, 130), (4700, 320)])
def test_sort_segmented_work_queue(dt, nseg, nlong):
    """MS_TUNE_SEG_PASSES = 2: every phase of the segment passes (histogram,
    P digit passes; one-tile segments sorted whole) in one persistent launch,
    each queue of consecutive segments going on to its next phase once its
    previous one is done.  Keys and pairs against the oracle, over one and
    several planning chunks."""
    from paper_1105_6040_amd import _native as N
    lengths = many_segment_lengths(nseg, nlong, nseg + 7)
    if nseg == 7:
        lengths = np.array([8192, 1, 0, 300_000, 4097, 8193, 65_536], dtype=np.int64)
    off = inputs.offsets_from_lengths(lengths)
    n = int(off[-1])
    assert n > 8192 * nseg
    say(f"work queue {dt} nseg={nseg} n={n}")
    k = inputs.keys(dt, n, "uniform" if nseg != 1025 else "bits16", seed=nseg + 3)
    v = np.arange(n, dtype=np.uint32)
    old = N.tune_get(N.MS_TUNE_SEG_PASSES)
    N.tune_set(N.MS_TUNE_SEG_PASSES, 2)
    try:
        assert np.array_equal(host(api.sort_segmented(dev(k), dev(off))), oracle.sort_segmented(k, off)), nseg
        ko, vo = api.sort_segmented(dev(k), dev(off), dev(v))
        ek, ev = oracle.sort_segmented(k, off, v)
        assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), nseg
    finally:
        N.tune_set(N.MS_TUNE_SEG_PASSES, old)


@pytest.mark.parametrize("seed", range(12))
def test_sort_segmented_work_queue_random_mix(seed):
    """The one-launch queue on seeded mixes of segment lengths around its
    boundaries (empty, one key, one tile exactly, one key past a tile, a
    few tiles, long ones), so that queue starts, one-tile segments and
    ragged last tiles fall everywhere; key types and values vary with the
    seed.  Every segment against the oracle."""
    rng = np.random.default_rng([11, seed])
    nseg = int(rng.integers(2, 48))
    pool = np.array([0, 1, 7, 8191, 8192, 8193, 16384, 16385, 24_000, 65_537, 150_000, 300_000])
    lengths = rng.choice(pool, size=nseg).astype(np.int64)
    lengths[rng.integers(0, nseg)] = 200_000 + int(rng.integers(0, 8192))
    while lengths.sum() <= 8192 * nseg:  # the segment passes take averages above one tile
        lengths[rng.integers(0, nseg)] += 100_000
    off = inputs.offsets_from_lengths(lengths)
    n = int(off[-1])
    assert n > 8192 * nseg
    dt = ("i32", "u32", "u64")[seed % 3]
    say(f"work queue mix seed={seed} {dt} nseg={nseg} n={n}")
    k = inputs.keys(dt, n, ("uniform", "few", "bits16")[(seed // 3) % 3], seed=seed + 40)
    v = np.arange(n, dtype=np.uint32) if seed % 2 else None
    old = N.tune_get(N.MS_TUNE_SEG_PASSES)
    N.tune_set(N.MS_TUNE_SEG_PASSES, 2)
    try:
        if v is None:
            assert np.array_equal(host(api.sort_segmented(dev(k), dev(off))), oracle.sort_segmented(k, off))
        else:
            ko, vo = api.sort_segmented(dev(k), dev(off), dev(v))
            ek, ev = oracle.sort_segmented(k, off, v)
            assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev)
    finally:
        N.tune_set(N.MS_TUNE_SEG_PASSES, old)


@pytest.mark.parametrize("seed", range(8))
def test_sort_segmented_work_queue_moderate_segments(seed):
    """MS_TUNE_SEG_PASSES = 2 takes segments averaging more than 1,024 keys
    (below one tile on average: most segments are sorted whole in LDS in the
    queue's first phase, a few span tiles).  Every segment against the
    oracle; with MS_TUNE_SEG_PASSES = 1 the same call (the persistent
    kernel while the average is at most 8,192) gives the same bytes."""
    rng = np.random.default_rng([12, seed])
    nseg = int(rng.integers(3, 400))
    lengths = rng.integers(1, 6000, nseg).astype(np.int64)
    lengths[rng.integers(0, nseg, 3)] = rng.choice([0, 1, 8192, 8193, 20_000, 70_000], 3)
    while lengths.sum() <= 1024 * nseg:
        lengths[rng.integers(0, nseg)] += 5000
    off = inputs.offsets_from_lengths(lengths)
    n = int(off[-1])
    assert n > 1024 * nseg
    dt = ("i32", "u32", "u64")[seed % 3]
    say(f"work queue moderate seed={seed} {dt} nseg={nseg} n={n}")
    k = inputs.keys(dt, n, ("uniform", "few")[seed % 2], seed=seed + 70)
    v = np.arange(n, dtype=np.uint32) if seed % 2 else None
    old = N.tune_get(N.MS_TUNE_SEG_PASSES)
    try:
        outs = []
        for mode in (2, 1):
            N.tune_set(N.MS_TUNE_SEG_PASSES, mode)
            if v is None:
                outs.append((host(api.sort_segmented(dev(k), dev(off))),))
            else:
                ko, vo = api.sort_segmented(dev(k), dev(off), dev(v))
                outs.append((host(ko), host(vo)))
    finally:
        N.tune_set(N.MS_TUNE_SEG_PASSES, old)
    if v is None:
        assert np.array_equal(outs[0][0], oracle.sort_segmented(k, off))
    else:
        ek, ev = oracle.sort_segmented(k, off, v)
        assert np.array_equal(outs[0][0], ek) and np.array_equal(outs[0][1], ev)
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("nseg,nlong", [(1025, 60), (2049, 130)])
def test_sort_segmented_one_launch_for_long_segments(nseg, nlong):
    """With MS_TUNE_SEG_PASSES = 0 segments averaging > 8,192 keys take the
    one-launch persistent kernel instead of the segment passes: keys and
    pairs against the oracle."""
    from paper_1105_6040_amd import _native as N
    lengths = many_segment_lengths(nseg, nlong, nseg + 1)
    off = inputs.offsets_from_lengths(lengths)
    n = int(off[-1])
    assert n > 8192 * nseg
    say(f"one launch for long segments nseg={nseg} n={n}")
    k = inputs.keys("i32", n, "uniform", seed=nseg + 1)
    v = np.arange(n, dtype=np.uint32)
    old = N.tune_get(N.MS_TUNE_SEG_PASSES)
    N.tune_set(N.MS_TUNE_SEG_PASSES, 0)
    try:
        assert np.array_equal(host(api.sort_segmented(dev(k), dev(off))), oracle.sort_segmented(k, off)), nseg
        ko, vo = api.sort_segmented(dev(k), dev(off), dev(v))
        ek, ev = oracle.sort_segmented(k, off, v)
        assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), nseg
    finally:
        N.tune_set(N.MS_TUNE_SEG_PASSES, old)


def test_sort_segmented_many_segments_u64_keys():
    """64-bit keys (eight passes) over 2,100 segments, key-only, duplicates."""
    lengths = many_segment_lengths(2100, 140, 7)
    off = inputs.offsets_from_lengths(lengths)
    n = int(off[-1])
    assert n > 8192 * 2100
    say(f"many long segments u64 n={n}")
    k = inputs.keys("u64", n, "few", seed=7)
    assert np.array_equal(host(api.sort_segmented(dev(k), dev(off))), oracle.sort_segmented(k, off))


def test_paper_method_small():
    """100,000 int32 keys, p = 4 equal parts: sort each part, merge (Figure 1)."""
    k, p = inputs.paper_small(0)
    off = api.part_offsets(k.size, p, "cuda")
    assert np.array_equal(host(off), oracle.part_offsets(k.size, p))
    v = np.arange(k.size, dtype=np.uint32)
    sk, sv = api.sort_segmented(dev(k), off, dev(v))
    mk, mv = api.merge_runs(sk, off, sv)
    ek, ev = oracle.paper_method(k, p, v)
    assert np.array_equal(host(mk), ek) and np.array_equal(host(mv), ev)


@pytest.mark.parametrize("n", [20001, 200000])
def test_paper_method_process_sweep(n):
    """The paper's method for every process count of its Experiment 1
    (p = 1, 2, 4, ..., 64, Table 1) on pairs: parts sorted by sort_segmented,
    then merged by merge_runs, against the oracle's stable sort."""
    g = np.random.default_rng(n)
    k = g.integers(0, 2**31, n, dtype=np.int64).astype(np.int32)
    v = np.arange(n, dtype=np.uint32)
    ek, ev = oracle.sort(k, v)
    tk, tv = dev(k), dev(v)
    for p in (1, 2, 4, 8, 16, 32, 64):
        say(f"process sweep n={n} p={p}")
        off = api.part_offsets(n, p, "cuda")
        sk, sv = api.sort_segmented(tk, off, tv)
        mk, mv = api.merge_runs(sk, off, sv)
        assert np.array_equal(host(mk), ek) and np.array_equal(host(mv), ev), (n, p)


# ---------------------------------------------------------------------------- full sizes
@pytest.mark.parametrize("dist", ["uniform", "sorted", "dup"])
def test_full_2p28_int32(dist):
    """2^28 int32 keys (all three distributions), compared with the oracle
    element by element: the oracle's method on the host's cores (parts on
    threads, then the master merge).  The closed forms are checked too:
    sorted input comes back unchanged, heavy duplicates as count[v] copies
    of v."""
    say(f"2^28 int32 {dist}: generating")
    k = inputs.keys_2p28(dist, seed=1)
    say(f"2^28 int32 {dist}: sorting")
    out = host(api.sort_keys(dev(k)))
    say(f"2^28 int32 {dist}: the oracle on {fullsize.THREADS} host threads")
    assert np.array_equal(out, fullsize.oracle_whole(k)), dist
    if dist == "dup":
        counts = np.bincount(k, minlength=1024)
        assert np.array_equal(out, np.repeat(np.arange(1024, dtype=np.int32), counts))
    elif dist == "sorted":
        assert np.array_equal(out, k)


def test_full_2p26_pairs_u64():
    say("2^26 u64 pairs: generating")
    k, v = inputs.pairs_2p26(seed=1)
    say("2^26 u64 pairs: sorting")
    ko, vo = api.sort_pairs(dev(k), dev(v))
    ko, vo = host(ko), host(vo)
    say("2^26 u64 pairs: certificate")
    certify_stable_sort(k, ko, vo)
    say(f"2^26 u64 pairs: the oracle on {fullsize.THREADS} host threads")
    ek, ev = fullsize.oracle_whole(k, v)
    assert np.array_equal(ko, ek) and np.array_equal(vo, ev)


def test_tie_dense_pairs():
    """2^24 pairs with keys masked to 16 bits: many ties, so the value order is tested."""
    k = inputs.keys("u64", 1 << 24, "bits16", seed=9)
    v = np.arange(k.size, dtype=np.uint32)
    ko, vo = api.sort_pairs(dev(k), dev(v))
    certify_stable_sort(k, host(ko), host(vo))


# ---------------------------------------------------------------------------- 64-bit counters
def _device_keys(n, seed, hi=2**31):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randint(0, hi, (n,), dtype=torch.int32, device="cuda", generator=g)


def test_big_list_sort_keys_64bit_counters():
    """2^30 + 5 int32 keys: lists of 2^30 keys and more count in 64-bit words
    (digit counts, bases and look-back status).  Compared with the oracle
    (its method on the host's cores) element by element."""
    n = (1 << 30) + 5
    say(f"big sort_keys n={n}")
    k = _device_keys(n, 30)
    out = host(api.sort_keys(k))
    kh = host(k)
    del k
    torch.cuda.empty_cache()
    say(f"big sort_keys: the oracle on {fullsize.THREADS} host threads")
    assert np.array_equal(out, fullsize.oracle_whole(kh))


def test_big_list_sort_pairs_64bit_counters():
    """2^30 + 3 (uint32 key, index) pairs with many ties (keys below 2^20):
    the O(n) certificate of the stable sort on the device — keys
    non-decreasing, values a permutation, keys follow their values, equal
    keys with increasing values."""
    n = (1 << 30) + 3
    say(f"big sort_pairs n={n}")
    k = _device_keys(n, 31, hi=1 << 20).view(torch.uint32)
    v = torch.arange(n, dtype=torch.int64, device="cuda").to(torch.int32).view(torch.uint32)
    ko, vo = api.sort_pairs(k, v)
    ki, vi = ko.view(torch.int32), vo.view(torch.int32).to(torch.int64)
    assert bool((ki[1:] >= ki[:-1]).all())
    seen = torch.zeros(n, dtype=torch.bool, device="cuda")
    seen[vi] = True
    assert bool(seen.all())
    assert torch.equal(k.view(torch.int32)[vi], ki)
    tie = ki[1:] == ki[:-1]
    assert bool((vi[1:][tie] > vi[:-1][tie]).all())
    del k, v, ko, vo, ki, vi, seen, tie
    torch.cuda.empty_cache()


@pytest.mark.parametrize("lengths,seg_passes", [([(1 << 30) + 5, 7, 100_000], 1), ([70_000, (1 << 30) + 1, 3], 1),
                                                 ([70_000, (1 << 30) + 1, 3], 2)])
def test_big_segment_wide_status(lengths, seg_passes):
    """A segment of more than 2^30 keys: the planner flags it and the passes
    (or the one-launch work queue) run with 64-bit look-back status words
    (the 32-bit form is launched too and returns at once).  Every segment
    equals the oracle's sort of it."""
    off = inputs.offsets_from_lengths(np.array(lengths))
    n = int(off[-1])
    say(f"big segment, wide status n={n} seg_passes={seg_passes}")
    k = _device_keys(n, 33)
    old = N.tune_get(N.MS_TUNE_SEG_PASSES)
    N.tune_set(N.MS_TUNE_SEG_PASSES, seg_passes)
    try:
        out = api.sort_segmented(k, dev(off))
        torch.cuda.synchronize()
    finally:
        N.tune_set(N.MS_TUNE_SEG_PASSES, old)
    say("big segment: every segment against the oracle")
    fullsize.compare_segments(k, out, off)
    del out, k
    torch.cuda.empty_cache()


@pytest.mark.parametrize("seg_passes", [1, 2])
def test_big_segments_64bit_counters(seg_passes):
    """Three segments of 2^30 + 11 keys in all (whole-device segment passes,
    or the one-launch work queue, with 64-bit bases; every segment below 2^30
    keys, so 32-bit look-back status words): every segment equals the
    oracle's sort of it."""
    lengths = [(1 << 29) + 7, 3, (1 << 29) + 1]
    off = inputs.offsets_from_lengths(np.array(lengths))
    n = int(off[-1])
    say(f"big sort_segmented n={n} seg_passes={seg_passes}")
    k = _device_keys(n, 32)
    old = N.tune_get(N.MS_TUNE_SEG_PASSES)
    N.tune_set(N.MS_TUNE_SEG_PASSES, seg_passes)
    try:
        out = api.sort_segmented(k, dev(off))
        torch.cuda.synchronize()
    finally:
        N.tune_set(N.MS_TUNE_SEG_PASSES, old)
    say("big sort_segmented: every segment against the oracle")
    fullsize.compare_segments(k, out, off)
    del out, k
    torch.cuda.empty_cache()


def test_segments_workload_full_size():
    """The 50,000-segment workload at its full size (lengths log-uniform in
    [16, 10^6], ~4.56e9 int32 keys, 64-bit counters), as the benchmark runs
    it: every one of the 50,000 segments equals the oracle's sort of the
    same keys, element by element (the oracle over the host's cores,
    tests/fullsize.py); the one-launch persistent kernel gives the same
    bytes."""
    lengths = inputs.segment_lengths(0)
    off = inputs.offsets_from_lengths(lengths)
    n = int(off[-1])
    say(f"segments workload full size n={n} nseg={lengths.size}")
    k = _device_keys(n, 0)
    toff = dev(off)
    out = api.sort_segmented(k, toff)
    torch.cuda.synchronize()
    say(f"segments workload: all {lengths.size} segments against the oracle on {fullsize.THREADS} host threads")
    assert fullsize.compare_segments(k, out, off) == lengths.size
    from paper_1105_6040_amd import _native as N
    old = N.tune_get(N.MS_TUNE_SEG_PASSES)
    try:
        for mode in (p for p in (0, 1, 2) if p != old):
            say(f"segments workload: path MS_TUNE_SEG_PASSES={mode} gives the same result")
            N.tune_set(N.MS_TUNE_SEG_PASSES, mode)
            assert torch.equal(api.sort_segmented(k, toff), out), mode
    finally:
        N.tune_set(N.MS_TUNE_SEG_PASSES, old)
    del out, k
    torch.cuda.empty_cache()


def test_segments_workload_stated_total():
    """The batched workload's segment count at the total it states (~2^27
    keys): 50,000 segments, lengths log-uniform in [16, 19,023], int32 keys
    uniform in [0, 2^31), as the benchmark runs it; every segment equals the
    oracle's sort of the same keys."""
    lengths = inputs.segment_lengths(0, hi=19_023)
    off = inputs.offsets_from_lengths(lengths)
    n = int(off[-1])
    say(f"segments workload [16, 19023] n={n} nseg={lengths.size}")
    k = _device_keys(n, 0)
    out = api.sort_segmented(k, dev(off))
    torch.cuda.synchronize()
    say(f"all {lengths.size} segments against the oracle on {fullsize.THREADS} host threads")
    assert fullsize.compare_segments(k, out, off) == lengths.size
    del out, k
    torch.cuda.empty_cache()
