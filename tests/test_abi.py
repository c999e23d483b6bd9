"""The C-ABI library loads, exports what the header declares, and rejects bad
arguments on the host before touching a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_1105_6040_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mi355sort.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("sort_keys", "sort_pairs", "sort_segmented", "merge_runs", "merge_split", "ms_workspace_size",
               "ms_last_error"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    lib = N.lib()
    for fn in declared_functions():
        assert hasattr(lib, fn), f"{fn} declared in mi355sort.h but not exported"


def test_workspace_sizes():
    ws = N.workspace_size
    assert ws(N.MS_OP_SORT_KEYS, N.MS_KEY_I32, False, 0) == 0
    assert ws(N.MS_OP_SORT_KEYS, N.MS_KEY_I32, False, 100) == 0          # one LDS tile: no workspace
    big = ws(N.MS_OP_SORT_KEYS, N.MS_KEY_I32, False, 2**28)
    assert 2**28 * 4 <= big <= 2**28 * 5                                  # ping-pong buffer + look-back state
    pairs = ws(N.MS_OP_SORT_PAIRS, N.MS_KEY_U64, True, 2**26)
    assert 2**26 * 12 <= pairs
    assert ws(N.MS_OP_MERGE_RUNS, N.MS_KEY_I32, False, 1000, 2) == 0     # one round: no workspace
    assert ws(N.MS_OP_MERGE_RUNS, N.MS_KEY_I32, True, 1000, 4) >= 1000 * 8
    assert ws(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_U32, True, 5000, 7) >= 5000 * 8


def test_workspace_size_errors():
    lib = N.lib()
    assert lib.ms_workspace_size(0, 0, 0, 10, 0, None) == N.MS_EINVAL
    out = ctypes.c_size_t()
    assert lib.ms_workspace_size(0, 7, 0, 10, 0, ctypes.byref(out)) == N.MS_ENOTSUP
    assert lib.ms_workspace_size(9, 0, 0, 10, 0, ctypes.byref(out)) == N.MS_ENOTSUP


def test_host_side_argument_errors():
    lib = N.lib()
    # n = 0 is a no-op with any pointers
    assert lib.sort_keys(None, None, 0, N.MS_KEY_I32, None, 0, None) == N.MS_OK
    assert lib.sort_keys(None, None, 10, N.MS_KEY_I32, None, 0, None) == N.MS_EINVAL
    assert "NULL" in N.last_error()
    assert lib.sort_keys(None, None, 10, 5, None, 0, None) == N.MS_ENOTSUP
    # short workspace: detected before any launch (pointers are never dereferenced)
    fake = ctypes.c_void_p(0x1000)
    assert lib.sort_keys(fake, fake, 10**6, N.MS_KEY_I32, None, 0, None) == N.MS_EINVAL
    assert "workspace" in N.last_error()
    # pairs: keys in place but values not
    assert lib.sort_pairs(fake, ctypes.c_void_p(0x2000), fake, ctypes.c_void_p(0x3000), 5, 0, None, 0,
                          None) == N.MS_EINVAL
    # segmented: no segments but items; one of vals_in / vals_out
    assert lib.sort_segmented(fake, None, fake, None, None, 0, 5, 0, None, 0, None) == N.MS_EINVAL
    assert lib.sort_segmented(fake, fake, fake, None, fake, 1, 5, 0, None, 0, None) == N.MS_EINVAL
    assert lib.sort_segmented(None, None, None, None, None, 0, 0, 0, None, 0, None) == N.MS_OK
    # merge: zero runs, aliasing
    assert lib.merge_runs(fake, None, ctypes.c_void_p(0x2000), None, fake, 0, 5, 0, None, 0, None) == N.MS_EINVAL
    assert lib.merge_runs(fake, None, fake, None, fake, 2, 5, 0, None, 0, None) == N.MS_EINVAL
    assert "alias" in N.last_error()


def _align(x, a=256):
    return (x + a - 1) // a * a


def test_sort_keys_workspace_follows_the_layout():
    """ms_workspace_size for sort_keys of int32 keys is the documented layout:
    plan (512 B), counters (256 B), digit histograms and bases (2 x 4 x 256 x
    4 B), two look-back status buffers of ceil(n / 4096) rows of 256 words,
    and the n-key ping-pong buffer; 1,207,968,512 B at 2^28 keys."""
    for n in (8193, 100_000, (1 << 20) + 1, 6_000_000, 1 << 28):
        rows = -(-n // 4096)
        expect = 512 + 256 + 2 * 4 * 256 * 4 + 2 * _align(rows * 256 * 4) + _align(4 * n)
        assert N.workspace_size(N.MS_OP_SORT_KEYS, N.MS_KEY_I32, False, n) == expect, n
    assert N.workspace_size(N.MS_OP_SORT_KEYS, N.MS_KEY_I32, False, 1 << 28) == 1_207_968_512


def test_memory_against_list_size():
    """The memory experiment (bench.py --memory): device bytes grow by 12.5 B
    per int32 key for sort_keys (in, out, ping-pong, status) over Table 2's
    2.5..5 x 10^6 range, and stay affine in n."""
    import bench
    t = bench.memory_table()
    assert t["bytes_per_key_2p5e6_to_5e6"]["sort_keys"] == 12.5
    big = [r for r in t["rows"] if r["n"] >= 2_500_000]
    steps = {b["sort_keys_bytes"] - a["sort_keys_bytes"] for a, b in zip(big, big[1:])}
    assert max(steps) - min(steps) <= 2 * 1024 + 256, steps  # status rows and alignment only


def test_merge_split_host_side_errors():
    """Figure 1's schedule needs p equal parts: checked on the host."""
    lib = N.lib()
    a, b = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
    assert lib.merge_split(a, None, b, None, 0, 3, N.MS_KEY_I32, None, 0, None) == N.MS_OK   # empty list
    assert lib.merge_split(a, None, b, None, 10, 0, N.MS_KEY_I32, None, 0, None) == N.MS_EINVAL
    assert lib.merge_split(a, None, b, None, 10, 3, N.MS_KEY_I32, None, 0, None) == N.MS_EINVAL
    assert "equal parts" in N.last_error()
    assert lib.merge_split(a, None, a, None, 12, 3, N.MS_KEY_I32, None, 0, None) == N.MS_EINVAL    # aliasing
    assert lib.merge_split(a, a, b, None, 12, 3, N.MS_KEY_I32, None, 0, None) == N.MS_EINVAL       # one of the values
    assert lib.merge_split(a, None, b, None, 12, 3, 9, None, 0, None) == N.MS_ENOTSUP
    assert lib.merge_split(a, None, b, None, 12 * 10**5, 3, N.MS_KEY_I32, None, 0, None) == N.MS_EINVAL
    assert "workspace" in N.last_error()
    ws = N.workspace_size
    assert ws(N.MS_OP_MERGE_SPLIT, N.MS_KEY_I32, False, 1000, 1) == 0      # one part: a copy
    assert ws(N.MS_OP_MERGE_SPLIT, N.MS_KEY_U64, True, 1000, 4) >= 1000 * 12


def test_tune_parameter_checks():
    """ms_tune_set accepts only the documented values and keeps the old one
    otherwise (host only)."""
    lib = N.lib()
    get = lib.ms_tune_get
    old = get(N.MS_TUNE_SEG_PASS_THREADS)
    assert old in (512, 1024)
    try:
        for bad in (0, 256, 2048):
            assert lib.ms_tune_set(N.MS_TUNE_SEG_PASS_THREADS, bad) == N.MS_EINVAL
            assert get(N.MS_TUNE_SEG_PASS_THREADS) == old
        assert lib.ms_tune_set(N.MS_TUNE_SEG_PASS_THREADS, 1024) == N.MS_OK
        assert get(N.MS_TUNE_SEG_PASS_THREADS) == 1024
    finally:
        lib.ms_tune_set(N.MS_TUNE_SEG_PASS_THREADS, old)
    assert lib.ms_tune_set(N.MS_TUNE_PASS_THREADS, 300) == N.MS_EINVAL
    assert lib.ms_tune_set(N.MS_TUNE_SMALL_SORT, 32) == N.MS_EINVAL
    old = get(N.MS_TUNE_SEG_PASSES)
    assert old in (0, 1, 2)
    assert lib.ms_tune_set(N.MS_TUNE_SEG_PASSES, 3) == N.MS_EINVAL
    assert lib.ms_tune_set(N.MS_TUNE_SEG_PASSES, -1) == N.MS_EINVAL
    assert get(N.MS_TUNE_SEG_PASSES) == old
    assert lib.ms_tune_set(6, 1) == N.MS_EINVAL  # MS_TUNE_COUNT is no parameter
    assert get(6) == 0


def test_segmented_workspace_for_the_queue_on_shorter_segments():
    """Segments averaging 1,024 - 8,192 keys: the workspace grows for the
    one-launch queue only while MS_TUNE_SEG_PASSES is 2 at sizing time (8 KiB
    of counters and bases per segment), and stays at the persistent kernel's
    otherwise."""
    ws = N.workspace_size
    old = N.tune_get(N.MS_TUNE_SEG_PASSES)
    try:
        for n, nseg in ((135_020_572, 50_000), (1 << 31, 1 << 18), (3000 * 7, 7)):
            N.tune_set(N.MS_TUNE_SEG_PASSES, 1)
            plain = ws(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, n, nseg)
            N.tune_set(N.MS_TUNE_SEG_PASSES, 0)
            assert ws(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, n, nseg) == plain
            N.tune_set(N.MS_TUNE_SEG_PASSES, 2)
            queue = ws(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, n, nseg)
            assert 4 * n <= plain <= 1.3 * 4 * n + 16 * nseg + (1 << 20), (n, nseg, plain)
            assert plain < queue <= plain + 8192 * nseg + 3 * 4 * n, (n, nseg, plain, queue)
        # 1,024 keys on average or fewer: the persistent kernel in every mode
        sizes = set()
        for mode in (0, 1, 2):
            N.tune_set(N.MS_TUNE_SEG_PASSES, mode)
            sizes.add(ws(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, 1024 * 100, 100))
        assert len(sizes) == 1
    finally:
        N.tune_set(N.MS_TUNE_SEG_PASSES, old)


def test_segmented_workspace_stays_near_the_keys():
    """sort_segmented's workspace is the ping-pong copy of the keys plus a
    bounded overhead on either path (host arithmetic only): the segment
    passes only take segments averaging more than 8,192 keys, whose
    per-segment histograms and bases cost at most 1 B per key."""
    ws = N.workspace_size
    for n, nseg in ((4_563_337_368, 50_000), (1 << 32, 1 << 26), (10**6, 3), (10**6, 10**5), (1 << 31, 1 << 18)):
        b = ws(N.MS_OP_SORT_SEGMENTED, N.MS_KEY_I32, False, n, nseg)
        assert 4 * n <= b <= 1.3 * 4 * n + 16 * nseg + (1 << 20), (n, nseg, b)
