"""Pins that tie the CPU oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function raises AssertionError when the oracle disagrees with an
independent fact: brute-force enumeration of the definition on tiny inputs,
closed forms, invariants, the paper's own bubble sort (Figure 2) and NumPy's
stable sort used as a library witness.  None of them re-types the oracle's
merge; they are chosen so that a plausible slip anywhere in ``oracle.c`` (tie
rule, signedness, a lost tail, a bad midpoint, a wrong part boundary, a
missing merge phase) trips at least one of them.  ``tests/test_oracle_mutants.py``
plants such slips and checks that they are caught.

The functions are plain (no pytest fixtures) so that the mutant test can run
them in a subprocess against a mutated build of the oracle.
"""
from __future__ import annotations

import itertools

import numpy as np

import oracle
from paper_1105_6040_amd import inputs

DTYPES = (np.int32, np.uint32, np.uint64)


def _extreme_triples(dt):
    """Ordered value triples x < y < z of dtype dt, including the type's extremes."""
    info = np.iinfo(dt)
    if dt == np.int32:
        return [(-2**31, -1, 0), (-1, 0, 2**31 - 1), (-5, 3, 2**31 - 1), (-2**31, 0, 1)]
    if dt == np.uint32:
        return [(0, 2**31 - 1, 2**31), (0, 1, 2**32 - 1), (7, 2**31, 2**32 - 1)]
    return [(0, 2**32, 2**63), (0, 2**63 - 1, 2**64 - 1), (1, 2**32 - 1, 2**32), (3, 2**63, int(info.max))]


def _stable_perm_by_enumeration(vals):
    """All index permutations of [0, n) that satisfy the definition of the stable
    ascending sort: keys non-decreasing and equal keys in increasing index order."""
    n = len(vals)
    out = []
    for perm in itertools.permutations(range(n)):
        ok = True
        for a, b in zip(perm, perm[1:]):
            if vals[a] > vals[b] or (vals[a] == vals[b] and a > b):
                ok = False
                break
        if ok:
            out.append(perm)
    return out


def _check_against_enumeration(keys):
    py = [int(v) for v in keys]
    perms = _stable_perm_by_enumeration(py)
    assert len(perms) == 1, "the stable sort must be unique"
    perm = np.array(perms[0], dtype=np.int64)
    ko, vo = oracle.sort(keys, np.arange(keys.size, dtype=np.uint32))
    assert np.array_equal(vo.astype(np.int64), perm), (keys, vo, perm)
    assert np.array_equal(ko, keys[perm]), (keys, ko)


def pin_enumeration_small_alphabet():
    """Every input in {x, y, z}^n for n <= 5 (x < y < z, type extremes included)."""
    for dt in DTYPES:
        for x, y, z in _extreme_triples(dt):
            alphabet = np.array([x, y, z], dtype=dt)
            for n in range(0, 6):
                for idx in itertools.product(range(3), repeat=n):
                    _check_against_enumeration(alphabet[list(idx)] if n else np.empty(0, dt))


def pin_enumeration_n7():
    """Random ties-heavy inputs of length 6 and 7 against full enumeration."""
    g = np.random.default_rng(7)
    for dt in DTYPES:
        for x, y, z in _extreme_triples(dt)[:2]:
            pool = np.array([x, y, z, x, z], dtype=dt)
            for n in (6, 7):
                for _ in range(6):
                    _check_against_enumeration(pool[g.integers(0, pool.size, n)])


def pin_all_permutations_distinct_n8():
    """Every ordering of 8 distinct keys sorts to the same ascending list."""
    distinct = {
        np.int32: [-2**31, -2**31 + 1, -70000, -1, 0, 1, 2**31 - 2, 2**31 - 1],
        np.uint32: [0, 1, 255, 256, 2**31 - 1, 2**31, 2**32 - 2, 2**32 - 1],
        np.uint64: [0, 1, 2**32 - 1, 2**32, 2**56, 2**63 - 1, 2**63, 2**64 - 1],
    }
    for dt in DTYPES:
        base = np.array(distinct[dt], dtype=dt)
        assert base.size == 8 and np.all(base[:-1] < base[1:])
        for perm in itertools.permutations(range(8)):
            ko = oracle.sort(base[list(perm)])
            assert np.array_equal(ko, base), (dt, perm, ko)


def pin_bubble_figure2():
    """Figure 2's exchange sort (strict '>' so equal items never pass) agrees."""
    for dt in DTYPES:
        for dist in ("uniform", "small", "few", "extremes", "reverse", "equal"):
            for n in (0, 1, 2, 3, 17, 64, 257, 1000):
                k = inputs.keys(dt, n, dist, seed=3)
                v = np.arange(n, dtype=np.uint32)
                kb, vb = oracle.bubble(k, v)
                ks, vs = oracle.sort(k, v)
                assert np.array_equal(kb, ks) and np.array_equal(vb, vs), (dt, dist, n)


def pin_library_witness():
    """NumPy's stable sort / argsort (a library routine, tests only)."""
    for dt in DTYPES:
        for dist in ("uniform", "pos31", "small", "bits16", "few", "extremes", "sorted", "reverse"):
            for n in (0, 1, 5, 1000, 4097, 65536 + 3):
                k = inputs.keys(dt, n, dist, seed=1)
                v = np.arange(n, dtype=np.uint32)
                ko, vo = oracle.sort(k, v)
                order = np.argsort(k, kind="stable")
                assert np.array_equal(vo, order.astype(np.uint32)), (dt, dist, n)
                assert np.array_equal(ko, k[order]), (dt, dist, n)


def certify_stable_sort(k_in, k_out, v_out):
    """O(n) certificate with values = original index: v_out is a permutation of
    [0, n); k_out[i] == k_in[v_out[i]]; keys non-decreasing; equal keys have
    increasing v_out.  Together these imply the unique stable sort."""
    n = k_in.size
    assert k_out.size == n and v_out.size == n
    if n == 0:
        return
    seen = np.zeros(n, dtype=bool)
    vi = v_out.astype(np.int64)
    assert vi.min() >= 0 and vi.max() < n
    seen[vi] = True
    assert seen.all(), "values are not a permutation"
    assert np.array_equal(k_out, k_in[vi]), "keys do not follow their values"
    a, b = k_out[:-1], k_out[1:]
    assert np.all(a <= b), "keys not non-decreasing"
    eq = a == b
    assert np.all(vi[:-1][eq] < vi[1:][eq]), "equal keys out of original order"


def pin_certificate_large():
    for dt in DTYPES:
        for dist in ("uniform", "small", "bits16"):
            k = inputs.keys(dt, 300_000, dist, seed=5)
            ko, vo = oracle.sort(k, np.arange(k.size, dtype=np.uint32))
            certify_stable_sort(k, ko, vo)


def pin_closed_forms():
    n = 5000
    for dt in DTYPES:
        idx = np.arange(n, dtype=np.uint32)
        e = inputs.keys(dt, n, "equal")
        ko, vo = oracle.sort(e, idx)
        assert np.array_equal(ko, e) and np.array_equal(vo, idx), "all-equal keeps the input order"
        r = inputs.keys(dt, n, "reverse")
        ko, vo = oracle.sort(r, idx)
        assert np.array_equal(ko, r[::-1]) and np.array_equal(vo, idx[::-1]), "reverse is reversed"
        s = np.sort(inputs.keys(dt, n, "uniform"))
        assert np.array_equal(oracle.sort(s), s), "sorted input is a fixed point"
    # heavy duplicates in [0, 1023]: count[v] copies of v for v = 0, 1, ...
    d = inputs.keys("i32", 200_000, "small", seed=2)
    counts = np.bincount(d, minlength=1024)
    assert np.array_equal(oracle.sort(d), np.repeat(np.arange(1024, dtype=np.int32), counts))


def pin_segmented():
    g = np.random.default_rng(11)
    for dt in DTYPES:
        for _ in range(4):
            lengths = g.integers(0, 600, 40)
            lengths[g.integers(0, 40, 6)] = 0
            off = inputs.offsets_from_lengths(lengths)
            n = int(off[-1])
            k = inputs.keys(dt, n, "few", seed=int(g.integers(0, 100)))
            v = np.arange(n, dtype=np.uint32)
            ko, vo = oracle.sort_segmented(k, off, v)
            for s in range(lengths.size):
                a, b = int(off[s]), int(off[s + 1])
                order = np.argsort(k[a:b], kind="stable") + a
                assert np.array_equal(vo[a:b], order.astype(np.uint32)), (dt, s)
                assert np.array_equal(ko[a:b], k[order]), (dt, s)


def pin_merge_runs():
    g = np.random.default_rng(12)
    for dt in DTYPES:
        for nruns in (1, 2, 3, 4, 7, 16):
            lengths = g.integers(0, 300, nruns)
            off = inputs.offsets_from_lengths(lengths)
            n = int(off[-1])
            k = inputs.keys(dt, n, "small", seed=nruns)
            for r in range(nruns):  # make every run sorted (input construction)
                a, b = int(off[r]), int(off[r + 1])
                k[a:b] = np.sort(k[a:b], kind="stable")
            v = np.arange(n, dtype=np.uint32)
            ko, vo = oracle.merge_runs(k, off, v)
            order = np.argsort(k, kind="stable")
            assert np.array_equal(vo, order.astype(np.uint32)), (dt, nruns)
            assert np.array_equal(ko, k[order])
    bad = np.array([3, 1, 2], dtype=np.int32)
    try:
        oracle.merge_runs(bad, np.array([0, 3], dtype=np.uint64))
    except oracle.OracleError:
        pass
    else:
        raise AssertionError("an unsorted run must be rejected")


def pin_paper_method_schedules():
    """Figure 1 / Section 3.2.2: any p, with the master merge or the odd/even
    merge-split schedule, gives the whole-array stable sort."""
    for dt in DTYPES:
        for n in (0, 1, 2, 7, 100, 1001, 4096):
            for p in (1, 2, 3, 4, 5, 8, 9, 64):
                k = inputs.keys(dt, n, "few", seed=n + p)
                v = np.arange(n, dtype=np.uint32)
                ks, vs = oracle.sort(k, v)
                km, vm = oracle.paper_method(k, p, v)
                assert np.array_equal(km, ks) and np.array_equal(vm, vs), (dt, n, p, "master")
            for p in (1, 2, 3, 4, 5, 8, 16):
                m = n - n % p  # the merge-split schedule needs equal parts
                k = inputs.keys(dt, m, "few", seed=n + p)
                v = np.arange(m, dtype=np.uint32)
                ks, vs = oracle.sort(k, v)
                kx, vx = oracle.merge_split(k, p, v)
                assert np.array_equal(kx, ks) and np.array_equal(vx, vs), (dt, m, p, "merge-split")
    assert list(oracle.part_offsets(100_000, 4)) == [0, 25_000, 50_000, 75_000, 100_000]
    assert list(oracle.part_offsets(10, 3)) == [0, 3, 6, 10]


def pin_paper_workload_small():
    """The small paper workload: 10^5 int32, p = 4 parts."""
    k, p = inputs.paper_small(0)
    v = np.arange(k.size, dtype=np.uint32)
    km, vm = oracle.paper_method(k, p, v)
    certify_stable_sort(k, km, vm)
    kt, vt = oracle.paper_method_threads(k, p, v)
    assert np.array_equal(kt, km) and np.array_equal(vt, vm)


ALL_PINS = [
    pin_enumeration_small_alphabet,
    pin_enumeration_n7,
    pin_all_permutations_distinct_n8,
    pin_bubble_figure2,
    pin_library_witness,
    pin_certificate_large,
    pin_closed_forms,
    pin_segmented,
    pin_merge_runs,
    pin_paper_method_schedules,
    pin_paper_workload_small,
]


def run_all():
    for pin in ALL_PINS:
        pin()


if __name__ == "__main__":
    run_all()
