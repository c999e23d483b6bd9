"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case copies ``oracle/oracle.c``, plants one plausible slip by a textual
substitution, builds the mutant with gcc into a temporary directory and runs
every pin against it in a subprocess.  The pins must fail for every mutant;
the unmodified oracle passes them (``test_oracle.py``).
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    # merge sort takes the right run's item on ties -> not stable
    "merge_tie_right": ("if (key_le(kt, left[i].key, right[j].key))",
                        "if (key_lt(kt, left[i].key, right[j].key))"),
    # int32 compared as unsigned -> negatives sort after positives
    "int32_unsigned": ("return (int32_t)(uint32_t)a <= (int32_t)(uint32_t)b;",
                       "return (uint32_t)a <= (uint32_t)b;"),
    # the left run's leftover tail is dropped in the merge
    "lost_left_tail": ("    while (i < lcount)\n        scratch[k++] = left[i++];\n    while (j < ucount)\n        scratch[k++] = right[j++];\n    memcpy",
                       "    while (j < ucount)\n        scratch[k++] = right[j++];\n    memcpy"),
    # Figure 3's lcount without the +1
    "lcount_off_by_one": ("uint64_t lcount = mid - first + 1;", "uint64_t lcount = mid - first;"),
    # the master merge puts the later run first on ties
    "master_merge_tie": ("if (key_le(kt, a[i].key, b[j].key))", "if (key_lt(kt, a[i].key, b[j].key))"),
    # part boundaries computed as i * (n / p): the tail past p * floor(n/p) is lost
    "partition_floor": ("return (uint64_t)(((unsigned __int128)i * n) / p);", "return i * (n / p);"),
    # merge-split without the odd phases
    "no_odd_phase": ("for (uint64_t id = step % 2; id + 1 < p; id += 2)",
                     "for (uint64_t id = 0; id + 1 < p; id += 2)"),
    # uint64 keys read as 32-bit
    "u64_truncated": ("    if (kt == ORACLE_U64)\n        return ((const uint64_t *)keys)[i];",
                      "    if (kt == ORACLE_U32)\n        return ((const uint64_t *)keys)[i];"),
    # Figure 2's inner loop one short
    "bubble_short": ("for (int64_t j = 0; j <= i; j++)", "for (int64_t j = 0; j < i; j++)"),
    # the last segment is left unsorted
    "last_segment_skipped": ("for (uint64_t s = 0; s < nseg && rc == 0; s++)",
                             "for (uint64_t s = 0; s + 1 < nseg && rc == 0; s++)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique in oracle.c"
    mut_src = tmp_path / "oracle_mut.c"
    mut_src.write_text(src.replace(old, new))
    lib = str(tmp_path / "liboracle_mut.so")
    oracle.build(out=lib, src=str(mut_src), extra_flags=("-w",))
    env = dict(os.environ, ORACLE_LIB=lib, PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", "from tests import oracle_pins; oracle_pins.run_all()"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} survived every pin"
    assert "AssertionError" in r.stderr or "OracleError" in r.stderr or r.returncode < 0, r.stderr[-2000:]
