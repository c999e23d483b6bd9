"""The scatter phase (Figure 1): p contiguous parts of about n/p items.

api.part_offsets is pinned to its definition, part i = [floor(i*n/p),
floor((i+1)*n/p)), through properties that any other split would break:
the parts tile [0, n) in order, every part holds floor(n/p) or ceil(n/p)
items, and item j lies in part ceil((j+1)*p/n) - 1.  The paper's own
sizes divide exactly (its 10^5-key, p = 4 configuration gives 25,000 each).
"""
import numpy as np
import pytest

import oracle
from paper_1105_6040_amd import api


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 100, 1000, 100000, 6000000, 2**33 + 5])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 7, 8, 16, 64, 1000])
def test_part_offsets_definition(n, p):
    off = api.part_offsets(n, p).numpy().astype(object)
    assert off[0] == 0 and off[-1] == n and len(off) == p + 1
    sizes = np.diff(off)
    assert all(s in (n // p, -(-n // p)) for s in sizes), (n, p, set(sizes))
    # Item j lies in part i exactly when i*n/p < j+1 <= (i+1)*n/p, i.e. part
    # ceil((j+1)*p/n) - 1: check the first and the last item of every
    # non-empty part.
    def part_of(j):
        return ((j + 1) * p + n - 1) // n - 1
    for i in range(p):
        if sizes[i]:
            assert part_of(off[i]) == i and part_of(off[i + 1] - 1) == i, (n, p, i)
    assert np.array_equal(api.part_offsets(n, p).numpy(), oracle.part_offsets(n, p))


def test_paper_configuration():
    assert api.part_offsets(100000, 4).tolist() == [0, 25000, 50000, 75000, 100000]


def test_part_offsets_rejects_bad_counts():
    with pytest.raises(ValueError):
        api.part_offsets(10, 0)
    with pytest.raises(ValueError):
        api.part_offsets(-1, 2)
