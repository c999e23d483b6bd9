"""The scatter phase (Figure 1): p contiguous parts of about n/p items.

The oracle's boundaries are pinned to the definition part i = [floor(i*n/p),
floor((i+1)*n/p)) through properties that any other split would break: the
parts tile [0, n) in order, every part holds floor(n/p) or ceil(n/p) items,
and item j lies in part ceil((j+1)*p/n) - 1.  The paper's own sizes divide
exactly (its 10^5-key, p = 4 configuration gives 25,000 each).  The library's
``part_offsets`` entry point (C ABI, computed on the GPU) must equal the
oracle bit for bit, including p that does not divide n and products i*n
beyond 64 bits.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1105_6040_amd import _native as N

SIZES = [0, 1, 2, 3, 7, 10, 100, 1000, 100000, 6000000, 2**33 + 5]
PARTS = [1, 2, 3, 4, 7, 8, 16, 64, 1000]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("p", PARTS)
def test_oracle_part_offsets_definition(n, p):
    off = oracle.part_offsets(n, p).astype(object)
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


def test_oracle_paper_configuration():
    assert oracle.part_offsets(100000, 4).tolist() == [0, 25000, 50000, 75000, 100000]
    assert oracle.part_offsets(10, 3).tolist() == [0, 3, 6, 10]


def test_part_offsets_host_errors():
    """Argument errors are found on the host, before anything is enqueued."""
    lib = N.lib()
    fake = ctypes.c_void_p(0x1000)
    assert lib.part_offsets(10, 0, fake, None) == N.MS_EINVAL
    assert "num_parts" in N.last_error()
    assert lib.part_offsets(10, 3, None, None) == N.MS_EINVAL
    assert "NULL" in N.last_error()
    assert lib.part_offsets(10, 2**64 - 1, fake, None) == N.MS_EINVAL


def test_binding_rejects_bad_counts():
    from paper_1105_6040_amd import api
    with pytest.raises(ValueError):
        api.part_offsets(10, 0, "cuda")
    with pytest.raises(ValueError):
        api.part_offsets(-1, 2, "cuda")
    with pytest.raises(ValueError):
        api.part_offsets(10, 2, "cpu")


@pytest.mark.gpu
@pytest.mark.parametrize("n", SIZES + [2**63 + 12345, 2**64 - 1])
@pytest.mark.parametrize("p", PARTS)
def test_part_offsets_on_the_gpu_match_the_oracle(n, p):
    import torch
    from paper_1105_6040_amd import api
    off = api.part_offsets(n, p, "cuda")
    torch.cuda.synchronize()
    got = off.cpu().numpy()
    assert np.array_equal(got, oracle.part_offsets(n, p)), (n, p)


@pytest.mark.gpu
def test_part_offsets_many_parts():
    """p + 1 boundaries beyond one workgroup per boundary (65,536 workgroups
    stride over them), with i*n beyond 64 bits."""
    import torch
    from paper_1105_6040_amd import api
    n, p = 2**40 + 7, 20_000_003
    off = api.part_offsets(n, p, "cuda").cpu().numpy()
    torch.cuda.synchronize()
    assert off.size == p + 1
    idx = np.unique(np.concatenate([np.arange(0, 300), np.arange(p - 300, p + 1),
                                    np.random.default_rng(3).integers(0, p + 1, 2000)]))
    want = np.array([(int(i) * n) // p for i in idx], dtype=np.uint64)
    assert np.array_equal(off[idx], want)
    d = np.diff(off.astype(np.int64))
    assert set(np.unique(d).tolist()) <= {n // p, n // p + 1}


@pytest.mark.gpu
def test_paper_configuration_on_the_gpu():
    from paper_1105_6040_amd import api
    assert api.part_offsets(100000, 4, "cuda").cpu().tolist() == [0, 25000, 50000, 75000, 100000]
    assert api.part_offsets(10, 3, "cuda").cpu().tolist() == [0, 3, 6, 10]
