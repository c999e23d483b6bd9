"""sort_keys_noalloc (C ABI) against sort_keys: the same bytes, with the
workspace taken from the library's static scratch array, on two calls in a
row (the second smaller, so stale scratch contents from the first must not
leak into it), for every key type; and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1105_6040_amd import _native as N, api, inputs

pytestmark = pytest.mark.gpu

KT = {"i32": (N.MS_KEY_I32, torch.int32), "u32": (N.MS_KEY_U32, torch.uint32), "u64": (N.MS_KEY_U64, torch.uint64)}
LIMIT = {"i32": 14_910_784, "u32": 14_910_784, "u64": 7_892_992}


def _noalloc(t: torch.Tensor, kt: int) -> torch.Tensor:
    out = torch.empty_like(t)
    st = N.lib().sort_keys_noalloc(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(out.data_ptr()), t.numel(), kt,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    N.check(st, "sort_keys_noalloc")
    return out


@pytest.mark.parametrize("dt", ["i32", "u32", "u64"])
def test_noalloc_matches_sort_keys_on_two_calls(dt):
    kt, _ = KT[dt]
    for n, dist, seed in ((LIMIT[dt], "uniform", 1), (300_001, "few", 2), (5000, "uniform", 3)):
        k = inputs.keys(dt, n, dist, seed=seed)
        t = torch.from_numpy(k).cuda()
        got = _noalloc(t, kt)
        ref = api.sort_keys(t)
        torch.cuda.synchronize()
        g = got.cpu().numpy()
        assert np.array_equal(g, ref.cpu().numpy()), (dt, n, dist)
        assert np.array_equal(g, oracle.sort(k)), (dt, n, dist)


def test_noalloc_in_place_and_limits():
    k = inputs.keys("i32", 1_000_003, "uniform", seed=4)
    t = torch.from_numpy(k).cuda()
    N.check(N.lib().sort_keys_noalloc(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(t.data_ptr()), t.numel(),
                                      N.MS_KEY_I32, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
            "sort_keys_noalloc")
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle.sort(k))
    fake = ctypes.c_void_p(t.data_ptr())
    assert N.lib().sort_keys_noalloc(fake, fake, LIMIT["i32"] + 1, N.MS_KEY_I32, None) == N.MS_EINVAL
    assert "scratch" in N.last_error()
    assert N.lib().sort_keys_noalloc(fake, fake, LIMIT["u64"] + 1, N.MS_KEY_U64, None) == N.MS_EINVAL
