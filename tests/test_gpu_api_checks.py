"""The binding refuses caller-supplied outputs that do not match the inputs
(device, dtype, length, layout) before anything is enqueued: the library
writes exactly n elements through each output pointer, so a short or
mistyped buffer would otherwise be written out of bounds."""
import numpy as np
import pytest
import torch

import oracle
from paper_1105_6040_amd import api

pytestmark = pytest.mark.gpu

N_KEYS = 1000


def _inputs():
    k = torch.randint(0, 2**31 - 1, (N_KEYS,), dtype=torch.int32, device="cuda")
    v = torch.arange(N_KEYS, dtype=torch.int32, device="cuda").to(torch.uint32)
    off = torch.tensor([0, 400, N_KEYS], dtype=torch.uint64, device="cuda")
    return k, v, off


def _bad_key_outputs(k):
    return [
        torch.empty(N_KEYS - 1, dtype=k.dtype, device="cuda"),         # short
        torch.empty(N_KEYS + 1, dtype=k.dtype, device="cuda"),         # long
        torch.empty(N_KEYS, dtype=torch.uint64, device="cuda"),        # wider dtype
        torch.empty(N_KEYS, dtype=k.dtype),                            # host memory
        torch.empty(2 * N_KEYS, dtype=k.dtype, device="cuda")[::2],    # strided
        torch.empty(N_KEYS, 1, dtype=k.dtype, device="cuda"),          # 2-D
    ]


def _bad_val_outputs():
    return [
        torch.empty(N_KEYS - 1, dtype=torch.uint32, device="cuda"),
        torch.empty(N_KEYS, dtype=torch.uint64, device="cuda"),
        torch.empty(N_KEYS, dtype=torch.uint32),
    ]


def test_sort_keys_rejects_bad_outputs():
    k, _, _ = _inputs()
    for bad in _bad_key_outputs(k):
        with pytest.raises((ValueError, TypeError)):
            api.sort_keys(k, out=bad)


def test_sort_pairs_rejects_bad_outputs():
    k, v, _ = _inputs()
    for bad in _bad_key_outputs(k):
        with pytest.raises((ValueError, TypeError)):
            api.sort_pairs(k, v, keys_out=bad)
    for bad in _bad_val_outputs():
        with pytest.raises((ValueError, TypeError)):
            api.sort_pairs(k, v, vals_out=bad)


@pytest.mark.parametrize("fn", ["sort_segmented", "merge_runs"])
def test_ranged_calls_reject_bad_outputs(fn):
    k, v, off = _inputs()
    call = getattr(api, fn)
    for bad in _bad_key_outputs(k):
        with pytest.raises((ValueError, TypeError)):
            call(k, off, keys_out=bad)
        with pytest.raises((ValueError, TypeError)):
            call(k, off, v, keys_out=bad)
    for bad in _bad_val_outputs():
        with pytest.raises((ValueError, TypeError)):
            call(k, off, v, vals_out=bad)
    with pytest.raises(ValueError):
        call(k, off, vals_out=torch.empty(N_KEYS, dtype=torch.uint32, device="cuda"))  # values out without values in
    with pytest.raises(ValueError):
        call(k, off.cpu())                                                            # offsets on the host
    with pytest.raises((ValueError, TypeError)):
        call(k, off, v.cpu())                                                         # values on the host


def test_merge_split_rejects_bad_outputs():
    k, v, _ = _inputs()
    for bad in _bad_key_outputs(k):
        with pytest.raises((ValueError, TypeError)):
            api.merge_split(k, 4, keys_out=bad)
    for bad in _bad_val_outputs():
        with pytest.raises((ValueError, TypeError)):
            api.merge_split(k, 4, v, vals_out=bad)


def test_workspace_on_the_wrong_device_is_rejected():
    k = torch.randint(0, 2**31 - 1, (1 << 20,), dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        api.sort_keys(k, ws=torch.empty(64 << 20, dtype=torch.uint8))


def test_good_outputs_still_work():
    k, v, off = _inputs()
    ko, vo = torch.empty_like(k), torch.empty_like(v)
    api.sort_segmented(k, off, v, keys_out=ko, vals_out=vo)
    torch.cuda.synchronize()
    ek, ev = oracle.sort_segmented(k.cpu().numpy(), off.cpu().numpy(), v.cpu().numpy())
    assert np.array_equal(ko.cpu().numpy(), ek)
    assert np.array_equal(vo.cpu().numpy(), ev)
