"""PyTorch-facing calls of the MI355X sort library.

Thin wrappers over the C ABI (``include/mi355sort.h``): they check shapes and
dtypes, allocate outputs and the workspace with PyTorch's caching allocator,
and pass device pointers plus the current HIP stream.  All work runs in the
library's kernels on that stream.

Key dtypes: ``torch.int32`` (signed order), ``torch.uint32``, ``torch.uint64``.
Values are ``torch.uint32`` (``torch.int32`` is accepted and treated as raw
32-bit payload).  Offsets are ``torch.uint64`` or ``torch.int64`` device
tensors with count + 1 entries.
"""
from __future__ import annotations

from typing import Optional, Tuple

import torch

from . import _native as N

KEY_TYPES = {torch.int32: N.MS_KEY_I32, torch.uint32: N.MS_KEY_U32, torch.uint64: N.MS_KEY_U64}


def key_type(keys: torch.Tensor) -> int:
    try:
        return KEY_TYPES[keys.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {keys.dtype}; use int32, uint32 or uint64") from None


def _check_1d(t: torch.Tensor, what: str) -> None:
    if not t.is_cuda:
        raise ValueError(f"{what} must be a GPU tensor")
    if t.dim() != 1:
        raise ValueError(f"{what} must be 1-D")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def _check_vals(vals: torch.Tensor, n: int, what: str = "values") -> None:
    _check_1d(vals, what)
    if vals.dtype not in (torch.uint32, torch.int32):
        raise TypeError(f"{what} must be uint32 (or int32 raw payload)")
    if vals.numel() != n:
        raise ValueError(f"{what} must have as many entries as the keys")


def _check_out(out: torch.Tensor, like: torch.Tensor, what: str) -> None:
    """A caller's output tensor must be a contiguous 1-D GPU tensor on the
    input's device, of the input's dtype and length: the library writes
    exactly n elements of that size through its pointer."""
    _check_1d(out, what)
    if out.device != like.device:
        raise ValueError(f"{what} must be on {like.device} (got {out.device})")
    if out.dtype != like.dtype:
        raise TypeError(f"{what} must have dtype {like.dtype} (got {out.dtype})")
    if out.numel() != like.numel():
        raise ValueError(f"{what} must have {like.numel()} entries (got {out.numel()})")


def _check_offsets(off: torch.Tensor, what: str) -> None:
    _check_1d(off, what)
    if off.dtype not in (torch.uint64, torch.int64):
        raise TypeError(f"{what} must be uint64 (or int64)")
    if off.numel() < 1:
        raise ValueError(f"{what} needs count + 1 >= 1 entries")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def workspace(op: int, kt: int, has_values: bool, n: int, num_segments: int, device,
              provided: Optional[torch.Tensor] = None) -> Tuple[Optional[torch.Tensor], int]:
    need = N.workspace_size(op, kt, has_values, n, num_segments)
    if provided is not None:
        if not provided.is_cuda or provided.device != torch.device(device) or not provided.is_contiguous():
            raise ValueError(f"workspace must be a contiguous tensor on {device}")
        if provided.numel() * provided.element_size() < need:
            raise ValueError(f"workspace too small: need {need} bytes")
        return provided, provided.numel() * provided.element_size()
    if need == 0:
        return None, 0
    return torch.empty(need, dtype=torch.uint8, device=device), need


def sort_keys(keys: torch.Tensor, out: Optional[torch.Tensor] = None,
              ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Stable ascending sort of a 1-D key tensor.  ``out`` may be ``keys`` (in place)."""
    _check_1d(keys, "keys")
    kt = key_type(keys)
    n = keys.numel()
    out = torch.empty_like(keys) if out is None else out
    _check_out(out, keys, "out")
    w, wb = workspace(N.MS_OP_SORT_KEYS, kt, False, n, 0, keys.device, ws)
    N.check(N.lib().sort_keys(_ptr(keys), _ptr(out), n, kt, _ptr(w), wb, _stream(keys.device)), "sort_keys")
    return out


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, keys_out: Optional[torch.Tensor] = None,
               vals_out: Optional[torch.Tensor] = None,
               ws: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """Stable sort of (key, value) pairs by key."""
    _check_1d(keys, "keys")
    kt = key_type(keys)
    n = keys.numel()
    _check_vals(vals, n)
    if vals.device != keys.device:
        raise ValueError(f"values must be on {keys.device} (got {vals.device})")
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    _check_out(keys_out, keys, "keys_out")
    _check_out(vals_out, vals, "vals_out")
    w, wb = workspace(N.MS_OP_SORT_PAIRS, kt, True, n, 0, keys.device, ws)
    N.check(N.lib().sort_pairs(_ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), n, kt, _ptr(w), wb,
                               _stream(keys.device)), "sort_pairs")
    return keys_out, vals_out


def part_offsets(n: int, p: int, device=None) -> torch.Tensor:
    """Scatter phase (Figure 1): the p + 1 boundaries of p contiguous parts of
    a list of n items, part i = [floor(i*n/p), floor((i+1)*n/p)), computed by
    the library's ``part_offsets`` entry point on the GPU (`device`, default
    the current one).  Returns a uint64 device tensor, ready for
    sort_segmented and merge_runs.  No data moves."""
    if p < 1:
        raise ValueError(f"part_offsets: p must be at least 1 (got {p})")
    if n < 0:
        raise ValueError(f"part_offsets: n must be non-negative (got {n})")
    if n >= 1 << 64 or p >= (1 << 64) - 1:
        raise ValueError("part_offsets: n and p must fit in 64 bits")
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    if dev.type != "cuda":
        raise ValueError(f"part_offsets: the library computes the offsets on a GPU, not on {dev}")
    off = torch.empty(p + 1, dtype=torch.uint64, device=dev)
    N.check(N.lib().part_offsets(n, p, _ptr(off), _stream(dev)), "part_offsets")
    return off


def _outputs(keys, vals, keys_out, vals_out):
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    _check_out(keys_out, keys, "keys_out")
    if vals is None:
        if vals_out is not None:
            raise ValueError("vals_out given without vals")
        return keys_out, None
    vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    _check_out(vals_out, vals, "vals_out")
    return keys_out, vals_out


def sort_segmented(keys: torch.Tensor, offsets: torch.Tensor, vals: Optional[torch.Tensor] = None,
                   keys_out: Optional[torch.Tensor] = None, vals_out: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None):
    """Sort every segment [offsets[s], offsets[s+1]) on its own.  Returns keys or (keys, vals)."""
    _check_1d(keys, "keys")
    _check_offsets(offsets, "offsets")
    if offsets.device != keys.device:
        raise ValueError(f"offsets must be on {keys.device} (got {offsets.device})")
    kt = key_type(keys)
    n = keys.numel()
    nseg = offsets.numel() - 1
    if vals is not None:
        _check_vals(vals, n)
        if vals.device != keys.device:
            raise ValueError(f"values must be on {keys.device} (got {vals.device})")
    keys_out, vals_out = _outputs(keys, vals, keys_out, vals_out)
    w, wb = workspace(N.MS_OP_SORT_SEGMENTED, kt, vals is not None, n, nseg, keys.device, ws)
    N.check(N.lib().sort_segmented(_ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), _ptr(offsets), nseg,
                                   n, kt, _ptr(w), wb, _stream(keys.device)), "sort_segmented")
    return keys_out if vals is None else (keys_out, vals_out)


def merge_runs(keys: torch.Tensor, offsets: torch.Tensor, vals: Optional[torch.Tensor] = None,
               keys_out: Optional[torch.Tensor] = None, vals_out: Optional[torch.Tensor] = None,
               ws: Optional[torch.Tensor] = None):
    """Stable merge of the sorted runs [offsets[r], offsets[r+1]).  Returns keys or (keys, vals)."""
    _check_1d(keys, "keys")
    _check_offsets(offsets, "offsets")
    if offsets.device != keys.device:
        raise ValueError(f"offsets must be on {keys.device} (got {offsets.device})")
    kt = key_type(keys)
    n = keys.numel()
    nruns = offsets.numel() - 1
    if vals is not None:
        _check_vals(vals, n)
        if vals.device != keys.device:
            raise ValueError(f"values must be on {keys.device} (got {vals.device})")
    keys_out, vals_out = _outputs(keys, vals, keys_out, vals_out)
    w, wb = workspace(N.MS_OP_MERGE_RUNS, kt, vals is not None, n, nruns, keys.device, ws)
    N.check(N.lib().merge_runs(_ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), _ptr(offsets), nruns, n,
                               kt, _ptr(w), wb, _stream(keys.device)), "merge_runs")
    return keys_out if vals is None else (keys_out, vals_out)


def merge_split(keys: torch.Tensor, p: int, vals: Optional[torch.Tensor] = None,
                keys_out: Optional[torch.Tensor] = None, vals_out: Optional[torch.Tensor] = None,
                ws: Optional[torch.Tensor] = None):
    """Merge p equal sorted parts by Figure 1's odd/even merge-split schedule
    (p phases).  Same result as merge_runs.  Returns keys or (keys, vals)."""
    _check_1d(keys, "keys")
    kt = key_type(keys)
    n = keys.numel()
    if vals is not None:
        _check_vals(vals, n)
        if vals.device != keys.device:
            raise ValueError(f"values must be on {keys.device} (got {vals.device})")
    keys_out, vals_out = _outputs(keys, vals, keys_out, vals_out)
    w, wb = workspace(N.MS_OP_MERGE_SPLIT, kt, vals is not None, n, p, keys.device, ws)
    N.check(N.lib().merge_split(_ptr(keys), _ptr(vals), _ptr(keys_out), _ptr(vals_out), n, p, kt, _ptr(w), wb,
                                _stream(keys.device)), "merge_split")
    return keys_out if vals is None else (keys_out, vals_out)
