"""MI355X (gfx950) stable sort: the paper's scatter / sort / merge method on one GPU.

The compute path is the HIP library ``libmi355sort.so`` behind the C ABI of
``include/mi355sort.h``; ``api`` wraps it for PyTorch tensors.  Importing this
package does not load the library or PyTorch; the sort calls do.
"""
_API = ("sort_keys", "sort_pairs", "part_offsets", "sort_segmented", "merge_runs", "merge_split", "key_type")


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
