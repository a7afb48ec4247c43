"""Kernel-level entry points (include/cayleygrowth_testing.h) on torch
device tensors: each runs one stage of the layer step on the caller's
buffers. Keys travel as ``torch.int64`` tensors holding the uint64 bits.
"""

from __future__ import annotations

import ctypes
from typing import Sequence, Tuple

import numpy as np

from . import _native as N
from .api import _check, _gens_array


def _stream(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dptr(t) -> int:
    return int(t.data_ptr())


def pack(n: int, rows: np.ndarray, device="cuda", stream=None):
    import torch

    rows = np.ascontiguousarray(rows, dtype=np.uint8).reshape(-1, n)
    out = torch.empty(rows.shape[0], dtype=torch.int64, device=device)
    _check(N.lib().cg_test_pack(n, rows.ctypes.data_as(N.u8p), rows.shape[0], _dptr(out), _stream(stream)))
    return out


def unpack(n: int, keys, stream=None) -> np.ndarray:
    out = np.zeros((keys.numel(), n), dtype=np.uint8)
    _check(N.lib().cg_test_unpack(n, _dptr(keys), keys.numel(), out.ctypes.data_as(N.u8p), _stream(stream)))
    return out


def expand(n: int, gens: Sequence[Sequence[int]], frontier, stream=None):
    import torch

    g = _gens_array(n, gens)
    out = torch.empty(frontier.numel() * g.shape[0], dtype=torch.int64, device=frontier.device)
    _check(N.lib().cg_test_expand(n, g.ctypes.data_as(N.u8p), g.shape[0], _dptr(frontier),
                                  frontier.numel(), _dptr(out), _stream(stream)))
    return out


def sort(keys, bit_lo: int, bit_hi: int, stream=None):
    import torch

    tmp = torch.empty_like(keys)
    _check(N.lib().cg_test_sort(_dptr(keys), _dptr(tmp), keys.numel(), bit_lo, bit_hi, _stream(stream)))
    return keys


def sort_below(keys, key_bits: int, stream=None):
    """Sorted in place on bits [0, key_bits) in digits of balanced widths
    (the sort of 64-bit ranks and of binary states)."""
    import torch

    tmp = torch.empty_like(keys)
    _check(N.lib().cg_test_sort_below(_dptr(keys), _dptr(tmp), keys.numel(), key_bits, _stream(stream)))
    return keys


def sort32(keys, bit_lo: int, bit_hi: int, stream=None):
    """32-bit keys (an int32 tensor holding the bit patterns), sorted in place."""
    import torch

    tmp = torch.empty_like(keys)
    _check(N.lib().cg_test_sort32(_dptr(keys), _dptr(tmp), keys.numel(), bit_lo, bit_hi, _stream(stream)))
    return keys


def dedup(sorted_keys, a, b, stream=None):
    import torch

    out = torch.empty(max(sorted_keys.numel(), 1), dtype=torch.int64, device=sorted_keys.device)
    cnt = ctypes.c_uint64(0)
    _check(N.lib().cg_test_dedup(_dptr(sorted_keys), sorted_keys.numel(), _dptr(a), a.numel(),
                                 _dptr(b), b.numel(), _dptr(out), ctypes.byref(cnt), _stream(stream)))
    return out[: cnt.value]


def layer_step(n: int, gens, frontier, prev, stream=None):
    import torch

    g = _gens_array(n, gens)
    out = torch.empty(max(frontier.numel() * g.shape[0], 1), dtype=torch.int64, device=frontier.device)
    cnt = ctypes.c_uint64(0)
    _check(N.lib().cg_test_layer_step(n, g.ctypes.data_as(N.u8p), g.shape[0], _dptr(frontier),
                                      frontier.numel(), _dptr(prev), prev.numel(), _dptr(out),
                                      ctypes.byref(cnt), _stream(stream)))
    return out[: cnt.value]


def copy(src, dst, repeats: int = 1, stream=None):
    """Plain device copy of src into dst (same byte size, a multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy needs buffers of the same byte size")
    _check(N.lib().cg_test_copy(_dptr(src), _dptr(dst), nbytes, repeats, _stream(stream)))


def to_u64(t) -> np.ndarray:
    """Copy a device int64 key tensor to host uint64."""
    return t.cpu().numpy().view(np.uint64)


def from_u64(a: np.ndarray, device="cuda"):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to(device)
