"""DovetailSort on MI355X: Python entry points over libdtsort.so.

torch is used only to hold device memory and to name the current stream; all
sorting work runs in the library's HIP kernels through its C ABI.  Keys are
unsigned integers carried in torch's signed dtypes (int32 / int64) by bit
pattern.
"""
from __future__ import annotations

import ctypes as C

from . import _lib
from ._lib import (MERGE_GATHER, MERGE_INPLACE, MERGE_NONE, MERGE_PLMERGE, MERGE_SPLIT, MODE_LEARNED,  # noqa: F401
                   MODE_PLAIN, MODE_SAMPLING, DTSortError, Opts, Stats)

__all__ = ["sort_u32", "sort_u64", "sort_pairs_u64", "sort_pairs_u32", "sort_segmented", "sort_segmented_noalloc", "graph_transpose",
           "morton_sort", "copy_u32", "make_opts", "Stats",
           "MODE_SAMPLING", "MODE_PLAIN", "MODE_LEARNED", "MERGE_GATHER", "MERGE_PLMERGE", "MERGE_INPLACE",
           "MERGE_NONE", "MERGE_SPLIT", "DTSortError"]


def make_opts(seed=0, key_bits=0, mode=MODE_SAMPLING, digit_bits=0, lds_cutoff=0, tuned=0,
              learned_steps=0, learned_batch=0, learned_lr=0.0, stats: Stats | None = None,
              workspace=None, profile=0, tile_shape=0, graph=0, ordered_ranks=0, merge_variant=0,
              learned_judge=0, digit_bits_below=0) -> Opts:
    o = Opts()
    _lib.load().dtsort_default_opts(C.byref(o))
    o.seed, o.key_bits, o.mode, o.digit_bits, o.lds_cutoff, o.tuned = seed, key_bits, mode, digit_bits, lds_cutoff, tuned
    o.learned_steps, o.learned_batch, o.learned_lr = learned_steps, learned_batch, learned_lr
    o.profile = profile
    o.tile_shape, o.graph, o.ordered_ranks, o.merge_variant = tile_shape, graph, ordered_ranks, merge_variant
    o.learned_judge, o.digit_bits_below = learned_judge, digit_bits_below
    if stats is not None:
        o.stats = C.pointer(stats)
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


def _stream(t):
    import torch
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _check_tensor(t, dtype_bytes):
    if not t.is_cuda:
        raise ValueError("dtsort sorts device tensors only")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if t.element_size() != dtype_bytes:
        raise ValueError(f"expected {dtype_bytes}-byte elements, got {t.element_size()}")


def sort_u32(keys, opts: Opts | None = None):
    """Stable in-place ascending sort of a 1-D device tensor of 32-bit keys."""
    _check_tensor(keys, 4)
    o = opts if opts is not None else make_opts()
    _lib.check(_lib.load().dtsort_u32(keys.data_ptr(), keys.numel(), C.byref(o), _stream(keys)))
    return keys


def sort_u64(keys, opts: Opts | None = None):
    """Stable in-place ascending sort of a 1-D device tensor of 64-bit keys."""
    _check_tensor(keys, 8)
    o = opts if opts is not None else make_opts()
    _lib.check(_lib.load().dtsort_u64(keys.data_ptr(), keys.numel(), C.byref(o), _stream(keys)))
    return keys


def sort_pairs_u64(keys, values, opts: Opts | None = None):
    """Stable in-place sort of (64-bit key, 64-bit value) records by key."""
    _check_tensor(keys, 8)
    _check_tensor(values, 8)
    if values.numel() != keys.numel():
        raise ValueError("keys and values differ in length")
    o = opts if opts is not None else make_opts()
    _lib.check(_lib.load().dtsort_pairs_u64(keys.data_ptr(), values.data_ptr(), keys.numel(), C.byref(o),
                                            _stream(keys)))
    return keys, values


def sort_pairs_u32(keys, values, opts: Opts | None = None):
    """Stable in-place sort of (32-bit key, 32-bit value) records by key."""
    _check_tensor(keys, 4)
    _check_tensor(values, 4)
    if values.numel() != keys.numel():
        raise ValueError("keys and values differ in length")
    o = opts if opts is not None else make_opts()
    _lib.check(_lib.load().dtsort_pairs_u32(keys.data_ptr(), values.data_ptr(), keys.numel(), C.byref(o),
                                            _stream(keys)))
    return keys, values


def sort_segmented(keys, offsets, values=None, opts: Opts | None = None):
    """Independent stable sorts of keys[offsets[s]:offsets[s+1]] (32-bit keys,
    optional 32-bit values); offsets is a device int64 tensor of n_seg + 1."""
    _check_tensor(keys, 4)
    _check_tensor(offsets, 8)
    vp = None
    if values is not None:
        _check_tensor(values, 4)
        if values.numel() != keys.numel():
            raise ValueError("keys and values differ in length")
        vp = values.data_ptr()
    o = opts if opts is not None else make_opts()
    _lib.check(_lib.load().dtsort_segmented(keys.data_ptr(), vp, keys.numel(), offsets.data_ptr(),
                                            offsets.numel() - 1, C.byref(o), _stream(keys)))
    return keys if values is None else (keys, values)


def sort_segmented_noalloc(keys, offsets, values=None, opts: Opts | None = None):
    """sort_segmented through the allocation-free entry point (buffers in the
    library's static device scratch; inputs of up to about 2^22 keys)."""
    _check_tensor(keys, 4)
    _check_tensor(offsets, 8)
    vp = None
    if values is not None:
        _check_tensor(values, 4)
        if values.numel() != keys.numel():
            raise ValueError("keys and values differ in length")
        vp = values.data_ptr()
    o = opts if opts is not None else make_opts()
    _lib.check(_lib.load().dtsort_segmented_noalloc(keys.data_ptr(), vp, keys.numel(), offsets.data_ptr(),
                                                    offsets.numel() - 1, C.byref(o), _stream(keys)))
    return keys if values is None else (keys, values)


def graph_transpose(offsets, targets, n_vertices: int, opts: Opts | None = None):
    """Reverse every edge of a CSR graph (offsets: int64 [V + 1], targets:
    int32 [E], device tensors); returns (t_offsets, t_targets) in CSR form,
    in-neighbours in edge-list order."""
    import torch
    _check_tensor(offsets, 8)
    _check_tensor(targets, 4)
    if offsets.numel() != n_vertices + 1:
        raise ValueError("offsets must hold n_vertices + 1 entries")
    t_off = torch.empty_like(offsets)
    t_tgt = torch.empty_like(targets)
    o = opts if opts is not None else make_opts()
    _lib.check(_lib.load().dtsort_graph_transpose(offsets.data_ptr(), targets.data_ptr(), n_vertices, targets.numel(),
                                                  t_off.data_ptr(), t_tgt.data_ptr(), C.byref(o), _stream(targets)))
    return t_off, t_tgt


def morton_sort(coords, opts: Opts | None = None):
    """Morton order of points coords [dims, n] (int32, dims 2 or 3, low
    32 // dims bits per coordinate): returns (sorted z-values, point indices)."""
    import torch
    if coords.dim() != 2:
        raise ValueError("coords must be [dims, n]")
    c = coords.contiguous()
    _check_tensor(c, 4)
    dims, n = c.shape
    codes = torch.empty(n, dtype=torch.int32, device=c.device)
    perm = torch.empty(n, dtype=torch.int32, device=c.device)
    o = opts if opts is not None else make_opts()
    _lib.check(_lib.load().dtsort_morton_u32(c.data_ptr(), dims, n, codes.data_ptr(), perm.data_ptr(), C.byref(o),
                                             _stream(c)))
    return codes, perm


def copy_u32(dst, src):
    """dst[:] = src with the library's copy kernel (32-bit words; a measurement
    aid for the practical HBM ceiling)."""
    _check_tensor(dst, 4)
    _check_tensor(src, 4)
    if dst.numel() != src.numel():
        raise ValueError("dst and src differ in length")
    _lib.check(_lib.load().dtsort_copy_u32(dst.data_ptr(), src.data_ptr(), src.numel(), _stream(src)))
    return dst
