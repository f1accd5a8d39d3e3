"""ctypes binding of libdtsort.so (the C ABI in include/dtsort.h).

Argument marshalling only: every step of the sort runs in the library's HIP
kernels.  There is no fallback: if the library is missing, loading fails.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdtsort.so")

OK, EINVAL, ENOMEM, EWORKSPACE, EHIP, EINTERNAL = 0, -1, -2, -3, -4, -5
MODE_SAMPLING, MODE_PLAIN, MODE_LEARNED = 0, 1, 2
MERGE_GATHER, MERGE_PLMERGE, MERGE_INPLACE, MERGE_NONE, MERGE_SPLIT = 0, 1, 2, 3, 4


class Stats(C.Structure):
    _fields_ = [
        ("levels", C.c_uint64),
        ("tasks", C.c_uint64),
        ("records_distributed", C.c_uint64),
        ("heavy_keys", C.c_uint64),
        ("heavy_records", C.c_uint64),
        ("merges", C.c_uint64),
        ("records_merged", C.c_uint64),
        ("leaf_sorts", C.c_uint64),
        ("records_leaf_sorted", C.c_uint64),
        ("records_copied", C.c_uint64),
        ("overflow_records", C.c_uint64),
        ("learned_used", C.c_int32),
        ("learned_balance", C.c_float),
        ("sampling_balance", C.c_float),
        ("learned_final_loss", C.c_float),
        ("learned_ms", C.c_double),
        ("kernel_ms", C.c_double * 8),
        ("kernel_bytes", C.c_double * 8),
        ("kernel_launches", C.c_uint32 * 8),
        ("records_pair_merged", C.c_uint64),
        ("learned_trained", C.c_int32),
        ("learned_cost", C.c_float),
        ("sampling_cost", C.c_float),
        ("ideal_cost", C.c_float),
    ]

    KINDS = ("plan", "hist", "scan", "scatter", "children", "leaf", "copy", "merge")

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if k.startswith("kernel_") else v
        return d


class Opts(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64),
        ("key_bits", C.c_int32),
        ("mode", C.c_int32),
        ("digit_bits", C.c_int32),
        ("lds_cutoff", C.c_int32),
        ("tuned", C.c_int32),
        ("learned_steps", C.c_int32),
        ("learned_batch", C.c_int32),
        ("learned_lr", C.c_float),
        ("profile", C.c_int32),
        ("tile_shape", C.c_int32),
        ("graph", C.c_int32),
        ("ordered_ranks", C.c_int32),
        ("learned_judge", C.c_int32),
        ("merge_variant", C.c_int32),
        ("digit_bits_below", C.c_int32),
        ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_size_t),
        ("stats", C.POINTER(Stats)),
    ]


_P = C.c_void_p
_Z = C.c_size_t
_I = C.c_int
_SIGS = {
    "dtsort_default_opts": (None, [C.POINTER(Opts)]),
    "dtsort_workspace_bytes": (_Z, [_I, _I, _Z]),
    "dtsort_u32": (_I, [_P, _Z, C.POINTER(Opts), _P]),
    "dtsort_u64": (_I, [_P, _Z, C.POINTER(Opts), _P]),
    "dtsort_pairs_u64": (_I, [_P, _P, _Z, C.POINTER(Opts), _P]),
    "dtsort_pairs_u32": (_I, [_P, _P, _Z, C.POINTER(Opts), _P]),
    "dtsort_segmented": (_I, [_P, _P, _Z, _P, _Z, C.POINTER(Opts), _P]),
    "dtsort_segmented_noalloc": (_I, [_P, _P, _Z, _P, _Z, C.POINTER(Opts), _P]),
    "dtsort_step_plan_u32": (_I, [_P, _Z, _I, _I, C.POINTER(Opts), _P, _P, _P, _P]),
    "dtsort_step_plan_u64": (_I, [_P, _Z, _I, _I, C.POINTER(Opts), _P, _P, _P, _P]),
    "dtsort_step_distribute_u32": (_I, [_P, _P, _Z, _I, C.POINTER(Opts), _P, _P, _P, _P, _P, _P, _P]),
    "dtsort_step_distribute_u64": (_I, [_P, _P, _Z, _I, C.POINTER(Opts), _P, _P, _P, _P, _P, _P, _P]),
    "dtsort_step_leaf_u32": (_I, [_P, _P, _P, _Z, _I, _P, _P, _P]),
    "dtsort_step_leaf_u64": (_I, [_P, _P, _P, _Z, _I, _P, _P, _P]),
    "dtsort_step_dtmerge_u64": (_I, [_P, _P, _Z, _P, _P, _Z, _P, _P, _P, _P]),
    "dtsort_mlp_loss_grad": (_I, [_P, _P, _P, _Z, _P, _P, _P]),
    "dtsort_mlp_forward": (_I, [_P, _P, _Z, _P, _P]),
    "dtsort_mlp_train_u64": (_I, [_P, _Z, C.c_uint64, _I, _I, C.c_float, _P, _P, _P]),
    "dtsort_graph_transpose": (_I, [_P, _P, C.c_uint32, _Z, _P, _P, C.POINTER(Opts), _P]),
    "dtsort_morton_u32": (_I, [_P, _I, _Z, _P, _P, C.POINTER(Opts), _P]),
    "dtsort_copy_u32": (_I, [_P, _P, _Z, _P]),
    "dtsort_release": (None, []),
    "dtsort_last_error": (C.c_char_p, []),
    "dtsort_strerror": (C.c_char_p, [_I]),
}

_lib = None


def load(path: str | None = None):
    """Load the library (once).  Raises OSError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError(f"libdtsort.so not found at {p}: build it with "
                      f"`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    return list(_SIGS)


class DTSortError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dtsort error {status}: {msg}")
        self.status = status


def check(status: int):
    if status != OK:
        lib = load()
        msg = lib.dtsort_last_error().decode() or lib.dtsort_strerror(status).decode()
        raise DTSortError(status, msg)
