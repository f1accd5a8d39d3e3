"""Multicore stable sort of the host (C++, libstdc++ parallel mode) --
TEST INFRASTRUCTURE ONLY: the benchmark's all-cores CPU baseline.

``build()`` compiles ``psort.cpp`` into ``libpsort.so`` beside it; the
functions below load it with ctypes.  The result is the definition of
Section 2.3 (non-decreasing keys, equal keys in input order), which the CPU
tests check against the one-thread numpy definition in ``oracle.sort``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "psort.cpp")
LIB = os.path.join(HERE, "libpsort.so")
_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.run(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", SRC, "-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = C.CDLL(LIB)
        lib.oracle_psort_u32.restype = C.c_int
        lib.oracle_psort_u32.argtypes = [C.c_void_p, C.c_size_t, C.c_int]
        lib.oracle_psort_pairs_u64.restype = C.c_int
        lib.oracle_psort_pairs_u64.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _lib = lib
    return _lib


def sort_u32_(keys: np.ndarray, threads: int = 0) -> int:
    """Sorts a contiguous uint32 array in place; returns the threads used."""
    assert keys.dtype == np.uint32 and keys.flags.c_contiguous
    return _load().oracle_psort_u32(keys.ctypes.data, keys.size, threads)


def sort_pairs_u64_(keys: np.ndarray, values: np.ndarray, threads: int = 0) -> int:
    """Stable sort of (key, value) records by key, in place; returns the threads used."""
    assert keys.dtype == np.uint64 and values.dtype == np.uint64 and keys.size == values.size
    assert keys.flags.c_contiguous and values.flags.c_contiguous
    return _load().oracle_psort_pairs_u64(keys.ctypes.data, values.ctypes.data, keys.size, threads)
