"""Definition of the problem the method solves (Section 2.3, integer sort).

Integer sort reorders n records by an integer key in [r] so that keys are
non-decreasing; a stable sort keeps equal keys in their input order
(Section 2.3).  The method (Alg. 2) is stable (Section 3), so its output is
the unique stable ascending order, which this module writes out directly.

TEST INFRASTRUCTURE ONLY -- see the package docstring.
"""
from __future__ import annotations

import numpy as np

_M = (1 << 64) - 1


def stable_sort_keys(keys: np.ndarray) -> np.ndarray:
    """Keys in non-decreasing order (keys-only: the sorted multiset)."""
    return np.sort(keys, kind="stable")


def stable_order(keys: np.ndarray) -> np.ndarray:
    """Permutation listing record indices in stable ascending key order."""
    return np.argsort(keys, kind="stable")


def stable_sort_pairs(keys: np.ndarray, values: np.ndarray):
    """(keys, values) records stably ordered by key."""
    o = stable_order(keys)
    return keys[o], values[o]


def stable_rank_bruteforce(keys) -> list[int]:
    """rank(i) = #{j : k_j < k_i} + #{j < i : k_j = k_i}, in O(n^2) pure Python.

    This is the position record i takes in the stable ascending order; it is
    an independent second oracle for small n.
    """
    ks = [int(k) for k in keys]
    n = len(ks)
    out = []
    for i in range(n):
        less = sum(1 for j in range(n) if ks[j] < ks[i])
        tie = sum(1 for j in range(i) if ks[j] == ks[i])
        out.append(less + tie)
    return out


def apply_ranks(items, ranks):
    out = [None] * len(items)
    for i, r in enumerate(ranks):
        out[r] = items[i]
    return out


def segmented_sort(keys: np.ndarray, offsets: np.ndarray, values: np.ndarray | None = None):
    """Each instance [offsets[s], offsets[s+1]) stably sorted on its own."""
    k = keys.copy()
    v = None if values is None else values.copy()
    for s in range(len(offsets) - 1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        o = np.argsort(keys[a:b], kind="stable")
        k[a:b] = keys[a:b][o]
        if v is not None:
            v[a:b] = values[a:b][o]
    return k, v


# ------------------------------------------------------------------ invariants
def is_nondecreasing(keys: np.ndarray) -> bool:
    return bool(np.all(keys[1:] >= keys[:-1])) if keys.size > 1 else True


def _mix(x: np.ndarray) -> np.ndarray:
    z = x.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def multiset_hash(keys: np.ndarray, values: np.ndarray | None = None) -> tuple[int, int, int]:
    """Order-independent digest: (count, sum mod 2^64, xor) of a 64-bit mix of
    each record.  Equal multisets give equal digests; a changed, dropped or
    duplicated record changes the sum with probability about 1 - 2^-64."""
    h = _mix(keys.astype(np.uint64))
    if values is not None:
        with np.errstate(over="ignore"):
            h = _mix(h ^ (_mix(values.astype(np.uint64)) * np.uint64(3)))
    with np.errstate(over="ignore"):
        s = int(np.sum(h, dtype=np.uint64))
    x = int(np.bitwise_xor.reduce(h)) if h.size else 0
    return (int(keys.size), s, x)


def is_stable_by_index(keys_out: np.ndarray, idx_out: np.ndarray) -> bool:
    """With values = original index: within equal keys the index increases."""
    if keys_out.size < 2:
        return True
    eq = keys_out[1:] == keys_out[:-1]
    return bool(np.all(idx_out[1:][eq] > idx_out[:-1][eq]))


def order_statistic(keys: np.ndarray, q: int):
    """The q-th smallest key (0-based) without sorting: the unique key v with
    #{k < v} <= q < #{k <= v}.  Found by bisection over counts (one pass each)."""
    lo, hi = int(keys.min()), int(keys.max())
    kt = keys.dtype.type
    while lo < hi:
        mid = lo + (hi - lo) // 2
        if int(np.count_nonzero(keys <= kt(mid))) > q:
            hi = mid
        else:
            lo = mid + 1
    return lo
