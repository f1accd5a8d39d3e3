"""Heavy-key lookup in the distribution kernels (GetBucketId, Alg. 2).

The histogram and scatter kernels of digits of at most 8 bits find a key's
heavy bucket through a small hash table of the task's heavy keys (at most
four keys per slot); a task whose heavy keys overflow a slot falls back to a
binary search among its zone's heavy keys.  These inputs make many heavy keys
share one slot, so that both the full slot and the overflow path carry a
large share of the records, and compare the result with the oracle's stable
sort element by element.
"""
import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
from oracle import sort as S
from tests._dev import dev_u32, dev_u64, host_u32, host_u64, require_gpu, say

pytestmark = pytest.mark.gpu

N = 1 << 20


def _slot(x: np.ndarray) -> np.ndarray:
    """The kernels' slot of a 32-bit value (multiplicative hashing, 9 bits)."""
    return ((x.astype(np.uint64) * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)) >> np.uint64(23)


def _colliding_u32(rs, count: int) -> np.ndarray:
    """`count` distinct 32-bit values that share one slot."""
    x = np.unique(rs.integers(0, 2 ** 32, 1 << 22, dtype=np.uint64))
    s = _slot(x)
    target = s[0]
    c = x[s == target]
    assert c.size >= count
    return rs.permutation(c)[:count].astype(np.uint32)


def _input(rs, heavy: np.ndarray, dtype) -> np.ndarray:
    """Each heavy value takes 4 % of the records; the rest are uniform."""
    per = N // 25
    parts = [np.repeat(heavy.astype(dtype), per)]
    rest = N - per * heavy.size
    hi = 2 ** 32 if dtype == np.uint32 else 2 ** 63
    parts.append(rs.integers(0, hi, rest, dtype=np.uint64).astype(dtype))
    return rs.permutation(np.concatenate(parts))


@pytest.mark.parametrize("count", [1, 4, 5, 12])
@pytest.mark.parametrize("digit", [8, 0])
def test_heavy_slot_u32(count, digit):
    require_gpu()
    say(f"heavy slot u32 count={count} digit={digit}")
    rs = np.random.default_rng(100 + count)
    k = _input(rs, _colliding_u32(rs, count), np.uint32)
    d = dev_u32(k)
    st = dt.Stats()
    dt.sort_u32(d, dt.make_opts(stats=st, digit_bits=digit, tuned=1))
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(d), S.stable_sort_keys(k))
    assert st.heavy_keys >= count


@pytest.mark.parametrize("count", [4, 6])
def test_heavy_slot_pairs_u64(count):
    require_gpu()
    say(f"heavy slot pairs u64 count={count}")
    rs = np.random.default_rng(200 + count)
    lo = _colliding_u32(rs, count).astype(np.uint64)
    hi = rs.integers(0, 2 ** 31, count, dtype=np.uint64)
    heavy = (hi << np.uint64(32)) | (lo ^ hi)  # the folded 32 bits are `lo`
    k = _input(rs, heavy, np.uint64)
    v = np.arange(N, dtype=np.uint64)
    dk, dv = dev_u64(k), dev_u64(v)
    st = dt.Stats()
    dt.sort_pairs_u64(dk, dv, dt.make_opts(stats=st, digit_bits=8, tuned=1))
    torch.cuda.synchronize()
    ek, ev = S.stable_sort_pairs(k, v)
    assert np.array_equal(host_u64(dk), ek)
    assert np.array_equal(host_u64(dv), ev)
    assert st.heavy_keys >= count
