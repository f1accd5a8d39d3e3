"""Paired leaves (32-bit keys without values): a child bucket of cutoff < c <=
2 * cutoff records is sorted as two half leaves into the buffer other than
its target, and the sorted halves are merged into the target.

The output must stay the oracle's stable order; the recursion shape must be
the oracle's Alg. 2 run with the base case of child subproblems raised to
twice the cutoff (the base case is any stable sort, Section 3.5).
"""
import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
from oracle import dtsort_ref as R
from oracle import sort as S
from tests._dev import dev_u32, dev_u64, host_u32, require_gpu, say

pytestmark = pytest.mark.gpu


def _run(k, graph=0, **kw):
    d = dev_u32(k)
    st = dt.Stats()
    dt.sort_u32(d, dt.make_opts(stats=st, graph=graph, **kw))
    torch.cuda.synchronize()
    return host_u32(d), st


@pytest.mark.parametrize("graph", [0, 1])
def test_pairs_shape_matches_oracle(graph):
    """Four zones of ~15000 keys with a cutoff of 10000: every child is a pair."""
    require_gpu()
    say(f"pairs shape graph={graph}")
    rs = np.random.default_rng(12)
    k = rs.integers(0, 2 ** 32, 60000, dtype=np.uint64).astype(np.uint32)
    got, st = _run(k, graph=graph, digit_bits=2, lds_cutoff=10000)
    ost = R.Stats()
    ok, _ = R.dtsort(k, None, R.Config(seed=0, key_bytes=4, gamma=2, cutoff=10000, pair_leaves=True), stats=ost)
    assert np.array_equal(got, ok)
    assert st.levels == ost.levels == 1
    assert st.tasks == ost.tasks
    assert st.records_leaf_sorted == ost.base_sorted == k.size
    assert st.leaf_sorts == 8  # two halves per zone


@pytest.mark.parametrize("graph", [0, 1])
def test_pairs_at_merge_capacity(graph):
    """Two buckets of exactly 32768 keys (the largest pair) under the default
    cutoff: halves of 16384, the largest leaf class."""
    require_gpu()
    say(f"pairs at capacity graph={graph}")
    rs = np.random.default_rng(3)
    lo = rs.integers(0, 2 ** 31, 32768, dtype=np.uint64)
    hi = rs.integers(2 ** 31, 2 ** 32, 32768, dtype=np.uint64)
    k = rs.permutation(np.concatenate([lo, hi])).astype(np.uint32)
    got, st = _run(k, graph=graph, digit_bits=1)
    assert np.array_equal(got, S.stable_sort_keys(k))
    assert st.levels == 1 and st.leaf_sorts == 4 and st.records_leaf_sorted == k.size


@pytest.mark.parametrize("kind", ["dups", "zipf", "sorted", "reversed"])
def test_pairs_key_patterns(kind):
    """Many equal keys across the two halves, heavy keys and presorted runs."""
    require_gpu()
    say(f"pairs pattern {kind}")
    rs = np.random.default_rng(21)
    n = 200_000
    if kind == "dups":
        k = (rs.integers(0, 3000, n, dtype=np.uint64) * np.uint64(1048573)).astype(np.uint32)
    elif kind == "zipf":
        k = (rs.zipf(1.2, n).astype(np.uint64) * np.uint64(0x9E3779B1) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    elif kind == "sorted":
        k = np.sort(rs.integers(0, 2 ** 32, n, dtype=np.uint64)).astype(np.uint32)
    else:
        k = np.sort(rs.integers(0, 2 ** 32, n, dtype=np.uint64))[::-1].astype(np.uint32)
    for graph in (0, 1):
        got, st = _run(k, graph=graph, digit_bits=4, lds_cutoff=9000)
        assert np.array_equal(got, S.stable_sort_keys(k)), f"graph={graph}"


@pytest.mark.parametrize("graph", [0, 1])
def test_pairs_segmented(graph):
    """Segments of 1500-3000 keys with a cutoff of 1500 are paired at seeding;
    larger ones pair their children."""
    require_gpu()
    say(f"pairs segmented graph={graph}")
    rs = np.random.default_rng(8)
    sizes = rs.integers(1, 3001, 400)
    sizes[:5] = [0, 1, 1500, 1501, 3000]
    sizes[5:15] = 40000
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    k = rs.integers(0, 2 ** 32, int(off[-1]), dtype=np.uint64).astype(np.uint32)
    d = dev_u32(k)
    do = dev_u64(off)
    st = dt.Stats()
    dt.sort_segmented(d, do, opts=dt.make_opts(lds_cutoff=1500, graph=graph, stats=st))
    torch.cuda.synchronize()
    ek, _ = S.segmented_sort(k, off)
    assert np.array_equal(host_u32(d), ek)
    assert st.records_leaf_sorted > 0
