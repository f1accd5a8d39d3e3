"""The paper's applications (Section 6.2) through the C ABI, against the
oracle's definitions: graph transpose (CSR in, CSR out, in-neighbours in
edge-list order) and Morton order (z-values and the stable order of the
points), on synthetic stand-ins for the paper's graphs and point sets."""
import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
import workloads as W
from oracle import apps as A
from tests._dev import dev_u32, dev_u64, host_u32, host_u64, require_gpu, say

pytestmark = pytest.mark.gpu


def _transpose(off, tgt, V, **kw):
    t_off, t_tgt = dt.graph_transpose(dev_u64(off), dev_u32(tgt), V, opts=dt.make_opts(**kw))
    torch.cuda.synchronize()
    return host_u64(t_off), host_u32(t_tgt)


def test_transpose_hand_example():
    require_gpu()
    off = np.array([0, 2, 3, 4, 6], dtype=np.uint64)
    tgt = np.array([1, 2, 2, 0, 2, 1], dtype=np.uint32)
    to, tt = _transpose(off, tgt, 4)
    assert to.tolist() == [0, 1, 3, 6, 6]
    assert tt.tolist() == [2, 0, 3, 0, 1, 3]


@pytest.mark.parametrize("V,E,s_in", [(1 << 6, 500, 1.0), (1 << 12, 200_000, 1.0), (1 << 14, 1_000_003, 1.2),
                                      (1 << 16, 3_000_017, 0.6), (1 << 20, 4_000_037, 1.0)])
def test_transpose_power_law(V, E, s_in):
    require_gpu()
    say(f"transpose V={V} E={E} s_in={s_in}")
    off, tgt = W.power_law_graph(V, E, s_in=s_in, seed=V)
    off, tgt = off.numpy().astype(np.uint64), tgt.numpy().astype(np.uint32)
    to, tt = _transpose(off, tgt, V, tuned=1)
    eo, et = A.transpose_csr_fast(off, tgt, V)
    assert np.array_equal(to, eo)
    assert np.array_equal(tt, et)
    if E <= 200_000:
        do, dtt = A.transpose_csr(off, tgt, V)
        assert np.array_equal(to, do) and np.array_equal(tt, dtt)


def test_transpose_edge_cases():
    require_gpu()
    # no edges; isolated vertices at both ends; one vertex with every edge
    to, tt = _transpose(np.zeros(9, dtype=np.uint64), np.zeros(0, dtype=np.uint32), 8)
    assert to.tolist() == [0] * 9 and tt.size == 0
    V, E = 1000, 70_000
    off = np.zeros(V + 1, dtype=np.uint64)
    off[501:] = E  # vertex 500 has all the out-edges
    tgt = np.full(E, 999, dtype=np.uint32)
    tgt[::3] = 0
    to, tt = _transpose(off, tgt, V)
    eo, et = A.transpose_csr_fast(off, tgt, V)
    assert np.array_equal(to, eo) and np.array_equal(tt, et)


def test_transpose_rejects_invalid_input():
    require_gpu()
    off = np.array([0, 2, 3], dtype=np.uint64)
    with pytest.raises(dt.DTSortError):
        _transpose(off, np.array([0, 5, 1], dtype=np.uint32), 2)  # target 5 >= V
    with pytest.raises(dt.DTSortError):
        _transpose(np.array([0, 2, 1], dtype=np.uint64), np.array([0, 1], dtype=np.uint32), 2)  # decreasing


@pytest.mark.parametrize("dims,n", [(2, 1), (2, 1000), (2, 1_000_003), (3, 777), (3, 2_000_011)])
def test_morton(dims, n):
    require_gpu()
    say(f"morton dims={dims} n={n}")
    c = W.varden_points(n, dims, seed=n).numpy().astype(np.uint32)
    codes, perm = dt.morton_sort(dev_u32(c.ravel()).view(dims, n), opts=dt.make_opts(tuned=1))
    torch.cuda.synchronize()
    ez, eo = A.morton_sort(c)
    assert np.array_equal(host_u32(codes), ez)
    assert np.array_equal(host_u32(perm), eo)


def test_morton_masks_high_coordinate_bits():
    require_gpu()
    rs = np.random.default_rng(3)
    c = rs.integers(0, 2 ** 32, (3, 50_000), dtype=np.uint64).astype(np.uint32)
    codes, perm = dt.morton_sort(dev_u32(c.ravel()).view(3, 50_000))
    torch.cuda.synchronize()
    ez, eo = A.morton_sort(c & np.uint32(0x3FF))
    assert np.array_equal(host_u32(codes), ez) and np.array_equal(host_u32(perm), eo)
