"""Pins of the applications' oracle (Section 6.2) against hand-worked
examples and properties that hold by definition."""
import numpy as np

from oracle import apps as A


def test_transpose_hand_example():
    # 0 -> 1, 0 -> 2, 1 -> 2, 2 -> 0, 3 -> 2, 3 -> 1
    off = np.array([0, 2, 3, 4, 6], dtype=np.uint64)
    tgt = np.array([1, 2, 2, 0, 2, 1], dtype=np.uint32)
    to, tt = A.transpose_csr(off, tgt, 4)
    # in-lists: 0 <- {2}; 1 <- {0, 3}; 2 <- {0, 1, 3}; 3 <- {}
    assert to.tolist() == [0, 1, 3, 6, 6]
    assert tt.tolist() == [2, 0, 3, 0, 1, 3]


def test_transpose_twice_is_identity_up_to_list_order():
    rs = np.random.default_rng(1)
    V = 50
    deg = rs.integers(0, 6, V)
    off = np.concatenate([[0], np.cumsum(deg)]).astype(np.uint64)
    tgt = rs.integers(0, V, int(off[-1])).astype(np.uint32)
    to, tt = A.transpose_csr(off, tgt, V)
    bo, bt = A.transpose_csr(to, tt, V)
    assert np.array_equal(bo, off)
    for u in range(V):  # the same out-lists, sorted (transposing orders each list by source)
        assert sorted(tgt[off[u]:off[u + 1]].tolist()) == bt[bo[u]:bo[u + 1]].tolist()
    fo, ft = A.transpose_csr_fast(off, tgt, V)
    assert np.array_equal(fo, to) and np.array_equal(ft, tt)


def test_morton_hand_examples():
    # 2-D: x in the even bits, y in the odd bits
    c = np.array([[1, 0, 3, 0xFFFF, 5], [0, 1, 3, 0, 6]], dtype=np.uint32)
    z = A.morton_code_u32(c)
    assert z.tolist() == [1, 2, 15, 0x55555555, 0b111001]  # x=101, y=110 -> y2x2 y1x1 y0x0 = 11 10 01
    # 3-D: bit i of x, y, z -> bits 3i, 3i + 1, 3i + 2
    c3 = np.array([[1, 0, 0, 1023], [0, 1, 0, 0], [0, 0, 1, 1023]], dtype=np.uint32)
    assert A.morton_code_u32(c3).tolist() == [1, 2, 4, 0x2DB6DB6D]


def test_morton_order_is_locality_order():
    # on a 4x4 grid the z-order visits 2x2 quadrants one after the other
    xs, ys = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
    c = np.stack([xs.ravel(), ys.ravel()]).astype(np.uint32)
    z, o = A.morton_sort(c)
    assert z.tolist() == list(range(16))
    first = {(int(c[0, i]), int(c[1, i])) for i in o[:4]}
    assert first == {(0, 0), (1, 0), (0, 1), (1, 1)}
