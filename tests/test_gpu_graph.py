"""Graph form: the device-driven schedule recorded once into a HIP graph and
replayed (dtsort_opts.graph = 1), and the scatter tile shapes.

The output is the unique stable order whatever the schedule, so every replay
must equal the CPU oracle bit for bit.  The recursion shape is fixed by the
seed (Appendix A), so the counters the graph leaves behind must equal those
of the eager level loop on the same input.
"""
import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
import workloads as W
from oracle import sort as S
from tests._dev import dev_u32, dev_u64, host_u32, host_u64, require_gpu, say

pytestmark = pytest.mark.gpu

SHAPE_FIELDS = ("tasks", "records_distributed", "heavy_keys", "heavy_records", "merges", "records_merged",
                "leaf_sorts", "records_leaf_sorted", "records_copied", "overflow_records")


def _shape(st):
    return {f: getattr(st, f) for f in SHAPE_FIELDS}


def _segmented_case(seed, n=2_000_000, n_seg=257):
    c = W.make_config("segmented_u32", n=n, n_seg=n_seg, seed=seed)
    k = c["keys"].numpy().astype(np.uint32)
    off = c["offsets"].numpy().astype(np.uint64)
    # empty and one-record segments in front
    off = np.concatenate([[0, 0, 1, 1], off[1:] + 1]).astype(np.uint64)
    k = np.concatenate([[4242], k]).astype(np.uint32)
    return k, off


@pytest.mark.parametrize("vals", [False, True])
def test_graph_segmented_replays(vals):
    """One recorded graph, replayed on three different inputs of the same
    shape placed in the same buffers, with eager work and synchronisations
    between the replays; every replay is checked."""
    require_gpu()
    k0, off = _segmented_case(11)
    dk = dev_u32(k0)
    dv = dev_u32(np.arange(k0.size, dtype=np.uint32))
    do = dev_u64(off)
    for rep in range(3):
        say(f"graph segmented vals={vals} replay {rep}")
        rs = np.random.default_rng(100 + rep)
        if rep == 0:
            k = k0
        elif rep == 1:
            k = rs.integers(0, 2 ** 32, k0.size, dtype=np.uint64).astype(np.uint32)
        else:
            k = (rs.zipf(1.3, k0.size).astype(np.uint64) * np.uint64(2654435761) & np.uint64(0xFFFFFFFF)).astype(
                np.uint32)
        v = np.arange(k.size, dtype=np.uint32)
        dk.copy_(dev_u32(k))
        dv.copy_(dev_u32(v))
        torch.cuda.synchronize()
        o = dt.make_opts(graph=1)
        if vals:
            dt.sort_segmented(dk, do, dv, opts=o)
        else:
            dt.sort_segmented(dk, do, opts=o)
        torch.cuda.synchronize()
        ek, ev = S.segmented_sort(k, off, v)
        assert np.array_equal(host_u32(dk), ek)
        if vals:
            assert np.array_equal(host_u32(dv), ev)
        # unrelated eager work between replays
        x = torch.randint(0, 1 << 30, (100_000,), dtype=torch.int32, device="cuda")
        dt.sort_u32(x)
        torch.cuda.synchronize()


def test_graph_segmented_stats_equal_eager():
    require_gpu()
    k, off = _segmented_case(5)
    do = dev_u64(off)
    st_e, st_g = dt.Stats(), dt.Stats()
    de = dev_u32(k)
    dt.sort_segmented(de, do, opts=dt.make_opts(stats=st_e, ordered_ranks=1))
    dg = dev_u32(k)
    dt.sort_segmented(dg, do, opts=dt.make_opts(stats=st_g, graph=1, ordered_ranks=1))
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(de), host_u32(dg))
    assert _shape(st_e) == _shape(st_g)
    assert st_e.levels == st_g.levels


def test_graph_bad_offsets_reported_with_stats():
    require_gpu()
    k = dev_u32(np.arange(100, dtype=np.uint32))
    bad = dev_u64(np.array([0, 50, 40, 100], np.uint64))
    with pytest.raises(dt.DTSortError):
        dt.sort_segmented(k, bad, opts=dt.make_opts(graph=1, stats=dt.Stats()))
    torch.cuda.synchronize()


@pytest.mark.parametrize("kind", ["uniform", "zipf", "equal", "bexp"])
def test_graph_whole_array(kind):
    require_gpu()
    say(f"graph whole array {kind}")
    rs = np.random.default_rng(7)
    n = 1_500_000
    if kind == "uniform":
        k = rs.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    elif kind == "zipf":
        k = (rs.zipf(1.1, n).astype(np.uint64) * np.uint64(0x9E3779B1) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    elif kind == "equal":
        k = np.full(n, 99, np.uint32)
    else:
        b = np.minimum(rs.geometric(0.1, n), 32)
        low = rs.integers(0, 2 ** 32, n, dtype=np.uint64)
        lead = np.left_shift(np.uint64(1), (b - 1).astype(np.uint64))
        k = (lead | (low & (lead - np.uint64(1)))).astype(np.uint32)
    # a seed of its own per input: a graph is cached per (pointers, sizes,
    # options), and this test compares a first recording's replay with the
    # eager schedule on the same input
    sd = 3 + ["uniform", "zipf", "equal", "bexp"].index(kind)
    st_e, st_g = dt.Stats(), dt.Stats()
    de, dg = dev_u32(k), dev_u32(k)
    dt.sort_u32(de, dt.make_opts(stats=st_e, seed=sd, ordered_ranks=1))
    for rep in range(2):  # the first call records (sorting eagerly), the second replays
        dg.copy_(dev_u32(k))
        dt.sort_u32(dg, dt.make_opts(stats=st_g, seed=sd, graph=1, ordered_ranks=1))
        torch.cuda.synchronize()
        ref = S.stable_sort_keys(k)
        assert np.array_equal(host_u32(de), ref)
        assert np.array_equal(host_u32(dg), ref)
        assert _shape(st_e) == _shape(st_g), f"call {rep}"


def test_graph_pairs_u64_heavy():
    """64-bit pairs with heavy keys at several levels: merges and value spills
    run inside the graph."""
    require_gpu()
    rs = np.random.default_rng(12)
    n = 1_200_000
    b = np.minimum(rs.geometric(0.1, n), 64)
    low = rs.integers(0, 2 ** 63, n, dtype=np.uint64)
    lead = np.left_shift(np.uint64(1), (b - 1).astype(np.uint64))
    k = lead | (low & (lead - np.uint64(1)))
    v = np.arange(n, dtype=np.uint64)
    ek, ev = S.stable_sort_pairs(k, v)
    for rep in range(2):
        dk, dv = dev_u64(k), dev_u64(v)
        st = dt.Stats()
        dt.sort_pairs_u64(dk, dv, dt.make_opts(graph=1, stats=st if rep else None))
        torch.cuda.synchronize()
        assert np.array_equal(host_u64(dk), ek)
        assert np.array_equal(host_u64(dv), ev)
    assert st.merges > 0


def test_graph_rejects_learned_and_profile():
    require_gpu()
    x = dev_u32(np.arange(1000, dtype=np.uint32)[::-1].copy())
    with pytest.raises(dt.DTSortError):
        dt.sort_u32(x, dt.make_opts(graph=1, mode=dt.MODE_LEARNED))
    with pytest.raises(dt.DTSortError):
        dt.sort_u32(x, dt.make_opts(graph=1, profile=1, stats=dt.Stats()))


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6])
def test_tile_shapes(tile):
    require_gpu()
    say(f"tile shape {tile}")
    rs = np.random.default_rng(tile)
    n = 700_001
    k = (rs.zipf(1.2, n).astype(np.uint64) * np.uint64(0x9E3779B1) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    d = dev_u32(k)
    dt.sort_u32(d, dt.make_opts(tile_shape=tile, digit_bits=8))
    k64 = rs.integers(0, 2 ** 40, n, dtype=np.uint64)
    v64 = np.arange(n, dtype=np.uint64)
    dk, dv = dev_u64(k64), dev_u64(v64)
    dt.sort_pairs_u64(dk, dv, dt.make_opts(tile_shape=tile, digit_bits=8))
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(d), S.stable_sort_keys(k))
    ek, ev = S.stable_sort_pairs(k64, v64)
    assert np.array_equal(host_u64(dk), ek)
    assert np.array_equal(host_u64(dv), ev)


def test_tuned_table_path():
    """tuned=1 takes the table's parameters; the output stays the oracle's."""
    require_gpu()
    rs = np.random.default_rng(21)
    k = rs.integers(0, 2 ** 32, 1_000_003, dtype=np.uint64).astype(np.uint32)
    d = dev_u32(k)
    dt.sort_u32(d, dt.make_opts(tuned=1))
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(d), S.stable_sort_keys(k))


@pytest.mark.parametrize("kind", ["uniform", "zipf", "bexp_pairs", "segmented"])
def test_graph_finishing_step(kind, monkeypatch):
    """With one recorded level and a small base-case cutoff, most buckets are
    left to the finishing step (a whole-task LSD sort per workgroup); the
    output must still be the oracle's."""
    require_gpu()
    say(f"graph finishing step {kind}")
    monkeypatch.setenv("DTSORT_GRAPH_LEVELS", "1")
    rs = np.random.default_rng(31)
    n = 400_000
    o = dt.make_opts(graph=1, lds_cutoff=300, seed=5)
    if kind in ("uniform", "zipf"):
        if kind == "uniform":
            k = rs.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
        else:
            k = (rs.zipf(1.3, n).astype(np.uint64) * np.uint64(0x9E3779B1) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        d = dev_u32(k)
        dt.sort_u32(d, o)
        torch.cuda.synchronize()
        assert np.array_equal(host_u32(d), S.stable_sort_keys(k))
    elif kind == "bexp_pairs":
        b = np.minimum(rs.geometric(0.1, n), 64)
        low = rs.integers(0, 2 ** 63, n, dtype=np.uint64)
        lead = np.left_shift(np.uint64(1), (b - 1).astype(np.uint64))
        k = lead | (low & (lead - np.uint64(1)))
        v = np.arange(n, dtype=np.uint64)
        dk, dv = dev_u64(k), dev_u64(v)
        dt.sort_pairs_u64(dk, dv, o)
        torch.cuda.synchronize()
        ek, ev = S.stable_sort_pairs(k, v)
        assert np.array_equal(host_u64(dk), ek)
        assert np.array_equal(host_u64(dv), ev)
    else:
        k, off = _segmented_case(3, n=n, n_seg=61)
        v = np.arange(k.size, dtype=np.uint32)
        dk, dv, do = dev_u32(k), dev_u32(v), dev_u64(off)
        dt.sort_segmented(dk, do, dv, opts=o)
        torch.cuda.synchronize()
        ek, ev = S.segmented_sort(k, off, v)
        assert np.array_equal(host_u32(dk), ek)
        assert np.array_equal(host_u32(dv), ev)


@pytest.mark.parametrize("graph", [0, 1])
def test_tile_shape_6_other_layouts(graph):
    """Tile 6 is 1024 x 16 only for bare 32-bit keys with unordered ranks;
    ordered ranks, 64-bit keys and the batched form take 1024 x 8 (x 4)."""
    require_gpu()
    say(f"tile shape 6 layouts graph={graph}")
    rs = np.random.default_rng(66)
    n = 600_007
    k = rs.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    k[rs.integers(0, n, n // 4)] = 12345  # a heavy key
    d = dev_u32(k)
    dt.sort_u32(d, dt.make_opts(tile_shape=6, digit_bits=8, ordered_ranks=1, graph=graph))
    k64 = rs.integers(0, 2 ** 64, n, dtype=np.uint64)
    d64 = dev_u64(k64)
    dt.sort_u64(d64, dt.make_opts(tile_shape=6, digit_bits=8, graph=graph))
    off = np.array([0, 1000, 1000, 250_000, n], dtype=np.uint64)
    ks = rs.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    ds = dev_u32(ks)
    dt.sort_segmented(ds, torch.from_numpy(off.view(np.int64)).cuda(), opts=dt.make_opts(tile_shape=6, graph=graph))
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(d), S.stable_sort_keys(k))
    assert np.array_equal(host_u64(d64), S.stable_sort_keys(k64))
    ek, _ = S.segmented_sort(ks, off)
    assert np.array_equal(host_u32(ds), ek)
