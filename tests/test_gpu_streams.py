"""Calls on different streams run concurrently: every stream has its own
context (buffers, events, lock), so host threads sorting on their own
streams do not wait for each other.  Results must stay bit-exact against the
oracle's stable sort (Section 2.3), also when more streams than the library
keeps contexts for take contexts over, and in the graph form."""
import threading

import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
from oracle import sort as S
from tests._dev import dev_u32, dev_u64, host_u32, host_u64, require_gpu, say
from tests._seeds import seed_of

pytestmark = pytest.mark.gpu


def _run_threads(fns):
    errs = []

    def wrap(f):
        try:
            f()
        except Exception as e:  # noqa: BLE001 - re-raised in the main thread
            errs.append(e)

    th = [threading.Thread(target=wrap, args=(f,)) for f in fns]
    for t in th:
        t.start()
    for t in th:
        t.join()
    if errs:
        raise errs[0]


@pytest.mark.parametrize("graph", [0, 1])
def test_threads_on_own_streams(graph):
    require_gpu()
    say(f"four threads, four streams, graph={graph}")
    rs = np.random.default_rng(seed_of("streams", graph))
    sizes = [3_000_001, 1_500_007, 700_001, 2_000_003]
    inputs = [rs.integers(0, 2 ** 32, m, dtype=np.uint64).astype(np.uint32) for m in sizes]
    inputs[1] = ((rs.zipf(1.2, sizes[1]).astype(np.uint64) * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)).astype(
        np.uint32)
    streams = [torch.cuda.Stream() for _ in sizes]
    results = [None] * len(sizes)

    def job(i):
        def f():
            with torch.cuda.stream(streams[i]):
                src = dev_u32(inputs[i])
                for _ in range(3):
                    x = src.clone()
                    dt.sort_u32(x, dt.make_opts(graph=graph))
                streams[i].synchronize()
                results[i] = host_u32(x)
        return f

    _run_threads([job(i) for i in range(len(sizes))])
    for i, k in enumerate(inputs):
        assert np.array_equal(results[i], S.stable_sort_keys(k)), i


def test_mixed_entry_points_concurrently():
    """64-bit pairs (stability visible through values = index) and a segmented
    sort on two streams at once."""
    require_gpu()
    say("pairs and segmented on two streams")
    rs = np.random.default_rng(seed_of("streams", "mixed"))
    n = 2_000_003
    k64 = rs.integers(0, 5000, n).astype(np.uint64)
    v64 = np.arange(n, dtype=np.uint64)
    k32 = rs.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    off = np.concatenate([[0], np.sort(rs.integers(0, n + 1, 99)), [n]]).astype(np.uint64)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    out = {}

    def pairs():
        with torch.cuda.stream(s1):
            dk, dv = dev_u64(k64), dev_u64(v64)
            dt.sort_pairs_u64(dk, dv)
            s1.synchronize()
            out["pairs"] = (host_u64(dk), host_u64(dv))

    def seg():
        with torch.cuda.stream(s2):
            dk = dev_u32(k32)
            dt.sort_segmented(dk, dev_u64(off))
            s2.synchronize()
            out["seg"] = host_u32(dk)

    _run_threads([pairs, seg])
    ek, ev = S.stable_sort_pairs(k64, v64)
    assert np.array_equal(out["pairs"][0], ek) and np.array_equal(out["pairs"][1], ev)
    assert np.array_equal(out["seg"], S.segmented_sort(k32, off)[0])


def test_more_streams_than_contexts():
    """Twelve streams one after another, then the first again: contexts are
    taken over least recently used first, each stream's sort still exact."""
    require_gpu()
    say("twelve streams in turn")
    rs = np.random.default_rng(seed_of("streams", "many"))
    streams = [torch.cuda.Stream() for _ in range(12)]
    for i, st in enumerate(streams + streams[:1]):
        k = rs.integers(0, 2 ** 32, 400_000 + 3 * i, dtype=np.uint64).astype(np.uint32)
        with torch.cuda.stream(st):
            d = dev_u32(k)
            dt.sort_u32(d)
            st.synchronize()
            assert np.array_equal(host_u32(d), np.sort(k)), i
    # releasing every stream's cache, then sorting again, allocates afresh
    torch.cuda.synchronize()
    import paper_2401_00710_amd._lib as L
    L.load().dtsort_release()
    k = rs.integers(0, 2 ** 32, 123457, dtype=np.uint64).astype(np.uint32)
    with torch.cuda.stream(streams[5]):
        d = dev_u32(k)
        dt.sort_u32(d)
        streams[5].synchronize()
    assert np.array_equal(host_u32(d), np.sort(k))
