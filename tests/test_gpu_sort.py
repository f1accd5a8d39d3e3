"""End-to-end parity of the HIP sort against the CPU oracle (bit-exact).

The method's output is the unique stable ascending order (Section 2.3; the
method is stable, Section 3), so every result must equal the oracle's stable
sort exactly.  Where the recursion shape is fixed by the seed (Appendix A),
the device statistics must also equal the oracle's run of Alg. 2.
"""
import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
import workloads as W
from oracle import dtsort_ref as R
from oracle import sort as S
from tests._dev import dev_u32, dev_u64, host_u32, host_u64, require_gpu, say
from tests._seeds import seed_of

pytestmark = pytest.mark.gpu


def _sort32(keys, **kw):
    d = dev_u32(keys)
    st = dt.Stats()
    dt.sort_u32(d, dt.make_opts(stats=st, **kw))
    torch.cuda.synchronize()
    return host_u32(d), st


def _sort64(keys, **kw):
    d = dev_u64(keys)
    st = dt.Stats()
    dt.sort_u64(d, dt.make_opts(stats=st, **kw))
    torch.cuda.synchronize()
    return host_u64(d), st


def _pairs64(keys, vals, **kw):
    dk, dv = dev_u64(keys), dev_u64(vals)
    st = dt.Stats()
    dt.sort_pairs_u64(dk, dv, dt.make_opts(stats=st, **kw))
    torch.cuda.synchronize()
    return host_u64(dk), host_u64(dv), st


def test_uniform_u32_2p20_config():
    require_gpu()
    say("uniform u32 2^20 seed 0")
    k = W.make_config("uniform_u32_2p20", seed=0)["keys"].numpy().astype(np.uint32)
    got, st = _sort32(k)
    assert np.array_equal(got, S.stable_sort_keys(k))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 100, 2047, 2048, 2049, 8192, 16383, 16384, 16385, 16386, 50000,
                               65536 + 1, 300007])
def test_sizes_u32(n):
    require_gpu()
    say(f"sizes u32 n={n}")
    rs = np.random.default_rng(n)
    k = rs.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    got, _ = _sort32(k)
    assert np.array_equal(got, np.sort(k))


DISTS = ["uniform", "zipf", "equal", "two", "exp", "bexp", "max", "small_range"]


def _keys(kind, n, wide, rs):
    if kind == "uniform":
        k = rs.integers(0, 2 ** 64 if wide else 2 ** 32, n, dtype=np.uint64)
    elif kind == "zipf":
        k = (rs.zipf(1.2, n).astype(np.uint64) * np.uint64(0x9E3779B1)) & np.uint64((1 << (64 if wide else 32)) - 1)
    elif kind == "equal":
        k = np.full(n, 777, np.uint64)
    elif kind == "two":
        k = rs.choice(np.array([3, 2 ** 31 + 5], np.uint64), n)
    elif kind == "exp":
        k = rs.exponential(1e5, n).astype(np.uint64)
    elif kind == "bexp":
        b = np.minimum(rs.geometric(0.1, n), 64 if wide else 32)
        low = rs.integers(0, 2 ** 63, n, dtype=np.uint64)
        lead = np.left_shift(np.uint64(1), (b - 1).astype(np.uint64))
        k = lead | (low & (lead - np.uint64(1)))
    elif kind == "max":
        k = np.full(n, 2 ** 64 - 1 if wide else 2 ** 32 - 1, np.uint64)
        k[::7] = 0
    elif kind == "small_range":
        k = rs.integers(0, 5000, n).astype(np.uint64)
    else:
        raise KeyError(kind)
    return k.astype(np.uint64 if wide else np.uint32)


@pytest.mark.parametrize("kind", DISTS)
@pytest.mark.parametrize("params", [dict(), dict(digit_bits=3, lds_cutoff=300), dict(digit_bits=6, mode=dt.MODE_PLAIN),
                                    dict(digit_bits=10, lds_cutoff=2000)])
def test_distributions_u32(kind, params):
    require_gpu()
    say(f"u32 kind={kind} params={params}")
    sd = seed_of("u32", kind, str(params))
    say(f"seed={sd}")
    rs = np.random.default_rng(sd)
    k = _keys(kind, 400000, False, rs)
    got, st = _sort32(k, **params)
    assert np.array_equal(got, np.sort(k))


@pytest.mark.parametrize("kind", DISTS)
@pytest.mark.parametrize("params", [dict(), dict(digit_bits=4, lds_cutoff=500)])
def test_distributions_u64_and_pairs(kind, params):
    require_gpu()
    say(f"u64 kind={kind} params={params}")
    sd = seed_of("64", kind, str(params))
    say(f"seed={sd}")
    rs = np.random.default_rng(sd)
    k = _keys(kind, 300000, True, rs)
    got, _ = _sort64(k, **params)
    assert np.array_equal(got, np.sort(k))
    v = np.arange(k.size, dtype=np.uint64)
    gk, gv, _ = _pairs64(k, v, **params)
    ek, ev = S.stable_sort_pairs(k, v)
    assert np.array_equal(gk, ek) and np.array_equal(gv, ev)
    assert S.is_stable_by_index(gk, gv)


@pytest.mark.parametrize("kind", DISTS)
@pytest.mark.parametrize("wide", [False, True])
def test_nine_bit_digits(kind, wide):
    """9-bit digits of bare keys run on a distribution variant of their own
    (776 counters, 1024-thread tiles); with ordered ranks they take the
    2048-counter variant.  Both against the definition."""
    require_gpu()
    say(f"nine-bit digits kind={kind} wide={wide}")
    sd = seed_of("nine", kind, wide)
    say(f"seed={sd}")
    rs = np.random.default_rng(sd)
    k = _keys(kind, 700001, wide, rs)
    sort = _sort64 if wide else _sort32
    for extra in (dict(), dict(ordered_ranks=1)):
        got, _ = sort(k, digit_bits=9, **extra)
        assert np.array_equal(got, np.sort(k)), extra


@pytest.mark.parametrize("wide", [False, True])
def test_nine_bit_digits_graph(wide):
    require_gpu()
    say(f"nine-bit digits graph wide={wide}")
    rs = np.random.default_rng(909 + wide)
    k = _keys("zipf", 900001, wide, rs)
    sort = _sort64 if wide else _sort32
    for _ in range(2):  # recorded, then replayed
        got, _ = sort(k, digit_bits=9, graph=1)
        assert np.array_equal(got, np.sort(k))


@pytest.mark.parametrize("kind,wide,params", [("zipf", False, dict(digit_bits=4, lds_cutoff=200)),
                                              ("exp", True, dict(digit_bits=3, lds_cutoff=100)),
                                              ("bexp", True, dict(digit_bits=5, lds_cutoff=150)),
                                              ("uniform", False, dict(digit_bits=2, lds_cutoff=64)),
                                              ("small_range", False, dict(digit_bits=3, lds_cutoff=100))])
def test_recursion_shape_matches_oracle(kind, wide, params):
    """Same seed -> same plans at every level (Appendix A): the device counters
    equal the oracle's counts for Alg. 2 run with the same parameters."""
    require_gpu()
    say(f"shape kind={kind} wide={wide} params={params}")
    rs = np.random.default_rng(5)
    k = _keys(kind, 60000, wide, rs)
    # 32-bit keys without values: children of up to twice the cutoff are sorted as paired leaves
    cfg = R.Config(seed=0, key_bytes=8 if wide else 4, gamma=params["digit_bits"], cutoff=params["lds_cutoff"],
                   pair_leaves=not wide)
    ost = R.Stats()
    ok, _ = R.dtsort(k, None, cfg, stats=ost)
    # ordered ranks: the recursion shape is a function of the seed alone
    got, st = (_sort64 if wide else _sort32)(k, ordered_ranks=1, **params)
    assert np.array_equal(got, ok)
    assert st.levels == ost.levels
    assert st.tasks == ost.tasks
    assert st.records_distributed == ost.distributed
    assert st.heavy_keys == ost.heavy_keys
    assert st.records_leaf_sorted == ost.base_sorted
    assert st.overflow_records == ost.overflow_records
    assert st.merges == ost.merged_zones


def test_determinism():
    require_gpu()
    rs = np.random.default_rng(9)
    k = _keys("zipf", 500000, False, rs)
    a, sa = _sort32(k, seed=3, digit_bits=5, lds_cutoff=300, ordered_ranks=1)
    b, sb = _sort32(k, seed=3, digit_bits=5, lds_cutoff=300, ordered_ranks=1)
    assert np.array_equal(a, b)
    assert sa.as_dict() == sb.as_dict()
    # unordered ranks: the recursion may differ from run to run, the output may not
    c, _ = _sort32(k, seed=3, digit_bits=5, lds_cutoff=300)
    assert np.array_equal(a, c)


@pytest.mark.parametrize("vals", [False, True])
def test_segmented(vals):
    require_gpu()
    say(f"segmented vals={vals}")
    c = W.make_config("segmented_u32", n=3_000_000, n_seg=300, seed=2)
    k = c["keys"].numpy().astype(np.uint32)
    off = c["offsets"].numpy().astype(np.uint64)
    # add empty and tiny segments
    off = np.concatenate([[0, 0, 1, 1], off[1:] + 1]).astype(np.uint64)
    k = np.concatenate([[123], k]).astype(np.uint32)
    v = np.arange(k.size, dtype=np.uint32)
    ek, ev = S.segmented_sort(k, off, v)
    dk, dv, do = dev_u32(k), dev_u32(v), dev_u64(off)
    if vals:
        dt.sort_segmented(dk, do, dv)
    else:
        dt.sort_segmented(dk, do)
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(dk), ek)
    if vals:
        assert np.array_equal(host_u32(dv), ev)


def test_segmented_bad_offsets():
    require_gpu()
    k = dev_u32(np.arange(100, dtype=np.uint32))
    bad = dev_u64(np.array([0, 50, 40, 100], np.uint64))
    with pytest.raises(dt.DTSortError):
        dt.sort_segmented(k, bad)
    torch.cuda.synchronize()


def test_key_bits_option():
    require_gpu()
    rs = np.random.default_rng(4)
    k = rs.integers(0, 2 ** 20, 500000).astype(np.uint32)
    got, _ = _sort32(k, key_bits=20)
    assert np.array_equal(got, np.sort(k))
