"""The implementations of Step 4 the paper's merge study compares (Section
6.3, Fig. scale c-d): the dovetail merge as one gather (default), a general
merge-path merge of each zone through the partner buffer (PLMerge-style) and
Alg. 3 literally (smaller side copied out, heavy buckets moved one by one
with two flips where a bucket overlaps its destination); and dovetailing
during distribution (each zone's light keys split at its heavy keys, no
merge).  All four must give
the oracle's stable order exactly; the no-merge knob (a timing aid, not a
sort) must run the same recursion without Step 4."""
import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
import workloads as W
from oracle import sort as S
from tests._dev import dev_u32, dev_u64, host_u32, host_u64, require_gpu, say
from tests._seeds import seed_of

pytestmark = pytest.mark.gpu

VARIANTS = [dt.MERGE_GATHER, dt.MERGE_PLMERGE, dt.MERGE_INPLACE, dt.MERGE_SPLIT]


def _keys(kind, n, bits, seed):
    if kind in ("zipf-1.5", "zipf-0.6", "exp-10", "unif-1000", "bexp-10", "bexp-300"):
        fam, prm = kind.split("-")
        k = W.paper_keys(fam, float(prm), n, bits, seed=seed).numpy()
    elif kind == "heavy_majority":
        # zones where heavy records outnumber light ones (the first branch of Alg. 3)
        rs = np.random.default_rng(seed)
        k = rs.integers(0, 2 ** (bits - 1), n, dtype=np.uint64)
        hot = rs.integers(0, 2 ** (bits - 1), 40, dtype=np.uint64)
        pick = rs.random(n) < 0.85
        k[pick] = hot[rs.integers(0, 40, int(pick.sum()))]
        return k.astype(np.uint32 if bits == 32 else np.uint64)
    elif kind == "light_majority":
        # a few heavy keys inside mostly light zones (the symmetric branch)
        rs = np.random.default_rng(seed)
        k = rs.integers(0, 2 ** bits if bits == 32 else 2 ** 63, n, dtype=np.uint64)
        hot = rs.integers(0, 2 ** 31, 6, dtype=np.uint64)
        pick = rs.random(n) < 0.2
        k[pick] = hot[rs.integers(0, 6, int(pick.sum()))]
        return k.astype(np.uint32 if bits == 32 else np.uint64)
    else:
        raise KeyError(kind)
    return k.astype(np.uint32) if bits == 32 else k.view(np.uint64)


def _run(layout, k, **kw):
    n = k.size
    st = dt.Stats()
    o = dt.make_opts(stats=st, **kw)
    if layout == "u32":
        d = dev_u32(k)
        dt.sort_u32(d, o)
        torch.cuda.synchronize()
        return host_u32(d), None, st
    if layout == "pairs32":
        dk, dv = dev_u32(k), dev_u32(np.arange(n, dtype=np.uint32))
        dt.sort_pairs_u32(dk, dv, o)
        torch.cuda.synchronize()
        return host_u32(dk), host_u32(dv), st
    dk, dv = dev_u64(k), dev_u64(np.arange(n, dtype=np.uint64))
    dt.sort_pairs_u64(dk, dv, o)
    torch.cuda.synchronize()
    return host_u64(dk), host_u64(dv), st


KINDS = ["zipf-1.5", "zipf-0.6", "exp-10", "unif-1000", "bexp-10", "bexp-300", "heavy_majority", "light_majority"]


@pytest.mark.parametrize("layout", ["u32", "pairs32", "pairs64"])
@pytest.mark.parametrize("kind", KINDS)
def test_merge_variants_match_oracle(layout, kind):
    require_gpu()
    bits = 64 if layout == "pairs64" else 32
    n = 600_011
    sd = seed_of("mv", layout, kind)
    say(f"merge variants {layout} {kind} seed={sd}")
    k = _keys(kind, n, bits, sd)
    v = np.arange(n, dtype=np.uint32 if bits == 32 else np.uint64)
    ek, ev = S.stable_sort_pairs(k, v)
    merged = []
    for params in (dict(), dict(digit_bits=4, lds_cutoff=500)):
        for mv in VARIANTS:
            gk, gv, st = _run(layout, k, merge_variant=mv, ordered_ranks=1, **params)
            assert np.array_equal(gk, ek), f"variant {mv} {params}: keys"
            if gv is not None:
                assert np.array_equal(gv, ev), f"variant {mv} {params}: values"
            merged.append((str(params), mv, st.merges, st.records_merged))
    # the recursion does not depend on the merge implementation; the split
    # layout merges nothing
    for p in {m[0] for m in merged}:
        rows = [m for m in merged if m[0] == p and m[1] != dt.MERGE_SPLIT]
        assert len({(r[2], r[3]) for r in rows}) == 1, rows
        assert all(m[2] == 0 for m in merged if m[0] == p and m[1] == dt.MERGE_SPLIT)
    if kind in ("zipf-1.5", "heavy_majority", "light_majority", "bexp-300"):
        assert max(m[2] for m in merged) > 0, "the case is meant to merge zones"


@pytest.mark.parametrize("mv", VARIANTS)
def test_merge_variants_graph_form(mv):
    require_gpu()
    say(f"merge variant {mv} graph form")
    k = _keys("zipf-1.5", 900_007, 64, 5)
    v = np.arange(k.size, dtype=np.uint64)
    ek, ev = S.stable_sort_pairs(k, v)
    dk, dv = dev_u64(k), dev_u64(v)
    for rep in range(2):
        dk.copy_(dev_u64(k))
        dv.copy_(dev_u64(v))
        dt.sort_pairs_u64(dk, dv, dt.make_opts(graph=1, merge_variant=mv, digit_bits=6))
        torch.cuda.synchronize()
        assert np.array_equal(host_u64(dk), ek) and np.array_equal(host_u64(dv), ev)


def test_no_merge_knob_runs_the_same_recursion():
    """The knob skips Step 4 only: the call succeeds and every other step
    does the work it does with merging (same counters, ordered ranks)."""
    require_gpu()
    k = _keys("zipf-1.5", 500_009, 32, 9)
    _, _, st = _run("pairs32", k, merge_variant=dt.MERGE_NONE, ordered_ranks=1)
    _, _, sg = _run("pairs32", k, merge_variant=dt.MERGE_GATHER, ordered_ranks=1)
    assert st.merges > 0
    for f in ("levels", "tasks", "records_distributed", "heavy_keys", "merges", "records_leaf_sorted"):
        assert getattr(st, f) == getattr(sg, f), f


@pytest.mark.parametrize("digits", [1, 2, 3, 8, 9, 10])
def test_split_layout_digit_widths(digits):
    """Dovetailing during distribution at every digit width class: the heavy
    cap 2^(g-2) (none at g = 1), the hash-table and binary-search lookups,
    and the wide-digit kernel variants; keys and 64-bit pairs."""
    require_gpu()
    say(f"split layout digits={digits}")
    for layout, kind in (("u32", "zipf-1.5"), ("pairs64", "heavy_majority"), ("pairs32", "bexp-300")):
        bits = 64 if layout == "pairs64" else 32
        k = _keys(kind, 400_009, bits, digits)
        v = np.arange(k.size, dtype=np.uint32 if bits == 32 else np.uint64)
        ek, ev = S.stable_sort_pairs(k, v)
        gk, gv, st = _run(layout, k, merge_variant=dt.MERGE_SPLIT, digit_bits=digits, lds_cutoff=300)
        assert np.array_equal(gk, ek), layout
        if gv is not None:
            assert np.array_equal(gv, ev), layout
        assert st.merges == 0
        if digits >= 2:
            assert st.heavy_keys > 0


def test_split_with_learned_root():
    """A learned root keeps its merges; the levels below split."""
    require_gpu()
    k = W.mixture_u64(1 << 21, seed=4).numpy().view(np.uint64)
    v = np.arange(k.size, dtype=np.uint64)
    ek, ev = S.stable_sort_pairs(k, v)
    gk, gv, st = _run("pairs64", k, merge_variant=dt.MERGE_SPLIT, mode=dt.MODE_LEARNED, learned_judge=1)
    assert np.array_equal(gk, ek) and np.array_equal(gv, ev)
    assert st.learned_used == 1
