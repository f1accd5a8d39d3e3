"""Seeded sweep over combinations of entry point, size, key distribution and
options, each result compared bit-exactly with the oracle's stable sort
(Section 2.3: the method's output is the unique stable ascending order).

The per-option tests elsewhere vary one knob at a time; here every case draws
all of them at once (digit width, base-case cutoff, scatter tile, merge
variant, heavy-key detection on or off, ordered ranks, graph form, digit
width below the root), so that
interactions between options are exercised too.  A case is fixed by its
index: its parameters are printed before it runs and are the same in every
process.
"""
import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
from oracle import sort as S
from tests._dev import dev_u32, dev_u64, host_u32, host_u64, require_gpu, say
from tests._seeds import seed_of

pytestmark = pytest.mark.gpu

ENTRIES = ["u32", "u64", "pairs_u64", "pairs_u32", "seg", "seg_vals"]
SIZES = [0, 1, 2, 7, 257, 1025, 4097, 8193, 16385, 32769, 65537, 123457, 200003]
KINDS = ["uniform", "zipf", "equal", "two", "exp", "bexp", "max", "small_range", "sorted", "reversed"]
N_CASES = 120


def _keys(kind, n, wide, rs):
    bits = 64 if wide else 32
    if kind == "uniform":
        k = rs.integers(0, 2 ** bits, n, dtype=np.uint64)
    elif kind == "zipf":
        k = (rs.zipf(1.3, n).astype(np.uint64) * np.uint64(0x9E3779B1)) & np.uint64((1 << bits) - 1)
    elif kind == "equal":
        k = np.full(n, 12345, np.uint64)
    elif kind == "two":
        k = rs.choice(np.array([9, 2 ** (bits - 1) + 3], np.uint64), n)
    elif kind == "exp":
        k = rs.exponential(3e4, n).astype(np.uint64)
    elif kind == "bexp":
        b = np.minimum(rs.geometric(0.1, n), bits)
        low = rs.integers(0, 2 ** 63, n, dtype=np.uint64)
        lead = np.left_shift(np.uint64(1), (b - 1).astype(np.uint64))
        k = lead | (low & (lead - np.uint64(1)))
    elif kind == "max":
        k = np.full(n, 2 ** bits - 1, np.uint64)
        k[::5] = 0
    elif kind == "small_range":
        k = rs.integers(0, 300, n).astype(np.uint64)
    elif kind == "sorted":
        k = np.sort(rs.integers(0, 2 ** bits, n, dtype=np.uint64))
    elif kind == "reversed":
        k = np.sort(rs.integers(0, 2 ** bits, n, dtype=np.uint64))[::-1].copy()
    else:
        raise KeyError(kind)
    return k.astype(np.uint64 if wide else np.uint32)


def _case(i):
    rs = np.random.default_rng(seed_of("combo", i))
    entry = ENTRIES[i % len(ENTRIES)]
    p = dict(
        n=int(rs.choice(SIZES)),
        kind=str(rs.choice(KINDS)),
        digit_bits=int(rs.choice([0, 0, 2, 4, 7, 8, 9, 10])),
        digit_bits_below=int(rs.choice([0, 0, 0, 3, 8, 9])),
        lds_cutoff=int(rs.choice([0, 0, 2, 50, 600, 5000, 20000])),
        tile_shape=int(rs.integers(0, 7)),
        merge_variant=int(rs.choice([dt.MERGE_GATHER, dt.MERGE_GATHER, dt.MERGE_PLMERGE, dt.MERGE_INPLACE,
                                     dt.MERGE_SPLIT])),
        mode=int(rs.choice([dt.MODE_SAMPLING, dt.MODE_SAMPLING, dt.MODE_PLAIN])),
        ordered_ranks=int(rs.integers(0, 2)),
        graph=int(rs.integers(0, 2)),
        seed=int(rs.integers(0, 2 ** 32)),
    )
    return entry, p, rs


@pytest.mark.parametrize("i", range(N_CASES))
def test_combination(i):
    require_gpu()
    entry, p, rs = _case(i)
    say(f"combo {i}: {entry} {p}")
    n, kind = p.pop("n"), p.pop("kind")
    o = dt.make_opts(**p)
    wide = entry in ("u64", "pairs_u64")
    k = _keys(kind, n, wide, rs)
    dev = dev_u64 if wide else dev_u32
    host = host_u64 if wide else host_u32
    dk = dev(k)
    if entry in ("u32", "u64"):
        (dt.sort_u64 if wide else dt.sort_u32)(dk, o)
        torch.cuda.synchronize()
        assert np.array_equal(host(dk), S.stable_sort_keys(k))
    elif entry in ("pairs_u64", "pairs_u32"):
        v = np.arange(n, dtype=np.uint64 if wide else np.uint32)
        dv = dev(v)
        (dt.sort_pairs_u64 if wide else dt.sort_pairs_u32)(dk, dv, o)
        torch.cuda.synchronize()
        ek, ev = S.stable_sort_pairs(k, v)
        assert np.array_equal(host(dk), ek)
        assert np.array_equal(host(dv), ev)
    else:
        # segments of random lengths, empty ones included
        n_seg = int(rs.integers(1, 40))
        cuts = np.sort(rs.integers(0, n + 1, n_seg - 1)) if n_seg > 1 else np.zeros(0, np.int64)
        off = np.concatenate([[0], cuts, [n]]).astype(np.uint64)
        v = np.arange(n, dtype=np.uint32)
        ek, ev = S.segmented_sort(k, off, v if entry == "seg_vals" else None)
        dv = dev_u32(v) if entry == "seg_vals" else None
        dt.sort_segmented(dk, dev_u64(off), dv, o)
        torch.cuda.synchronize()
        assert np.array_equal(host_u32(dk), ek)
        if dv is not None:
            assert np.array_equal(host_u32(dv), ev)
