"""Pins of the oracle functions the first pin file leaves open: the segmented
sort, the sample positions, the digit-width rule and the learned model's
training data and batches.

Each is checked against something other than its own formula: brute-force
ranks, the published splitmix64 sequence, exact integer arithmetic at points
whose result is known in closed form, a chi-square test of uniformity, and
values worked out by hand.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats as sps

from oracle import dtsort_ref as R
from oracle import mlp
from oracle import rng
from oracle import sort as S
from tests._seeds import seed_of


# ------------------------------------------------------------ segmented sort
def _bruteforce_segmented(keys, offsets, values):
    """Every segment on its own through the O(n^2) rank formula of Section 2.3."""
    k_out, v_out = list(keys), list(values)
    for s in range(len(offsets) - 1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        ranks = S.stable_rank_bruteforce(keys[a:b])
        k_out[a:b] = S.apply_ranks(list(keys[a:b]), ranks)
        v_out[a:b] = S.apply_ranks(list(values[a:b]), ranks)
    return k_out, v_out


@pytest.mark.parametrize("case", range(8))
def test_segmented_sort_matches_bruteforce_per_segment(case):
    rs = np.random.default_rng(seed_of("segmented", case))
    # segment sizes with empty, one-record and tied segments among them
    sizes = [0, 1, 0, int(rs.integers(2, 40)), 1, int(rs.integers(0, 60)), 0, int(rs.integers(1, 30))]
    rs.shuffle(sizes)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(offsets[-1])
    hi = 4 if case % 2 == 0 else 2 ** 32      # many ties / few ties
    keys = rs.integers(0, hi, n).astype(np.uint32)
    values = np.arange(n, dtype=np.uint32)[::-1].copy()   # distinct, not in key order
    gk, gv = S.segmented_sort(keys, offsets, values)
    ek, ev = _bruteforce_segmented(keys, offsets, values)
    assert list(gk) == ek and list(gv) == ev
    # no record crosses a segment boundary
    for s in range(len(sizes)):
        a, b = int(offsets[s]), int(offsets[s + 1])
        assert sorted(gv[a:b].tolist()) == sorted(values[a:b].tolist())
    # keys only
    k2, v2 = S.segmented_sort(keys, offsets)
    assert v2 is None and list(k2) == ek


def test_segmented_sort_hand_example():
    keys = np.array([5, 3, 9, 9, 1, 7, 7, 2], np.uint32)
    vals = np.array([0, 1, 2, 3, 4, 5, 6, 7], np.uint32)
    off = np.array([0, 3, 3, 4, 8], np.uint64)          # [5 3 9] [] [9] [1 7 7 2]
    k, v = S.segmented_sort(keys, off, vals)
    assert k.tolist() == [3, 5, 9, 9, 1, 2, 7, 7]
    assert v.tolist() == [1, 0, 2, 3, 4, 7, 5, 6]
    # the input is left untouched
    assert keys.tolist() == [5, 3, 9, 9, 1, 7, 7, 2]


# --------------------------------------------------------- sample positions
def test_sample_words_are_a_splitmix64_sequence(golden_dir):
    # The i-th sample word is output i+1 of the published splitmix64 generator
    # (its output sequence is pinned by the golden file) started at the
    # subproblem's base state.
    g = json.load(open(os.path.join(golden_dir, "splitmix64.json")))
    assert rng.splitmix64_stream(g["state"], len(g["outputs"])) == g["outputs"]
    for seed, off, level in [(0, 0, 0), (7, 123456, 2), (2 ** 63 + 5, 2 ** 40, 9)]:
        h2 = rng.sample_base(seed, off, level)
        words = rng.sample_words(seed, off, level, 50)
        assert [int(w) for w in words] == rng.splitmix64_stream(h2, 50)


def test_multiply_high_exact_points():
    # floor(r * n / 2^64) at words whose product is known exactly
    n = 1_000_000_007
    pts = np.array([0, 1, 2 ** 63, 2 ** 62, 3 * 2 ** 62, 2 ** 64 - 1], dtype=np.uint64)
    got = rng.mulhi64(pts, n).tolist()
    assert got == [0, 0, n // 2, n // 4, (3 * n) // 4, n - 1]
    # n a power of two: the top bits of the word
    pts = np.array([0xDEADBEEFCAFEBABE, 0x0123456789ABCDEF, 2 ** 64 - 1], dtype=np.uint64)
    assert rng.mulhi64(pts, 1 << 20).tolist() == [int(p) >> 44 for p in pts.tolist()]
    # n = 2^64 - 1 (largest): r * (2^64 - 1) / 2^64 = r - 1 for r > 0
    assert rng.mulhi64(np.array([5, 2 ** 63], np.uint64), 2 ** 64 - 1).tolist() == [4, 2 ** 63 - 1]


@pytest.mark.parametrize("n_sub", [1, 2, 97, 100003])
def test_sample_positions_in_range_and_uniform(n_sub):
    count = 40000
    pos = rng.sample_positions(3, 4096, 1, n_sub, count)
    assert pos.dtype == np.int64 and pos.size == count
    assert int(pos.min()) >= 0 and int(pos.max()) < n_sub
    if n_sub == 1:
        assert (pos == 0).all()
        return
    bins = min(n_sub, 64)
    # equal-width bins over [0, n_sub); expected count proportional to width
    edges = np.linspace(0, n_sub, bins + 1)
    obs, _ = np.histogram(pos, bins=np.floor(edges).astype(np.int64))
    width = np.diff(np.floor(edges)).astype(np.float64)
    exp = count * width / n_sub
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert chi2 < sps.chi2.ppf(0.999, bins - 1), chi2


def test_sample_positions_depend_on_seed_offset_level():
    a = rng.sample_positions(0, 0, 0, 1 << 30, 64)
    assert not np.array_equal(a, rng.sample_positions(1, 0, 0, 1 << 30, 64))
    assert not np.array_equal(a, rng.sample_positions(0, 8192, 0, 1 << 30, 64))
    assert not np.array_equal(a, rng.sample_positions(0, 0, 1, 1 << 30, 64))
    assert np.array_equal(a, rng.sample_positions(0, 0, 0, 1 << 30, 64))


# ------------------------------------------------------------- digit width
# Section 6: gamma is log2 of the cube root of n, capped by 8 and 12; read with
# the integer floor(log2 n), i.e. gamma = clamp(round(floor(log2 n) / 3)).
# Values worked out by hand at the boundaries where floor(log2 n) changes.
@pytest.mark.parametrize("n,g10,g11", [
    (2, 8, 8), (1 << 20, 8, 8), ((1 << 23) - 1, 8, 8), (1 << 23, 8, 8),
    ((1 << 26) - 1, 8, 8), (1 << 26, 9, 9), ((1 << 29) - 1, 9, 9), (1 << 29, 10, 10),
    (10 ** 9, 10, 10), ((1 << 32) - 1, 10, 10), (1 << 32, 10, 11), (1 << 35, 10, 11),
])
def test_gamma_auto_boundaries(n, g10, g11):
    assert R.gamma_auto(n, 8, 10) == g10
    assert R.gamma_auto(n, 8, 11) == g11
    # against the real-valued rule at powers of two, where floor(log2 n) = log2 n
    if n & (n - 1) == 0:
        assert R.gamma_auto(n, 8, 12) == max(8, min(12, round(math.log2(n) / 3)))


# ------------------------------------------------ learned model: data, batches
def test_training_data_hand_values():
    # keys 0, 1, 2, 4, 8 under 4-bit keys: t = 0, 1/5, 2/5, 3/5, 4/5 (each a
    # power of two starts a new binary order of magnitude), so x is evenly
    # spaced; y = (i + 0.5) / 5
    x, y = mlp.training_data(np.array([0, 1, 2, 4, 8], np.uint64), key_bits=4)
    assert np.allclose(x, [0.0, 0.25, 0.5, 0.75, 1.0], rtol=0, atol=1e-15)
    assert np.allclose(y, [0.1, 0.3, 0.5, 0.7, 0.9], rtol=0, atol=1e-15)
    # keys 3, 6, 12 (8-bit): halfway through orders 1, 2, 3 -> t = 2.5, 3.5, 4.5 (/ 9)
    x, y = mlp.training_data(np.array([3, 6, 12], np.uint32), key_bits=8)
    assert np.allclose(x, [0.0, 0.5, 1.0], rtol=0, atol=1e-15)
    assert np.allclose(y, [1 / 6, 0.5, 5 / 6], rtol=0, atol=1e-15)
    # keys 5, 6, 7, 8, 12 (8-bit): 5 = 4 + 1 -> e = 2, t = 3 + 1/4; 6 -> 3.5;
    # 7 -> 3.75; 8 -> e = 3, t = 4; 12 -> 4.5 (all over 9)
    x, _ = mlp.training_data(np.array([5, 6, 7, 8, 12], np.uint64), key_bits=8)
    t = np.array([3.25, 3.5, 3.75, 4.0, 4.5])
    assert np.allclose(x, (t - 3.25) / (4.5 - 3.25), rtol=0, atol=1e-15)
    # all keys equal: x = 0
    x, y = mlp.training_data(np.full(4, 77, np.uint64))
    assert (x == 0).all() and np.allclose(y, [0.125, 0.375, 0.625, 0.875])


def test_loglinear_word_range():
    # the full 64-bit range maps into [0, 1]: 2^63 -> 64 / 65; 2^64 - 1 -> 1
    # (its fraction (2^63 - 1) / 2^63 rounds to 1 in float64)
    t = mlp.loglinear(np.array([0, 1, 2 ** 63, 2 ** 63 + 2 ** 62, 2 ** 64 - 1], np.uint64), 64)
    assert t[0] == 0.0 and math.isclose(t[1], 1 / 65) and math.isclose(t[2], 64 / 65)
    assert math.isclose(t[3], 64.5 / 65) and t[4] == 1.0


def test_batch_indices_hand_values():
    # n = 10, batch 3: stride 3, offset = step mod 3
    assert mlp.batch_indices(10, 3, 0).tolist() == [0, 3, 6]
    assert mlp.batch_indices(10, 3, 4).tolist() == [1, 4, 7]
    assert mlp.batch_indices(10, 3, 5).tolist() == [2, 5, 8]
    # batch = n: every index every step
    assert mlp.batch_indices(5, 5, 3).tolist() == [0, 1, 2, 3, 4]
    # every index is drawn once per stride steps, and all lie in range
    n, b = 1 << 16, 1024
    seen = np.concatenate([mlp.batch_indices(n, b, s) for s in range(n // b)])
    assert np.array_equal(np.sort(seen), np.arange(n))


# ------------------------------------------------- multicore host stable sort
@pytest.mark.parametrize("threads", [1, 4])
def test_parallel_host_sort_is_the_stable_order(threads):
    from oracle import psort
    rs = np.random.default_rng(seed_of("psort", threads))
    k = rs.integers(0, 2 ** 32, 300001).astype(np.uint32)
    e = S.stable_sort_keys(k)
    assert psort.sort_u32_(k, threads) == threads
    assert np.array_equal(k, e)
    # pairs with many ties: stability is visible through the values
    keys = rs.integers(0, 50, 200000).astype(np.uint64)
    vals = np.arange(keys.size, dtype=np.uint64)
    ek, ev = S.stable_sort_pairs(keys, vals)
    psort.sort_pairs_u64_(keys, vals, threads)
    assert np.array_equal(keys, ek) and np.array_equal(vals, ev)
    # tiny input against the brute-force ranks
    small = rs.integers(0, 4, 40).astype(np.uint64)
    sv = np.arange(40, dtype=np.uint64)
    ranks = S.stable_rank_bruteforce(small)
    bk, bv = S.apply_ranks(list(small), ranks), S.apply_ranks(list(sv), ranks)
    psort.sort_pairs_u64_(small, sv, threads)
    assert list(small) == bk and list(sv) == bv
