"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Sources: the problem statement (Section 2.3: non-decreasing order; stable =
equal keys keep input order), brute-force ranks, hand-worked examples of the
method's steps (Alg. 2, Sections 3.1-3.4, the overflow bucket of Section 5),
the counting-sort formula of Appendix B, Alg. 3's closed-form positions, the
published splitmix64 sequence, and special cases whose outcome the theory
fixes (Section 4: few distinct keys are all heavy; unique keys are never
heavy).
"""
import json
import os

import numpy as np
import pytest

from oracle import dtsort_ref as R
from oracle import rng
from oracle import sort as S
from tests._seeds import seed_of


def test_splitmix64_published_sequence(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64.json")))
    assert rng.splitmix64_stream(g["state"], len(g["outputs"])) == g["outputs"]


@pytest.mark.parametrize("seed", range(6))
def test_stable_sort_matches_bruteforce_rank(seed):
    rs = np.random.default_rng(seed)
    n = int(rs.integers(0, 120))
    if seed % 3 == 0:
        keys = rs.integers(0, 5, n).astype(np.uint32)            # many ties
    elif seed % 3 == 1:
        keys = rs.integers(0, 2 ** 63, n, dtype=np.uint64) * np.uint64(2) + np.uint64(seed % 2)
    else:
        keys = np.concatenate([np.full(n // 2, 2 ** 32 - 1), rs.integers(0, 2 ** 32, n - n // 2)]).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint64)
    ranks = S.stable_rank_bruteforce(keys)
    exp_k = S.apply_ranks(list(keys), ranks)
    exp_v = S.apply_ranks(list(vals), ranks)
    ok, ov = S.stable_sort_pairs(keys, vals)
    assert list(ok) == exp_k and list(ov) == exp_v


def test_invariant_checkers_catch_planted_mistakes():
    rs = np.random.default_rng(1)
    k = np.sort(rs.integers(0, 50, 1000).astype(np.uint64))
    v = np.argsort(np.argsort(k, kind="stable"), kind="stable").astype(np.uint64)
    idx = np.arange(1000, dtype=np.uint64)
    assert S.is_nondecreasing(k) and S.is_stable_by_index(k, idx)
    bad = k.copy(); bad[10], bad[900] = bad[900], bad[10]
    assert not S.is_nondecreasing(bad)
    assert S.multiset_hash(bad) == S.multiset_hash(k)            # a swap keeps the multiset
    drop = k.copy(); drop[5] = k[-1]                            # one record replaced
    assert S.multiset_hash(drop) != S.multiset_hash(k)
    j = int(np.flatnonzero(k[1:] == k[:-1])[0])
    swapped = idx.copy(); swapped[j], swapped[j + 1] = swapped[j + 1], swapped[j]
    assert not S.is_stable_by_index(k, swapped)
    assert S.multiset_hash(k, v) != S.multiset_hash(k, v[::-1].copy())


def test_order_statistic_by_counting():
    rs = np.random.default_rng(2)
    k = rs.integers(0, 1000, 5000).astype(np.uint32)
    s = np.sort(k)
    for q in [0, 1, 17, 2500, 4999]:
        assert S.order_statistic(k, q) == int(s[q])


def _golden_cases(golden_dir):
    return json.load(open(os.path.join(golden_dir, "dtsort_hand.json")))["cases"]


def test_hand_worked_examples(golden_dir):
    for c in _golden_cases(golden_dir):
        keys = np.array(c["keys"], dtype=np.uint64)
        idx = np.arange(keys.size, dtype=np.uint64)
        p = R.make_plan(c["hi"], c["top"], c["w"], c["shift"], c["heavy"])
        assert list(p.light_id) == c["L"], c["name"]
        ids = R.bucket_ids(keys, p)
        assert list(ids) == c["bucket_ids"], c["name"]
        assert list(R.bucket_ids_np(keys, p)) == c["bucket_ids"], c["name"]
        for dist in (R.distribute, R.distribute_counting):
            dk, dv, cnt = dist(keys, ids, p.n_buckets, values=idx)
            assert list(dk) == c["distributed_keys"] and list(dv) == c["distributed_index"], c["name"]
            assert list(cnt) == c["counts"], c["name"]
        for mz in c["merge_zones"]:
            pos = R.dtmerge_positions(np.array(mz["b0_sorted"], np.uint64), np.array(mz["heavy"], np.uint64),
                                      np.array(mz["sizes"], np.int64))
            assert list(pos) == mz["p"]
        sk, sv = S.stable_sort_pairs(keys, idx)
        assert list(sk) == c["sorted_keys"] and list(sv) == c["sorted_index"], c["name"]


@pytest.mark.parametrize("seed", range(5))
def test_counting_sort_formula_equals_stable_sort_by_id(seed):
    rs = np.random.default_rng(seed)
    n, nb = 3000, 37
    ids = rs.integers(0, nb, n)
    keys = rs.integers(0, 2 ** 32, n).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint64)
    a = R.distribute_counting(keys, ids, nb, n_sub=int(rs.integers(1, 9)), values=vals)
    b = R.distribute(keys, ids, nb, values=vals)
    o = np.argsort(ids, kind="stable")
    for x in (a, b):
        assert (x[0] == keys[o]).all() and (x[1] == vals[o]).all()
        assert (x[2] == np.bincount(ids, minlength=nb)).all()


@pytest.mark.parametrize("seed", range(40))
def test_dtmerge_matches_stable_merge(seed):
    rs = np.random.default_rng(seed)
    m = int(rs.integers(1, 6))
    heavy = np.sort(rs.choice(200, m, replace=False)).astype(np.uint64)
    light_pool = np.setdiff1d(np.arange(200), heavy)
    nb0 = int(rs.integers(0, 60))
    b0 = np.sort(rs.choice(light_pool, nb0)).astype(np.uint64)
    sizes = rs.integers(1, 40, m).astype(np.int64)
    zone = np.concatenate([b0] + [np.full(s, h, np.uint64) for h, s in zip(heavy, sizes)])
    vals = np.arange(zone.size, dtype=np.uint64)
    ek, ev = S.stable_sort_pairs(zone, vals)
    zk, zv = zone.copy(), vals.copy()
    R.dtmerge_inplace(zk, zv, nb0, heavy, sizes)
    assert (zk == ek).all() and (zv == ev).all()
    hv, st = [], nb0
    for s in sizes:
        hv.append(vals[st:st + s]); st += s
    gk, gv = R.dtmerge_gather(zone[:nb0], vals[:nb0], heavy, hv, sizes)
    assert (gk == ek).all() and (gv == ev).all()
    p = R.dtmerge_positions(zone[:nb0], heavy, sizes)
    for i in range(m):
        first = int(np.searchsorted(ek, heavy[i], side="left"))
        assert p[i] == first


def _inputs(kind, n, rs):
    if kind == "uniform32":
        return rs.integers(0, 2 ** 32, n).astype(np.uint32)
    if kind == "zipf":
        return (rs.zipf(1.2, n) % 100000).astype(np.uint32)
    if kind == "exp64":
        return rs.exponential(3e4, n).astype(np.uint64)
    if kind == "bexp64":
        k = np.minimum(rs.geometric(0.1, n), 64)
        low = rs.integers(0, 2 ** 63, n, dtype=np.uint64)
        lead = np.left_shift(np.uint64(1), (k - 1).astype(np.uint64))
        return lead | (low & (lead - np.uint64(1)))
    if kind == "equal":
        return np.full(n, 123456789, np.uint64)
    if kind == "two":
        return rs.choice(np.array([5, 2 ** 31], np.uint32), n)
    if kind == "max":
        return np.full(n, 2 ** 64 - 1, np.uint64)
    raise KeyError(kind)


@pytest.mark.parametrize("kind", ["uniform32", "zipf", "exp64", "bexp64", "equal", "two", "max"])
@pytest.mark.parametrize("cfg", [dict(), dict(gamma=3, cutoff=64), dict(gamma=5, cutoff=200, plain=True),
                                 dict(gamma=2, cutoff=8)])
def test_recursive_method_equals_definition(kind, cfg):
    rs = np.random.default_rng(seed_of(kind, str(cfg)))
    n = 20000 if not cfg else 3000
    keys = _inputs(kind, n, rs)
    vals = np.arange(n, dtype=np.uint64)
    c = R.Config(key_bytes=keys.dtype.itemsize, **cfg)
    st = R.Stats()
    ok, ov = R.dtsort(keys, vals, c, stats=st)
    ek, ev = S.stable_sort_pairs(keys, vals)
    assert (ok == ek).all() and (ov == ev).all()


def test_all_equal_keys_single_heavy_key():
    keys = np.full(50000, 77, np.uint32)
    p = R.plan(keys, 32, keys.size, 0, 0, R.Config(key_bytes=4))
    assert list(p.heavy) == [77]
    assert p.top == 7


def test_unique_keys_are_never_heavy():
    keys = np.random.default_rng(3).permutation(200000).astype(np.uint32)
    for seed in range(5):
        p = R.plan(keys, 32, keys.size, 0, 0, R.Config(key_bytes=4, seed=seed))
        assert p.heavy.size == 0


def test_few_distinct_keys_all_heavy_one_level():
    # Section 4 (special case of few distinct keys): with at most 2^gamma / 4
    # equally frequent distinct keys, every key is heavy at the root and one
    # level suffices.
    rs = np.random.default_rng(4)
    distinct = rs.choice(2 ** 32, 64, replace=False).astype(np.uint32)
    keys = distinct[rs.integers(0, 64, 400000)]
    for seed in range(3):
        st = R.Stats()
        c = R.Config(key_bytes=4, seed=seed)
        p = R.plan(keys, 32, keys.size, 0, 0, c)
        assert set(p.heavy.tolist()) == set(distinct.tolist())
        R.dtsort(keys, None, c, stats=st)
        assert st.levels == 1 and st.base_sorted == 0


def test_planted_heavy_key_is_found():
    # A key holding at least 4 n' / 2^gamma records is flagged (Section 2.5:
    # keys seen twice in the subsample have Omega(n/p) occurrences, and
    # conversely heavy enough keys are seen twice with high probability).
    rs = np.random.default_rng(5)
    n = 300000
    found = 0
    for seed in range(20):
        keys = rs.integers(0, 2 ** 32, n).astype(np.uint32)
        g = R.gamma_auto(n)
        pos = rs.choice(n, 4 * n // (1 << g), replace=False)
        keys[pos] = 4242
        p = R.plan(keys, 32, n, 0, 0, R.Config(key_bytes=4, seed=seed))
        found += int(4242 in set(p.heavy.tolist()))
    assert found >= 19


def test_sampled_range_and_overflow():
    rs = np.random.default_rng(6)
    keys = rs.integers(0, 2 ** 20, 100000).astype(np.uint64)
    keys[rs.integers(0, keys.size, 3)] = 2 ** 40 + 5          # rare keys above the sampled range
    p = R.plan(keys, 64, keys.size, 0, 0, R.Config(key_bytes=8))
    assert p.top <= 20
    ids = R.bucket_ids_np(keys, p)
    assert np.count_nonzero(ids == p.overflow_id) >= 3
    ok, _ = R.dtsort(keys, None, R.Config(key_bytes=8))
    assert (ok == np.sort(keys)).all()


def test_work_per_level_at_most_n():
    # Each level distributes at most n' records in total (Section 4, the
    # per-level work lemma): total distributed <= n * levels.
    rs = np.random.default_rng(7)
    keys = rs.integers(0, 2 ** 32, 60000).astype(np.uint32)
    st = R.Stats()
    R.dtsort(keys, None, R.Config(key_bytes=4, gamma=3, cutoff=50), stats=st)
    assert st.distributed <= keys.size * st.levels


def test_determinism_given_seed():
    # Appendix A: all operations are deterministic once the seed is fixed.
    rs = np.random.default_rng(8)
    keys = (rs.zipf(1.1, 50000) % 5000).astype(np.uint32)
    a, b = R.Stats(), R.Stats()
    R.dtsort(keys, None, R.Config(key_bytes=4, seed=9, gamma=4, cutoff=100), stats=a)
    R.dtsort(keys, None, R.Config(key_bytes=4, seed=9, gamma=4, cutoff=100), stats=b)
    assert a == b


def test_pair_leaves_rule():
    # The base case of a child subproblem grows to 2 * cutoff with pair_leaves;
    # the output is the same stable order, and children of cutoff < n' <= 2 *
    # cutoff are no longer distributed.
    rs = np.random.default_rng(12)
    keys = rs.integers(0, 2 ** 32, 60000, dtype=np.uint64).astype(np.uint32)
    plain, paired = R.Stats(), R.Stats()
    a, _ = R.dtsort(keys, None, R.Config(key_bytes=4, gamma=2, cutoff=10000), stats=plain)
    b, _ = R.dtsort(keys, None, R.Config(key_bytes=4, gamma=2, cutoff=10000, pair_leaves=True), stats=paired)
    assert (a == np.sort(keys)).all() and (b == a).all()
    assert plain.levels == 2 and paired.levels == 1
    assert paired.tasks == 1 and paired.base_sorted == keys.size
    # the root itself stays a distributed subproblem
    small = keys[:15000]
    st = R.Stats()
    R.dtsort(small, None, R.Config(key_bytes=4, gamma=2, cutoff=10000, pair_leaves=True), stats=st)
    assert st.tasks >= 1
