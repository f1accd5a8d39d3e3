"""DovetailSort's steps, in the paper's order, on the CPU (float-free, integer only).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Each recursive call (Alg. 2) runs four steps on the current subproblem A of
n' records whose keys all share the bits at and above ``hi``:

1. Sampling (Section 3.1, Alg. 2 "Sampling"; the sampled key range and the
   overflow bucket of Section 5).  ``plan`` below.
2. Distributing (Section 3.2): a stable counting sort by GetBucketId
   (Appendix B).  ``bucket_ids``, ``distribute_counting`` and ``distribute``.
3. Recursing (Section 3.3) into light buckets only; heavy buckets are final.
4. Dovetail merging (Section 3.4, Alg. 3) of each MSD zone.  ``dtmerge_inplace``
   follows Alg. 3 (copy the smaller side out, move buckets one by one with a
   direct copy or two flips, copy back); ``dtmerge_positions`` gives the closed
   form of where every heavy bucket ends.

Base cases (Section 3.5): no bits left, or n' at most the cutoff, which is
handed to a stable comparison sort (the method must stay stable).  With
``pair_leaves`` (the GPU path for 32-bit keys without values) a child
subproblem of at most twice the cutoff is a base case too: the GPU sorts its
two halves and merges them, a stable comparison sort of n' records.

Readings of points the paper leaves open (each listed in the design notes):
* digit width: gamma = clamp(floor((floor(log2 n') + 1) / 3), gmin, gmax), the
  paper's "log2 of the cube root of n, capped by 8 and 12" (Section 6) with an
  integer rounding, or a caller override;
* sample size: 2^gamma * t keys with t = ceil(log2 n) for the original size n
  (Section 3.1 asks for Theta(2^gamma log n)), t reduced so the sample fits a
  cap (32768 keys of 4 bytes, 16384 of 8 bytes), at least 1;
* sampling is with replacement at the positions of ``oracle.rng``;
* the subsample is S[0], S[t], S[2t], ... (2^gamma keys); a key is heavy when
  it occurs at least twice in the subsample;
* key range (Section 5): top = bit length of the sample maximum below ``hi``;
  keys with a one bit in [top, hi) go to the overflow bucket (last id); the
  overflow bucket recurses as a general subproblem with the skip turned off
  (so its digits start at ``hi``) instead of a comparison sort;
* the digit is bits [shift, shift + w) with w = min(gamma, top), shift = top - w;
* last digit: when hi <= gamma the whole remaining range is one plain digit
  (w = hi, shift = 0) and no sample is drawn; every light bucket then holds one
  key value, which is what heavy detection would have isolated anyway.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import rng


def bitlen(x: int) -> int:
    return int(x).bit_length()


def gamma_auto(n_sub: int, gmin: int = 8, gmax: int = 11) -> int:
    lg = bitlen(n_sub) - 1  # floor(log2 n')
    return max(gmin, min(gmax, (lg + 1) // 3))


@dataclass
class Config:
    seed: int = 0
    key_bytes: int = 4
    gamma: int = 0            # 0 = automatic
    gmin: int = 8
    gmax: int = 11
    cutoff: int = 16384       # base-case threshold (theta)
    plain: bool = False       # heavy-key detection off (the paper's "Plain" ablation)
    pair_leaves: bool = False  # children of at most 2 * cutoff records are base cases

    @property
    def sample_cap(self) -> int:
        return 32768 if self.key_bytes == 4 else 16384


@dataclass
class Plan:
    gamma: int
    hi: int
    top: int
    w: int
    shift: int
    heavy: np.ndarray                 # sorted distinct heavy keys
    sampled: bool
    t: int = 0
    sample: np.ndarray | None = None  # sorted sample S (when drawn)
    light_id: np.ndarray = field(default=None)  # L[z] for z in [0, 2^w], L[2^w] = overflow id

    @property
    def zones(self) -> int:
        return 1 << self.w

    @property
    def n_heavy(self) -> int:
        return int(self.heavy.size)

    @property
    def n_buckets(self) -> int:
        return self.zones + self.n_heavy + 1

    @property
    def overflow_id(self) -> int:
        return self.n_buckets - 1


def _mask(hi: int) -> int:
    return (1 << hi) - 1


def plan(keys: np.ndarray, hi: int, n_root: int, offset: int, level: int, cfg: Config,
         skip_disabled: bool = False) -> Plan:
    """Step 1 (Section 3.1, Alg. 2 sampling lines; Section 5 overflow bucket)."""
    n_sub = int(keys.size)
    g = cfg.gamma if cfg.gamma > 0 else gamma_auto(n_sub, cfg.gmin, cfg.gmax)
    if hi <= g:
        p = Plan(gamma=g, hi=hi, top=hi, w=hi, shift=0, heavy=np.zeros(0, keys.dtype), sampled=False)
    else:
        t = max(1, min(bitlen(max(n_root - 1, 1)), cfg.sample_cap >> g))
        s = t << g
        pos = rng.sample_positions(cfg.seed, offset, level, n_sub, s)
        S = np.sort(keys[pos], kind="stable")
        mx = int(S[-1]) & _mask(hi)
        top = hi if skip_disabled else bitlen(mx)
        w = min(g, top)
        shift = top - w
        if cfg.plain:
            heavy = np.zeros(0, keys.dtype)
        else:
            sub = S[::t][: 1 << g]                     # S[0], S[t], S[2t], ...
            vals, cnt = np.unique(sub, return_counts=True)
            heavy = vals[cnt >= 2]
        p = Plan(gamma=g, hi=hi, top=top, w=w, shift=shift, heavy=heavy, sampled=True, t=t, sample=S)
    # bucket ids in order: per zone one light bucket then its heavy keys ascending;
    # the overflow bucket last (Section 3.1 "merge h and l", Section 5).
    zones = p.zones
    hz = np.array([zone_of(int(h), p) for h in p.heavy], dtype=np.int64)
    L = np.zeros(zones + 1, dtype=np.int64)
    for z in range(zones + 1):
        L[z] = z + int(np.count_nonzero(hz < z))
    p.light_id = L
    return p


def make_plan(hi: int, top: int, w: int, shift: int, heavy) -> Plan:
    """A plan with given range and heavy keys (no sampling): used to check the
    bucket-id rule on hand-worked examples."""
    p = Plan(gamma=w, hi=hi, top=top, w=w, shift=shift,
             heavy=np.array(sorted(heavy), dtype=np.uint64), sampled=False)
    hz = np.array([zone_of(int(h), p) for h in p.heavy], dtype=np.int64)
    p.light_id = np.array([z + int(np.count_nonzero(hz < z)) for z in range((1 << w) + 1)], dtype=np.int64)
    return p


def zone_of(key: int, p: Plan) -> int:
    low = key & _mask(p.hi)
    return (low >> p.shift) & ((1 << p.w) - 1)


def bucket_id(key: int, p: Plan) -> int:
    """GetBucketId (Alg. 2): heavy id if the key is heavy, else its zone's light id;
    keys above the sampled range go to the overflow bucket (Section 5)."""
    low = int(key) & _mask(p.hi)
    if (low >> p.top) != 0:
        return p.overflow_id
    z = (low >> p.shift) & ((1 << p.w) - 1)
    j = int(np.searchsorted(p.heavy, key))
    if j < p.heavy.size and int(p.heavy[j]) == int(key):
        return z + 1 + j
    return int(p.light_id[z])


def bucket_ids(keys: np.ndarray, p: Plan) -> np.ndarray:
    return np.array([bucket_id(int(k), p) for k in keys.tolist()], dtype=np.int64)


def bucket_ids_np(keys: np.ndarray, p: Plan) -> np.ndarray:
    """Vectorised GetBucketId for larger inputs (same definition)."""
    k = keys.astype(np.uint64)
    low = k & np.uint64(_mask(p.hi)) if p.hi < 64 else k
    over = (low >> np.uint64(p.top)) != 0 if p.top < 64 else np.zeros(k.shape, bool)
    z = ((low >> np.uint64(p.shift)) & np.uint64((1 << p.w) - 1)).astype(np.int64)
    ids = p.light_id[z]
    if p.heavy.size:
        hk = p.heavy.astype(np.uint64)
        j = np.searchsorted(hk, k)
        jc = np.minimum(j, hk.size - 1)
        is_h = hk[jc] == k
        ids = np.where(is_h, z + 1 + jc, ids)
    return np.where(over, p.overflow_id, ids)


def distribute_counting(keys: np.ndarray, ids: np.ndarray, n_buckets: int, n_sub: int = 4,
                        values: np.ndarray | None = None):
    """Stable counting sort by bucket id (Appendix B): split into subarrays,
    count C[i][j], offsets X[i][j] = sum of C[i'][j'] over j' < j or
    (j' = j and i' < i), then every subarray writes its records in order."""
    n = keys.size
    bounds = np.linspace(0, n, n_sub + 1).astype(np.int64)
    C = np.zeros((n_sub, n_buckets), dtype=np.int64)
    for i in range(n_sub):
        C[i] = np.bincount(ids[bounds[i]:bounds[i + 1]], minlength=n_buckets)
    col_major = C.T.reshape(-1)                     # j-major, then i
    X = (np.cumsum(col_major) - col_major).reshape(n_buckets, n_sub).T
    out_k = np.empty_like(keys)
    out_v = None if values is None else np.empty_like(values)
    for i in range(n_sub):
        nxt = X[i].copy()
        for r in range(bounds[i], bounds[i + 1]):
            j = ids[r]
            out_k[nxt[j]] = keys[r]
            if values is not None:
                out_v[nxt[j]] = values[r]
            nxt[j] += 1
    counts = C.sum(axis=0)
    return out_k, out_v, counts


def distribute(keys: np.ndarray, ids: np.ndarray, n_buckets: int, values: np.ndarray | None = None):
    """The same stable counting sort, via a library stable sort by bucket id."""
    o = np.argsort(ids, kind="stable")
    counts = np.bincount(ids, minlength=n_buckets)
    return keys[o], (None if values is None else values[o]), counts


def dtmerge_positions(b0_keys: np.ndarray, heavy: np.ndarray, sizes: np.ndarray) -> np.ndarray:
    """Start of every heavy bucket in the merged zone (Alg. 3, first line):
    p_i = lower_bound(B0, h_i) + sum_{j<i} |B_j| (no light key equals a heavy key)."""
    lb = np.searchsorted(b0_keys, heavy, side="left")
    before = np.concatenate([[0], np.cumsum(sizes)[:-1]]) if sizes.size else np.zeros(0, np.int64)
    return lb + before


def _flip(a: np.ndarray, s: int, e: int):
    a[s:e] = a[s:e][::-1].copy()


def dtmerge_inplace(zone_k: np.ndarray, zone_v, b0_size: int, heavy: np.ndarray, sizes: np.ndarray):
    """Alg. 3 on one MSD zone stored as [B0 | B1 | ... | Bm] (modified in place).

    If B0 is not larger than all heavy buckets together, B0 goes to a temporary
    array, heavy buckets move left one by one (a direct copy, or two flips when
    a bucket's target overlaps its own current place), then B0's blocks go to the
    gaps.  Otherwise the heavy buckets go to the temporary array, B0's blocks
    move right one by one starting from the last (two flips on overlap), then
    the heavy buckets are copied into the gaps.
    """
    arrs = [zone_k] + ([zone_v] if zone_v is not None else [])
    m = heavy.size
    if m == 0:
        return
    p = dtmerge_positions(zone_k[:b0_size], heavy, sizes)
    lb = np.searchsorted(zone_k[:b0_size], heavy, side="left")
    if b0_size <= int(sizes.sum()):
        T = [a[:b0_size].copy() for a in arrs]
        cur = b0_size
        for i in range(m):
            s, sz = cur, int(sizes[i])
            if p[i] + sz > s:          # target overlaps the bucket's own place
                for a in arrs:
                    _flip(a, s, s + sz)
                    _flip(a, p[i], s + sz)
            else:
                for a in arrs:
                    a[p[i]:p[i] + sz] = a[s:s + sz].copy()
            cur += sz
        # light blocks: block k = B0[lb_k : lb_{k+1}] lands after k heavy buckets
        edges = np.concatenate([[0], lb, [b0_size]])
        shift = np.concatenate([[0], np.cumsum(sizes)])
        for k in range(m + 1):
            a0, a1 = int(edges[k]), int(edges[k + 1])
            for a, t in zip(arrs, T):
                a[a0 + shift[k]:a1 + shift[k]] = t[a0:a1]
    else:
        T = [a[b0_size:].copy() for a in arrs]
        edges = np.concatenate([[0], lb, [b0_size]])
        shift = np.concatenate([[0], np.cumsum(sizes)])
        for k in range(m, -1, -1):     # light blocks move right, the last one first
            a0, a1, d = int(edges[k]), int(edges[k + 1]), int(shift[k])
            if d == 0 or a1 == a0:
                continue
            if a0 + d < a1:            # target overlaps the block's own place: two flips
                for a in arrs:
                    _flip(a, a0, a1)
                    _flip(a, a0, a1 + d)
            else:
                for a in arrs:
                    a[a0 + d:a1 + d] = a[a0:a1].copy()
        start = 0
        for i in range(m):
            sz = int(sizes[i])
            for a, t in zip(arrs, T):
                a[p[i]:p[i] + sz] = t[start:start + sz]
            start += sz


def dtmerge_gather(b0_k: np.ndarray, b0_v, heavy: np.ndarray, heavy_vals: list, sizes: np.ndarray):
    """Out-of-place form of the same merge: output position q takes heavy
    bucket i if q in [p_i, p_i + |B_i|), else the next unused light record."""
    total = b0_k.size + int(sizes.sum())
    p = dtmerge_positions(b0_k, heavy, sizes)
    out_k = np.empty(total, dtype=b0_k.dtype)
    out_v = None if b0_v is None else np.empty(total, dtype=b0_v.dtype)
    is_heavy = np.zeros(total, bool)
    for i in range(heavy.size):
        sz = int(sizes[i])
        out_k[p[i]:p[i] + sz] = heavy[i]
        if out_v is not None:
            out_v[p[i]:p[i] + sz] = heavy_vals[i]
        is_heavy[p[i]:p[i] + sz] = True
    out_k[~is_heavy] = b0_k
    if out_v is not None:
        out_v[~is_heavy] = b0_v
    return out_k, out_v


@dataclass
class Stats:
    levels: int = 0
    tasks: int = 0
    heavy_keys: int = 0
    heavy_records: int = 0
    distributed: int = 0
    base_sorted: int = 0
    merged_zones: int = 0
    merged_records: int = 0
    overflow_records: int = 0


def dtsort(keys: np.ndarray, values: np.ndarray | None = None, cfg: Config | None = None,
           key_bits: int | None = None, stats: Stats | None = None):
    """Alg. 2 end to end (recursive); returns sorted (keys, values)."""
    cfg = cfg or Config(key_bytes=keys.dtype.itemsize)
    kb = key_bits if key_bits is not None else 8 * keys.dtype.itemsize
    st = stats if stats is not None else Stats()
    k = keys.copy()
    v = None if values is None else values.copy()
    _rec(k, v, 0, k.size, kb, k.size, 0, cfg, False, st)
    return k, v


def _rec(k, v, off, n, hi, n_root, level, cfg, skip_disabled, st):
    if n <= 1 or hi == 0:                                  # all bits sorted
        return
    base = cfg.cutoff * (2 if (cfg.pair_leaves and level > 0) else 1)
    if n <= base:                                          # base case: stable sort
        o = np.argsort(k[off:off + n], kind="stable")
        k[off:off + n] = k[off:off + n][o]
        if v is not None:
            v[off:off + n] = v[off:off + n][o]
        st.base_sorted += n
        return
    st.tasks += 1
    st.levels = max(st.levels, level + 1)
    st.distributed += n
    seg_k = k[off:off + n]
    p = plan(seg_k, hi, n_root, off, level, cfg, skip_disabled)
    ids = bucket_ids_np(seg_k, p)
    dk, dv, counts = distribute(seg_k, ids, p.n_buckets, None if v is None else v[off:off + n])
    k[off:off + n] = dk
    if v is not None:
        v[off:off + n] = dv
    starts = np.concatenate([[0], np.cumsum(counts)])
    st.heavy_keys += p.n_heavy
    st.overflow_records += int(counts[-1])
    # step 3: recurse into light buckets (and the overflow bucket)
    for z in range(p.zones):
        b = int(p.light_id[z])
        _rec(k, v, off + int(starts[b]), int(counts[b]), p.shift, n_root, level + 1, cfg, False, st)
    ob = p.overflow_id
    _rec(k, v, off + int(starts[ob]), int(counts[ob]), p.hi, n_root, level + 1, cfg, True, st)
    # step 4: dovetail-merge every zone that has heavy buckets
    for z in range(p.zones):
        b0 = int(p.light_id[z])
        m = int(p.light_id[z + 1]) - b0 - 1
        if m == 0:
            continue
        hidx = np.arange(b0 + 1, b0 + 1 + m)
        sizes = counts[hidx].astype(np.int64)
        hkeys = p.heavy[hidx - z - 1]
        zs, ze = off + int(starts[b0]), off + int(starts[b0 + m + 1])
        st.heavy_records += int(sizes.sum())
        st.merged_zones += 1
        st.merged_records += ze - zs
        zk = k[zs:ze]
        zv = None if v is None else v[zs:ze]
        dtmerge_inplace(zk, zv, int(counts[b0]), hkeys, sizes)
