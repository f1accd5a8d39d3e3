"""Step-level parity of the HIP path against the CPU oracle (bit-exact).

Each step entry point of the C ABI runs the production kernels on one
subproblem: Step 1 (sampling: digit range, heavy keys, bucket-id tables;
Section 3.1 and Section 5), Steps 1+2 (the stable counting sort by bucket id,
Section 3.2 / Appendix B), the base case (Section 3.5) and Step 4 (the
dovetail merge, Alg. 3).  The oracle computes the same step on the same
seeded input; everything is integer, so results must be identical.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import dtsort_ref as R
from oracle import sort as S
from tests._dev import dev_u32, dev_u64, host_u32, host_u64, require_gpu, say
from tests._seeds import seed_of

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2401_00710_amd._lib as L
    return L.load()


def _opts(seed=0, digit_bits=0, plain=False):
    import paper_2401_00710_amd as dt
    return dt.make_opts(seed=seed, digit_bits=digit_bits, mode=dt.MODE_PLAIN if plain else dt.MODE_SAMPLING)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _inputs(kind, n, rs, wide):
    if kind == "uniform":
        k = rs.integers(0, 2 ** 64 if wide else 2 ** 32, n, dtype=np.uint64)
    elif kind == "zipf":
        k = (rs.zipf(1.1, n) * 2654435761) % (2 ** 32)
    elif kind == "small_range":
        k = rs.integers(0, 3000, n)
    elif kind == "equal":
        k = np.full(n, 12345, np.uint64)
    elif kind == "exp":
        k = rs.exponential(2e4, n).astype(np.uint64)
    elif kind == "top_bits":
        k = rs.integers(0, 2 ** 20, n, dtype=np.uint64)
        k[rs.integers(0, n, 5)] = (2 ** 63 if wide else 2 ** 31) + 7
    else:
        raise KeyError(kind)
    return k.astype(np.uint64 if wide else np.uint32)


CASES = [(kind, wide, g, plain) for kind in ["uniform", "zipf", "small_range", "equal", "exp", "top_bits"]
         for wide in (False, True) for (g, plain) in [(0, False), (4, False), (9, True)]]


def _oracle_plan(keys, hi, seed, g, plain, wide, skip=False):
    cfg = R.Config(seed=seed, key_bytes=8 if wide else 4, gamma=g, plain=plain)
    return R.plan(keys, hi, keys.size, 0, 0, cfg, skip_disabled=skip)


def _gpu_plan(keys, hi, seed, g, plain, wide, skip=False):
    lib = _lib()
    n = keys.size
    d = dev_u64(keys) if wide else dev_u32(keys)
    plan = np.zeros(6, np.int32)
    heavy = np.zeros(1024, np.uint64 if wide else np.uint32)
    light = np.zeros(2049, np.uint32)
    o = _opts(seed, g, plain)
    f = lib.dtsort_step_plan_u64 if wide else lib.dtsort_step_plan_u32
    st = f(d.data_ptr(), n, hi, int(skip), C.byref(o), plan.ctypes.data, heavy.ctypes.data, light.ctypes.data,
           _stream())
    assert st == 0
    return plan, heavy[:plan[4]], light[:(1 << plan[1]) + 1]


@pytest.mark.parametrize("kind,wide,g,plain", CASES)
def test_step_plan(kind, wide, g, plain):
    require_gpu()
    sd = seed_of(kind, wide, g)
    say(f"seed={sd}")
    rs = np.random.default_rng(sd)
    n = 200000
    keys = _inputs(kind, n, rs, wide)
    hi = 64 if wide else 32
    for seed in (0, 7):
        say(f"plan kind={kind} wide={wide} g={g} plain={plain} seed={seed}")
        p = _oracle_plan(keys, hi, seed, g, plain, wide)
        plan, heavy, light = _gpu_plan(keys, hi, seed, g, plain, wide)
        assert list(plan[:5]) == [p.gamma, p.w, p.shift, p.top, p.n_heavy]
        assert plan[5] == p.n_buckets
        assert list(heavy) == [int(h) for h in p.heavy]
        assert list(light) == [int(v) for v in p.light_id]


def test_step_plan_skip_and_lower_hi():
    require_gpu()
    rs = np.random.default_rng(3)
    keys = rs.integers(0, 2 ** 20, 100000).astype(np.uint32)
    for hi, skip in [(20, False), (20, True), (24, True), (9, False), (3, False)]:
        say(f"plan hi={hi} skip={skip}")
        p = _oracle_plan(keys & np.uint32((1 << hi) - 1) if hi < 20 else keys, hi, 0, 0, False, False, skip)
        src = keys & np.uint32((1 << hi) - 1) if hi < 20 else keys
        plan, heavy, light = _gpu_plan(src, hi, 0, 0, False, False, skip)
        assert list(plan[:5]) == [p.gamma, p.w, p.shift, p.top, p.n_heavy]
        assert list(light) == [int(v) for v in p.light_id]


@pytest.mark.parametrize("kind,wide,g,plain", CASES[::2])
def test_step_distribute(kind, wide, g, plain):
    require_gpu()
    lib = _lib()
    sd = seed_of("d", kind, wide, g)
    say(f"seed={sd}")
    rs = np.random.default_rng(sd)
    n = 300001
    keys = _inputs(kind, n, rs, wide)
    hi = 64 if wide else 32
    vals = np.arange(n, dtype=np.uint64 if wide else np.uint32)
    say(f"distribute kind={kind} wide={wide} g={g} plain={plain}")
    p = _oracle_plan(keys, hi, 0, g, plain, wide)
    ids = R.bucket_ids_np(keys, p)
    ek, ev, ecnt = R.distribute(keys, ids, p.n_buckets, values=vals)
    dk = dev_u64(keys) if wide else dev_u32(keys)
    dv = dev_u64(vals) if wide else dev_u32(vals)
    ok = torch.empty_like(dk)
    ov = torch.empty_like(dv)
    counts = np.zeros(4097, np.uint32)
    plan = np.zeros(6, np.int32)
    heavy = np.zeros(1024, np.uint64 if wide else np.uint32)
    light = np.zeros(2049, np.uint32)
    o = _opts(0, g, plain)
    f = lib.dtsort_step_distribute_u64 if wide else lib.dtsort_step_distribute_u32
    st = f(dk.data_ptr(), dv.data_ptr(), n, hi, C.byref(o), ok.data_ptr(), ov.data_ptr(), counts.ctypes.data,
           plan.ctypes.data, heavy.ctypes.data, light.ctypes.data, _stream())
    assert st == 0
    assert plan[5] == p.n_buckets
    assert np.array_equal(counts[:p.n_buckets], ecnt)
    h = host_u64 if wide else host_u32
    assert np.array_equal(h(ok), ek)
    assert np.array_equal(h(ov), ev)
    # keys only with ordered ranks: the oracle's order
    o.ordered_ranks = 1
    ok2 = torch.empty_like(dk)
    st = f(dk.data_ptr(), None, n, hi, C.byref(o), ok2.data_ptr(), None, counts.ctypes.data, plan.ctypes.data,
           heavy.ctypes.data, light.ctypes.data, _stream())
    assert st == 0 and np.array_equal(h(ok2), ek)
    # keys only with unordered ranks (the default): the same buckets, each
    # holding the oracle's keys in some order
    o.ordered_ranks = 0
    ok3 = torch.empty_like(dk)
    st = f(dk.data_ptr(), None, n, hi, C.byref(o), ok3.data_ptr(), None, counts.ctypes.data, plan.ctypes.data,
           heavy.ctypes.data, light.ctypes.data, _stream())
    assert st == 0 and np.array_equal(counts[:p.n_buckets], ecnt)
    bidx = np.repeat(np.arange(p.n_buckets), ecnt.astype(np.int64))
    got3 = h(ok3)
    assert np.array_equal(got3[np.lexsort((got3, bidx))], ek[np.lexsort((ek, bidx))])


@pytest.mark.parametrize("wide,vals", [(False, False), (False, True), (True, False), (True, True)])
def test_step_leaf(wide, vals):
    require_gpu()
    lib = _lib()
    rs = np.random.default_rng(11)
    cap = 8192 if (wide and vals) else 16384
    sizes = [1, 2, 3, 63, 64, 65, 1000, 2047, 2048, 2049, 5000, 8191, 8192, cap - 1, cap, 0, 17]
    sizes = [s for s in sizes if s <= cap]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    n = int(off[-1])
    bits = 64 if wide else 32
    keys = rs.integers(0, 2 ** bits, n, dtype=np.uint64).astype(np.uint64 if wide else np.uint32)
    keys[:3000] = keys[:3000] % np.array(97, keys.dtype)           # ties
    v = np.arange(n, dtype=np.uint64 if wide else np.uint32)
    exp_k, exp_v = S.segmented_sort(keys, off, v)
    dk = dev_u64(keys) if wide else dev_u32(keys)
    dv = (dev_u64(v) if wide else dev_u32(v)) if vals else None
    do = dev_u64(off)
    ok = torch.empty_like(dk)
    ov = torch.empty_like(dv) if vals else None
    say(f"leaf wide={wide} vals={vals}")
    f = lib.dtsort_step_leaf_u64 if wide else lib.dtsort_step_leaf_u32
    st = f(dk.data_ptr(), dv.data_ptr() if vals else None, do.data_ptr(), len(sizes), bits, ok.data_ptr(),
           ov.data_ptr() if vals else None, _stream())
    assert st == 0
    h = host_u64 if wide else host_u32
    assert np.array_equal(h(ok), exp_k)
    if vals:
        assert np.array_equal(h(ov), exp_v)


def _prefix_case(kind, rs, wide):
    """Leaves whose keys differ in more than 16 bits, built to exercise the
    prefix sort and its run fix-up: runs of equal top-16-bit prefix of chosen
    lengths (FIX_MAX = 32 is the longest run the fix-up sorts; longer runs with
    a descent take the full radix passes), and runs of equal keys."""
    bits = 64 if wide else 32
    hb = bits - 16
    sizes = [4096, 4096, 300, 1000, 777]
    parts = []
    for i, sz in enumerate(sizes):
        low = rs.integers(0, 2 ** hb, sz, dtype=np.uint64)
        if kind == "unique":       # prefixes (nearly) unique: few or no runs to fix
            pre = rs.integers(0, 2 ** 16, sz, dtype=np.uint64)
        elif kind == "run32":      # runs of exactly 32 equal prefixes, lows out of order
            pre = np.repeat(rs.choice(2 ** 16, sz // 32 + 1, replace=False).astype(np.uint64), 32)[:sz]
        elif kind == "run33":      # runs of 33: the fix-up must give way to full passes
            pre = np.repeat(rs.choice(2 ** 16, sz // 33 + 1, replace=False).astype(np.uint64), 33)[:sz]
        elif kind == "few":        # four prefixes, random lows: long runs
            pre = rs.choice(np.array([5, 6, 900, 65535], np.uint64), sz)
        else:                      # duplicates: 50 distinct keys repeated (runs hold no descent)
            dist = rs.integers(0, 2 ** bits, 50, dtype=np.uint64)
            parts.append(rs.choice(dist, sz))
            continue
        parts.append((pre << np.uint64(hb)) | low)
    keys = np.concatenate(parts).astype(np.uint64 if wide else np.uint32)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    return keys, off, bits


@pytest.mark.parametrize("kind", ["unique", "run32", "run33", "few", "dups"])
@pytest.mark.parametrize("wide", [False, True])
def test_step_leaf_prefix_fixup(kind, wide):
    require_gpu()
    lib = _lib()
    rs = np.random.default_rng(77)
    keys, off, bits = _prefix_case(kind, rs, wide)
    n = keys.size
    v = np.arange(n, dtype=np.uint64 if wide else np.uint32)
    exp_k, exp_v = S.segmented_sort(keys, off, v)
    dk = dev_u64(keys) if wide else dev_u32(keys)
    dv = dev_u64(v) if wide else dev_u32(v)
    do = dev_u64(off)
    ok, ov = torch.empty_like(dk), torch.empty_like(dv)
    say(f"leaf prefix fix-up {kind} wide={wide}")
    f = lib.dtsort_step_leaf_u64 if wide else lib.dtsort_step_leaf_u32
    assert f(dk.data_ptr(), dv.data_ptr(), do.data_ptr(), len(off) - 1, bits, ok.data_ptr(), ov.data_ptr(),
             _stream()) == 0
    h = host_u64 if wide else host_u32
    assert np.array_equal(h(ok), exp_k)
    assert np.array_equal(h(ov), exp_v)


@pytest.mark.parametrize("seed", range(6))
def test_step_dtmerge(seed):
    require_gpu()
    lib = _lib()
    rs = np.random.default_rng(100 + seed)
    m = int(rs.integers(1, 40)) if seed < 5 else 512
    heavy = np.sort(rs.choice(2 ** 40, m, replace=False)).astype(np.uint64) * np.uint64(2)
    nb0 = [0, 1, 5000, 100000, 33333, 20000][seed]
    b0 = np.sort(rs.integers(0, 2 ** 40, nb0).astype(np.uint64) * np.uint64(2) + np.uint64(1))
    sizes = rs.integers(1, 9000, m).astype(np.uint32)
    b0v = rs.integers(0, 2 ** 63, nb0, dtype=np.uint64)
    hv_list = [rs.integers(0, 2 ** 63, s, dtype=np.uint64) for s in sizes]
    hv = np.concatenate(hv_list) if m else np.zeros(0, np.uint64)
    ek, ev = R.dtmerge_gather(b0, b0v, heavy, hv_list, sizes.astype(np.int64))
    zs = ek.size
    ok = torch.empty(zs, dtype=torch.int64, device="cuda")
    ov = torch.empty(zs, dtype=torch.int64, device="cuda")
    d_b0 = dev_u64(b0) if nb0 else torch.empty(1, dtype=torch.int64, device="cuda")
    d_b0v = dev_u64(b0v) if nb0 else torch.empty(1, dtype=torch.int64, device="cuda")
    d_hv = dev_u64(hv)
    say(f"dtmerge seed={seed} m={m} b0={nb0}")
    st = lib.dtsort_step_dtmerge_u64(d_b0.data_ptr(), d_b0v.data_ptr(), nb0, heavy.ctypes.data, sizes.ctypes.data,
                                     m, d_hv.data_ptr(), ok.data_ptr(), ov.data_ptr(), _stream())
    assert st == 0
    assert np.array_equal(host_u64(ok), ek)
    assert np.array_equal(host_u64(ov), ev)


# Zone layouts whose gather units (4096 outputs each) lie wholly inside one
# heavy run, wholly inside one stretch of light records, or straddle a
# boundary, with run ends on unit edges: the gather fills a unit inside a run
# with the run's key and copies a unit inside a light stretch as one shifted
# range, and searches the run starts per output only in straddling units.
# Heavy keys are even and light keys odd, so none is equal.
_RUN_LAYOUTS = {
    "runs_on_unit_edges": (0, [(10, 4096), (20, 8192), (30, 4096)]),
    "one_long_run_inside_light": (30000, [(2 ** 39, 50000)]),
    "light_starts_on_unit_edge": (3 * 4096, [(2, 4095), (4, 1)]),
    "runs_above_all_light": (10000, [(2 ** 42 + 2 * i, 12289 + 4096 * i) for i in range(5)]),
    "light_between_long_runs": (9000, [(2, 9000), (2 ** 42, 4097)]),
}


@pytest.mark.parametrize("layout", sorted(_RUN_LAYOUTS))
def test_step_dtmerge_runs(layout):
    require_gpu()
    lib = _lib()
    nb0, runs = _RUN_LAYOUTS[layout]
    rs = np.random.default_rng(seed_of("dtmerge_runs", layout))
    heavy = np.array([h for h, _ in runs], np.uint64)
    sizes = np.array([c for _, c in runs], np.uint32)
    b0 = np.sort(rs.integers(0, 2 ** 40, nb0).astype(np.uint64) * np.uint64(2) + np.uint64(1))
    b0v = rs.integers(0, 2 ** 63, nb0, dtype=np.uint64)
    hv_list = [rs.integers(0, 2 ** 63, int(c), dtype=np.uint64) for c in sizes]
    ek, ev = R.dtmerge_gather(b0, b0v, heavy, hv_list, sizes.astype(np.int64))
    zs = ek.size
    ok = torch.empty(zs, dtype=torch.int64, device="cuda")
    ov = torch.empty(zs, dtype=torch.int64, device="cuda")
    d_b0 = dev_u64(b0) if nb0 else torch.empty(1, dtype=torch.int64, device="cuda")
    d_b0v = dev_u64(b0v) if nb0 else torch.empty(1, dtype=torch.int64, device="cuda")
    d_hv = dev_u64(np.concatenate(hv_list))
    say(f"dtmerge runs {layout}: b0={nb0} runs={[int(c) for c in sizes]}")
    st = lib.dtsort_step_dtmerge_u64(d_b0.data_ptr(), d_b0v.data_ptr(), nb0, heavy.ctypes.data, sizes.ctypes.data,
                                     len(runs), d_hv.data_ptr(), ok.data_ptr(), ov.data_ptr(), _stream())
    assert st == 0
    assert np.array_equal(host_u64(ok), ek)
    assert np.array_equal(host_u64(ov), ev)
