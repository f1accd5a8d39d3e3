"""Parity at the benchmark's full sizes, in the configuration bench.py times
(tuned parameters, the same seeded inputs).

At 10^9 records the CPU oracle cannot sort the input in test time, so each
output is checked against what holds at any size and what the oracle can
compute one by one:
* 32/64-bit keys (the 64-bit mixture both with the learned partitioner and
  with sampling, whose tuned 9-bit digits run on a variant of their own):
  non-decreasing, the same multiset as the input (the oracle's
  order-independent digest, taken chunk by chunk), and the exact order
  statistics at sampled positions (numpy's selection on the input);
* pairs with values = original index: keys non-decreasing, every output key
  equals the input key its value points to, the values are a permutation of
  0..n-1, and equal keys keep increasing values — together exactly the
  unique stable order;
* the batched workload (2e8 keys): element by element against the oracle.
"""
import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
import workloads as W
from oracle import sort as S
from tests._dev import require_gpu, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 10 ** 9
CHUNK = 1 << 26


def _digest(a: np.ndarray):
    """The oracle's multiset digest, combined over chunks (count and sum add,
    xor xors: the digest of the whole array)."""
    c, s, x = 0, 0, 0
    for i in range(0, a.size, CHUNK):
        ci, si, xi = S.multiset_hash(a[i:i + CHUNK])
        c, s, x = c + ci, (s + si) % (1 << 64), x ^ xi
    return c, s, x


def _nondecreasing(a: np.ndarray) -> bool:
    for i in range(0, a.size - 1, CHUNK):
        seg = a[i:i + CHUNK + 1]
        if not np.all(seg[1:] >= seg[:-1]):
            return False
    return True


def _host(t: torch.Tensor, dtype) -> np.ndarray:
    return t.cpu().numpy().view(dtype)


def _check_keys(inp: np.ndarray, out: np.ndarray, seed: int):
    say("  sorted")
    assert _nondecreasing(out)
    say("  digest")
    assert _digest(out) == _digest(inp)
    say("  order statistics")
    rs = np.random.default_rng(seed)
    qs = np.unique(np.concatenate([[0, inp.size - 1, inp.size // 2], rs.integers(0, inp.size, 5)]))
    ref = np.partition(inp, qs)[qs]
    assert np.array_equal(out[qs], ref)


@pytest.mark.parametrize("kind,mv", [("uniform", 0), ("zipf1", 0), ("zipf1", dt.MERGE_SPLIT)])
def test_full_u32(kind, mv):
    """mv = MERGE_SPLIT: dovetailing during distribution (no merges)."""
    require_gpu()
    say(f"full u32 {kind} merge_variant={mv}: generate")
    if kind == "uniform":
        src = W.uniform_u32(N, seed=0, device="cuda").to(torch.int32)
    else:
        src = W.zipf_u32(N, 1.0, N, seed=0, device="cuda").to(torch.int32)
    inp = _host(src, np.uint32)
    say("  sort")
    st = dt.Stats()
    dt.sort_u32(src, dt.make_opts(tuned=1, merge_variant=mv, stats=st))
    if mv == dt.MERGE_SPLIT:
        assert st.merges == 0 and st.heavy_keys > 0
    torch.cuda.synchronize()
    out = _host(src, np.uint32)
    del src
    torch.cuda.empty_cache()
    _check_keys(inp, out, 1)


@pytest.mark.timeout(900)
def test_full_u32_beyond_2p31():
    """2^31 + 3 keys: task sizes, chunk ends and scatter places above 2^31
    (unsigned 32-bit arithmetic throughout; the interface admits n < 2^32)."""
    require_gpu()
    n = (1 << 31) + 3
    say(f"u32 n={n}: generate")
    src = W.uniform_u32(n, seed=5, device="cuda").to(torch.int32)
    inp = _host(src, np.uint32)
    say("  sort")
    st = dt.Stats()
    dt.sort_u32(src, dt.make_opts(tuned=1, stats=st))
    torch.cuda.synchronize()
    out = _host(src, np.uint32)
    del src
    torch.cuda.empty_cache()
    assert st.records_distributed >= n
    _check_keys(inp, out, 3)


@pytest.mark.parametrize("kind,mode", [("exp", "sampling"), ("bexp", "sampling"), ("bexp", "learned"),
                                       ("bexp", "split")])
def test_full_pairs_u64(kind, mode):
    """mode "split": sampling with dovetailing during distribution."""
    require_gpu()
    say(f"full pairs {kind} {mode}: generate")
    k = (W.exponential_keys(N, 1e-5, seed=0, device="cuda") if kind == "exp"
         else W.bit_exponential_keys(N, 0.1, seed=0, device="cuda"))
    v = torch.arange(N, dtype=torch.int64, device="cuda")
    inp = _host(k, np.uint64)
    say("  sort")
    st = dt.Stats()
    m = dt.MODE_LEARNED if mode == "learned" else dt.MODE_SAMPLING
    mv = dt.MERGE_SPLIT if mode == "split" else dt.MERGE_GATHER
    dt.sort_pairs_u64(k, v, dt.make_opts(tuned=1, mode=m, merge_variant=mv, stats=st))
    torch.cuda.synchronize()
    if mode == "split":
        assert st.merges == 0 and st.heavy_keys > 0
    if mode == "learned":
        # the benchmark reports this configuration with the model's zones in use
        say(f"  learned_used={st.learned_used} balance {st.learned_balance:.2f} vs {st.sampling_balance:.2f}")
        assert st.learned_used == 1
    ok, ov = _host(k, np.uint64), _host(v, np.uint64)
    del k, v
    torch.cuda.empty_cache()
    say("  sorted")
    assert _nondecreasing(ok)
    say("  values: a permutation")
    seen = np.zeros(N, dtype=bool)
    seen[ov] = True
    assert seen.all()
    del seen
    say("  keys follow their values")
    for i in range(0, N, CHUNK):
        assert np.array_equal(ok[i:i + CHUNK], inp[ov[i:i + CHUNK]])
    say("  stable")
    for i in range(0, N - 1, CHUNK):
        kk, vv = ok[i:i + CHUNK + 1], ov[i:i + CHUNK + 1]
        eq = kk[1:] == kk[:-1]
        assert np.all(vv[1:][eq] > vv[:-1][eq])


@pytest.mark.parametrize("mode", ["learned", "learned_forced", "sampling"])
def test_full_mixture_u64(mode):
    """learned: the cost judge decides (its decision must follow its own
    predicted costs); learned_forced: the model's zones in use, so that the
    learned root's levels run at full size."""
    require_gpu()
    say(f"full mixture u64, {mode}: generate")
    src = W.mixture_u64(N, seed=0, device="cuda")
    inp = _host(src, np.uint64)
    st = dt.Stats()
    say("  sort")
    m = dt.MODE_SAMPLING if mode == "sampling" else dt.MODE_LEARNED
    dt.sort_u64(src, dt.make_opts(tuned=1, mode=m, stats=st, learned_judge=1 if mode == "learned_forced" else 0))
    torch.cuda.synchronize()
    out = _host(src, np.uint64)
    del src
    torch.cuda.empty_cache()
    say(f"  learned_trained={st.learned_trained} used={st.learned_used} costs digit {st.sampling_cost:.3g} "
        f"learned {st.learned_cost:.3g} ideal {st.ideal_cost:.3g}")
    if mode == "learned_forced":
        assert st.learned_used == 1
    if mode == "learned":
        assert st.learned_trained == (st.sampling_cost > 1.25 * st.ideal_cost)
        assert st.learned_used == (st.learned_trained == 1 and st.learned_cost < 0.9 * st.sampling_cost)
    _check_keys(inp, out, 2)


@pytest.mark.parametrize("graph", [0, 1])
def test_full_batched(graph):
    require_gpu()
    say(f"full batched graph={graph}: generate")
    c = W.make_config("segmented_u32", seed=0, device="cuda")
    keys, off = c["keys"].to(torch.int32), c["offsets"]
    inp = _host(keys, np.uint32)
    offs = off.cpu().numpy().view(np.uint64)
    say("  sort")
    dt.sort_segmented(keys, off, opts=dt.make_opts(tuned=1, graph=graph))
    torch.cuda.synchronize()
    out = _host(keys, np.uint32)
    say("  oracle")
    ek, _ = S.segmented_sort(inp, offs)
    assert np.array_equal(out, ek)
