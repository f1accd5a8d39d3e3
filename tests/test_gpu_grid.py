"""The record layout of the paper's 32-bit experiments (32-bit keys with
32-bit values, dtsort_pairs_u32) and the paper's synthetic grid (Section 6,
Tab. synthetic: Unif-mu, Exp-lambda, Zipf-s, BExp-t at both key widths),
bit-exact against the CPU oracle's stable order, with the method's heavy-key
detection on (SAMPLING) and off (the paper's Plain ablation, Section 6.3)."""
import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
import workloads as W
from oracle import sort as S
from tests._dev import dev_u32, dev_u64, host_u32, host_u64, require_gpu, say
from tests._seeds import seed_of

pytestmark = pytest.mark.gpu


def _pairs(k, bits, **kw):
    n = k.size
    if bits == 32:
        dk, dv = dev_u32(k), dev_u32(np.arange(n, dtype=np.uint32))
        st = dt.Stats()
        dt.sort_pairs_u32(dk, dv, dt.make_opts(stats=st, **kw))
        torch.cuda.synchronize()
        return host_u32(dk), host_u32(dv), st
    dk, dv = dev_u64(k), dev_u64(np.arange(n, dtype=np.uint64))
    st = dt.Stats()
    dt.sort_pairs_u64(dk, dv, dt.make_opts(stats=st, **kw))
    torch.cuda.synchronize()
    return host_u64(dk), host_u64(dv), st


def _check(k, bits, **kw):
    gk, gv, st = _pairs(k, bits, **kw)
    ek, ev = S.stable_sort_pairs(k, np.arange(k.size, dtype=np.uint32 if bits == 32 else np.uint64))
    assert np.array_equal(gk, ek), "keys differ from the oracle"
    assert np.array_equal(gv, ev), "values differ from the oracle (stability)"
    return st


@pytest.mark.parametrize("n", [0, 1, 2, 17, 2047, 8192, 16383, 16384, 16385, 32769, 65537, 300007])
def test_pairs_u32_sizes(n):
    require_gpu()
    say(f"pairs u32 n={n}")
    rs = np.random.default_rng(seed_of("pairs32", n))
    k = rs.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    _check(k, 32)
    k2 = (k % np.uint32(97)).astype(np.uint32)  # many equal keys: stability shows
    _check(k2, 32, digit_bits=5, lds_cutoff=700)


@pytest.mark.parametrize("params", [dict(graph=1), dict(tile_shape=2, ordered_ranks=1), dict(tuned=1),
                                    dict(mode=dt.MODE_LEARNED, tuned=1)])
def test_pairs_u32_forms(params):
    require_gpu()
    say(f"pairs u32 forms {params}")
    n = 1_500_001
    k = W.paper_keys("zipf", 1.0, n, 32, seed=3).numpy().astype(np.uint32)
    for rep in range(2 if params.get("graph") else 1):
        st = _check(k, 32, **params)
    if params.get("mode") == dt.MODE_LEARNED:
        assert st.sampling_balance > 0  # the judge ran (it trains only where a gain is predicted)


GRID = [(f, p) for f, ps in W.PAPER_GRID.items() for p in ps]


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("family,param", GRID)
def test_paper_grid_instances(family, param, bits):
    """Every instance of the grid at 2^20 + 3 records, in the tuned
    configuration the grid benchmark times, with detection on and off."""
    require_gpu()
    n = (1 << 20) + 3
    say(f"grid {family}-{param} bits={bits}")
    k = W.paper_keys(family, param, n, bits, seed=1).numpy()
    k = k.astype(np.uint32) if bits == 32 else k.view(np.uint64)
    st = _check(k, bits, tuned=1)
    stp = _check(k, bits, tuned=1, mode=dt.MODE_PLAIN)
    assert stp.heavy_keys == 0
    if family == "unif" and param <= 10:
        assert st.heavy_keys > 0  # few distinct keys: every one is heavy at the root
