"""The copy kernel the sorts use for finished buckets (16-byte words when the
two ranges share their alignment, record by record otherwise), through
dtsort_copy_u32 and through sorts whose finished buckets end in the partner
buffer, with caller arrays that start off a 16-byte boundary."""
import numpy as np
import pytest
import torch

import paper_2401_00710_amd as dt
import workloads as W
from oracle import sort as S
from tests._dev import dev_u32, dev_u64, host_u32, host_u64, require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,so,do", [(1, 0, 0), (3, 1, 2), (17, 3, 0), (65536, 0, 0), (65537, 1, 1),
                                     (65536 * 3 + 5, 2, 3), (1_000_003, 0, 1), (4_194_311, 3, 3)])
def test_copy_u32(n, so, do):
    require_gpu()
    say(f"copy n={n} src_off={so} dst_off={do}")
    rs = np.random.default_rng(n + 7 * so + 13 * do)
    a = rs.integers(0, 2 ** 32, n + 8, dtype=np.uint64).astype(np.uint32)
    src = dev_u32(a)
    dst = torch.full((n + 8,), -1, dtype=torch.int32, device="cuda")
    dt.copy_u32(dst[do:do + n], src[so:so + n])
    torch.cuda.synchronize()
    got = host_u32(dst)
    assert np.array_equal(got[do:do + n], a[so:so + n])
    assert (got[:do] == 0xFFFFFFFF).all() and (got[do + n:] == 0xFFFFFFFF).all(), "wrote outside the range"


@pytest.mark.parametrize("off", [0, 1, 3])
def test_sort_with_copies_at_offsets(off):
    """Exponential keys (about 21 significant bits) need three levels at the
    default digit width; the last one's finished buckets are copied back from
    the partner buffer.  The arrays start `off` records into a tensor."""
    require_gpu()
    n = 3_000_017
    k = W.exponential_keys(n, 1e-5, seed=off).numpy().view(np.uint64)
    say(f"pairs with copies off={off}")
    kd = torch.zeros(n + 4, dtype=torch.int64, device="cuda")
    vd = torch.zeros(n + 4, dtype=torch.int64, device="cuda")
    kd[off:off + n] = dev_u64(k)
    vd[off:off + n] = torch.arange(n, dtype=torch.int64, device="cuda")
    st = dt.Stats()
    dt.sort_pairs_u64(kd[off:off + n], vd[off:off + n], dt.make_opts(stats=st, digit_bits=8, lds_cutoff=64))
    torch.cuda.synchronize()
    ek, ev = S.stable_sort_pairs(k, np.arange(n, dtype=np.uint64))
    assert st.records_copied > 0, "the case is meant to exercise copies"
    assert np.array_equal(host_u64(kd)[off:off + n], ek)
    assert np.array_equal(host_u64(vd)[off:off + n], ev)
    k32 = (k & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    d32 = torch.zeros(n + 4, dtype=torch.int32, device="cuda")
    d32[off:off + n] = dev_u32(k32)
    st2 = dt.Stats()
    dt.sort_u32(d32[off:off + n], dt.make_opts(stats=st2, digit_bits=8, lds_cutoff=64))
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(d32)[off:off + n], np.sort(k32, kind="stable"))
