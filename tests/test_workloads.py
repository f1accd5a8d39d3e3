"""The seeded input generators: determinism and the distribution shapes the
paper's synthetic workloads call for (Section 6, synthetic distributions)."""
import math

import numpy as np
import torch

import workloads as W


def test_deterministic_and_seeded():
    a = W.uniform_u32(1000, seed=3)
    assert torch.equal(a, W.uniform_u32(1000, seed=3))
    assert not torch.equal(a, W.uniform_u32(1000, seed=4))
    assert int(a.min()) >= 0 and int(a.max()) < 2 ** 32


def test_zipf_head_frequency():
    s, N = 1.0, 10 ** 9
    r = W.zipf_ranks(1 << 18, s, N, seed=1)
    Hn = sum(1.0 / i for i in range(1, 100000)) + math.log(N / 100000)   # harmonic number (tail by log)
    p1 = 1.0 / Hn
    share = float((r == 1).double().mean())
    assert abs(share - p1) < 4 * math.sqrt(p1 / (1 << 18))
    p2 = 0.5 / Hn
    assert abs(float((r == 2).double().mean()) - p2) < 4 * math.sqrt(p2 / (1 << 18))
    assert int(r.min()) >= 1 and int(r.max()) <= N


def test_zipf_steep_exponent():
    s, N = 1.5, 1000
    r = W.zipf_ranks(1 << 17, s, N, seed=2)
    Z = sum(k ** -s for k in range(1, N + 1))
    for k in (1, 2, 5):
        p = k ** -s / Z
        assert abs(float((r == k).double().mean()) - p) < 4 * math.sqrt(p / (1 << 17))


def test_exponential_mean():
    e = W.exponential_keys(1 << 18, 1e-5, seed=3)
    assert abs(float(e.double().mean()) - (1e5 - 0.5)) < 4 * 1e5 / math.sqrt(1 << 18)


def test_bit_exponential_lengths():
    b = W.bit_exponential_keys(1 << 16, 0.1, seed=4).numpy().view(np.uint64)
    bl = np.array([int(x).bit_length() for x in b.tolist()])
    # P(k) = 0.9^(k-1) 0.1 for k < 64
    for k in (1, 2, 10):
        p = 0.9 ** (k - 1) * 0.1
        assert abs(np.mean(bl == k) - p) < 4 * math.sqrt(p / b.size)
    assert bl.min() >= 1 and bl.max() <= 64


def test_feistel_bijective():
    x = torch.arange(0, 1 << 16, dtype=torch.int64) * 65521
    y = W.feistel32(x & 0xFFFFFFFF, 9)
    assert torch.unique(y).numel() == x.numel()
    assert int(y.min()) >= 0 and int(y.max()) < 2 ** 32
    y64 = W.feistel64(x, 9)
    assert torch.unique(y64).numel() == x.numel()


def test_segment_sizes_shape():
    s = W.segment_sizes(4096, seed=0)
    assert int(s.min()) >= 1000 and int(s.max()) <= 10 ** 7
    med = float(s.double().median())
    assert 0.8 * 2 ** 14 < med < 1.25 * 2 ** 14
    assert 1.5e8 < float(s.sum()) < 2.6e8


def test_make_config_small():
    for name in W.CONFIGS:
        c = W.make_config(name, n=5000, n_seg=32)
        assert c["keys"].numel() > 0
        if name == "segmented_u32":
            off = c["offsets"]
            assert int(off[0]) == 0 and int(off[-1]) == c["keys"].numel()


def test_paper_grid_unif_distinct_keys():
    """Unif-mu: at most mu distinct keys, all of them hit when n >> mu, spread
    over the whole key range by the bijection."""
    for bits in (32, 64):
        k = W.paper_keys("unif", 1000, 1 << 17, bits, seed=1).numpy().view(np.uint64)
        u = np.unique(k)
        assert u.size == 1000
        assert int(u.max()) > 2 ** (bits - 2)
        k7 = W.paper_keys("unif", 10, 4096, bits, seed=2)
        assert torch.unique(k7).numel() == 10


def test_paper_grid_exp_frequencies():
    """Exp-lambda: rounded exponential of rate 1e-5 lambda; the frequency of
    the rounded value 0 is P(X < 0.5) = 1 - exp(-0.5 rate); keys bijected."""
    n = 1 << 18
    for lam in (1, 10):
        rate = 1e-5 * lam
        k = W.paper_keys("exp", lam, n, 64, seed=3)
        inv = W.feistel64(torch.zeros(1, dtype=torch.int64), 3 * 131 + 17)  # the key of value 0
        p0 = 1 - math.exp(-0.5 * rate)
        share = float((k == inv[0]).double().mean())
        assert abs(share - p0) < 5 * math.sqrt(p0 / n) + 1e-6
    # the number of distinct keys is about the range of rounded values actually drawn
    k = W.paper_keys("exp", 10, n, 32, seed=4)
    assert 4000 < torch.unique(k).numel() < 60000


def test_paper_grid_zipf_head():
    n = 1 << 17
    k = W.paper_keys("zipf", 1.5, n, 32, seed=5)
    top = torch.unique(k, return_counts=True)[1].max().item() / n
    Z = sum(i ** -1.5 for i in range(1, 200000)) + 2 / math.sqrt(200000)
    assert abs(top - 1 / Z) < 5 * math.sqrt(1 / Z / n)


def test_paper_grid_bexp_bits():
    """BExp-t: every bit is 0 with probability 1/t, independently."""
    n = 1 << 16
    for bits, t in ((32, 10), (64, 300)):
        k = W.paper_keys("bexp", t, n, bits, seed=6).numpy().view(np.uint64)
        for b in (0, 1, bits // 2, bits - 1):
            zeros = np.mean(((k >> np.uint64(b)) & np.uint64(1)) == 0)
            assert abs(zeros - 1 / t) < 5 * math.sqrt((1 / t) / n), (bits, t, b)
        if bits == 32:
            assert int(k.max()) < 2 ** 32
    # all ones is the most frequent 32-bit key: P = (1 - 1/t)^32
    k = W.paper_keys("bexp", 10, n, 32, seed=7).numpy().view(np.uint64)
    p = 0.9 ** 32
    assert abs(np.mean(k == 2 ** 32 - 1) - p) < 5 * math.sqrt(p / n)


def test_paper_grid_chunks_deterministic(monkeypatch):
    """Generated in chunks: the result does not depend on the chunk size, and
    a prefix equals the same call at a smaller n."""
    from workloads import gen
    for fam, prm in (("unif", 10 ** 5), ("exp", 2), ("bexp", 30)):
        a = W.paper_keys(fam, prm, 5000, 64, seed=8)
        b = W.paper_keys(fam, prm, 3000, 64, seed=8)
        assert torch.equal(a[:3000], b)
        monkeypatch.setattr(gen, "_CHUNK", 777)
        assert torch.equal(W.paper_keys(fam, prm, 5000, 64, seed=8), a)
        monkeypatch.undo()


def test_power_law_graph_shape():
    V, E = 1 << 12, 200_000
    off, tgt = W.power_law_graph(V, E, seed=3)
    assert off.numel() == V + 1 and int(off[0]) == 0 and int(off[-1]) == E
    assert bool((off[1:] >= off[:-1]).all())
    assert int(tgt.min()) >= 0 and int(tgt.max()) < V
    indeg = torch.bincount(tgt, minlength=V)
    # Zipf(1) over 4096 vertices: the top vertex takes about 1/H_4096 ~ 11 % of the edges
    assert 0.09 < float(indeg.max()) / E < 0.14
    outdeg = off[1:] - off[:-1]
    assert int(outdeg.max()) > 20 * E // V  # skewed out-degrees too


def test_varden_points_range_and_density():
    p = W.varden_points(100_000, 2, seed=4)
    assert p.shape == (2, 100_000)
    assert int(p.min()) >= 0 and int(p.max()) < 1 << 16
    q = W.varden_points(50_000, 3, seed=5)
    assert int(q.max()) < 1 << 10
    # varying density: some grid cells are far fuller than the average
    cells = torch.bincount((p[0] >> 12) * 16 + (p[1] >> 12), minlength=256)
    assert int(cells.max()) > 4 * 100_000 // 256 and int(cells.min()) < 100_000 // 256 // 2
