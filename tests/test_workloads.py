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
