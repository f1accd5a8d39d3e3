"""Learned partitioner in float64 (not part of the paper; TEST INFRASTRUCTURE ONLY).

A CDF model y = F(x) for x in [0, 1] (keys normalised by the sample's range),
y = rank fraction.  Architecture 1 -> 64 -> 64 -> 1:

    h1 = relu(W1 x + b1)          W1: 64x1
    h2 = relu(W2 h1 + b2)         W2: 64x64 (row = output unit)
    yhat = W3 . h2 + b3           W3: 1x64

Inputs: the log-linear transform t(k) of a key (one unit per binary order of
magnitude, linear inside it), rescaled to [0, 1] over the training sample.

Flat parameter order: W1[64], b1[64], W2[64*64] (row-major [out][in]),
b2[64], W3[64], b3[1] -> 4353 values.

Loss: mean squared error over a batch.  Optimiser: Adam (Kingma & Ba 2015):
m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr (m / (1-b1^t)) /
(sqrt(v / (1-b2^t)) + eps).

Batches: step s uses the strided subsample {j * (N/B) + (s mod N/B) : j < B}
of the N sorted training keys, so every batch spans the whole key range.

Initial weights: u_i = (r_i >> 11) 2^-53 with r_i = mix64(h + (i+1) G),
h = mix64(mix64(seed + G) ^ 0x4D4C50); per hidden unit j of layer 1 a kink at
a_j = u, a slope magnitude sqrt(6) (0.5 + 0.5 u') and sign from u'' (< 0.5 ->
negative): W1_j = slope, b1_j = -slope * a_j; W2 and W3 are (2u - 1)
sqrt(6 / 64); b2 = 0, b3 = 0.5.  Parameter index i draws u_{3i}, u_{3i+1},
u_{3i+2} where it needs more than one uniform.

Splitters: predictions p_i on the sorted sample, made monotone by a running
maximum; splitter b (1 <= b < B) is the first sample key whose monotone
prediction reaches b / B (one past the largest key if none does), then made
non-decreasing.  Zone of a key = number of splitters <= key.

Balance error: max over zones of (light held-out keys in the zone) divided by
(light held-out keys / B).
"""
from __future__ import annotations

import math

import numpy as np

from .rng import G, mix64_int

H = 64
N_PARAMS = 64 + 64 + 64 * 64 + 64 + 64 + 1
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 64, 128, 128 + 4096, 128 + 4096 + 64, 128 + 4096 + 128


def _u(h: int, i: int) -> float:
    r = mix64_int(h + (i + 1) * G)
    return (r >> 11) * (2.0 ** -53)


def init_params(seed: int) -> np.ndarray:
    h = mix64_int(mix64_int(seed + G) ^ 0x4D4C50)
    p = np.zeros(N_PARAMS, dtype=np.float64)
    s6 = math.sqrt(6.0)
    s664 = math.sqrt(6.0 / 64.0)
    for j in range(H):
        i = OFF_W1 + j
        a = _u(h, 3 * i)
        mag = s6 * (0.5 + 0.5 * _u(h, 3 * i + 1))
        sgn = -1.0 if _u(h, 3 * i + 2) < 0.5 else 1.0
        slope = sgn * mag
        p[OFF_W1 + j] = slope
        p[OFF_B1 + j] = -slope * a
    for k in range(64 * 64):
        i = OFF_W2 + k
        p[i] = (2.0 * _u(h, 3 * i) - 1.0) * s664
    for j in range(H):
        i = OFF_W3 + j
        p[i] = (2.0 * _u(h, 3 * i) - 1.0) * s664
    p[OFF_B3] = 0.5
    return p


def unpack(p: np.ndarray):
    W1 = p[OFF_W1:OFF_W1 + 64]
    b1 = p[OFF_B1:OFF_B1 + 64]
    W2 = p[OFF_W2:OFF_W2 + 4096].reshape(64, 64)
    b2 = p[OFF_B2:OFF_B2 + 64]
    W3 = p[OFF_W3:OFF_W3 + 64]
    b3 = p[OFF_B3]
    return W1, b1, W2, b2, W3, b3


def forward(p: np.ndarray, x: np.ndarray):
    W1, b1, W2, b2, W3, b3 = unpack(p.astype(np.float64))
    x = x.astype(np.float64)
    z1 = np.outer(x, W1) + b1            # [N,64]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2                  # [N,64]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y, (x, z1, h1, z2, h2)


def loss(p: np.ndarray, x: np.ndarray, y: np.ndarray) -> float:
    yh, _ = forward(p, x)
    return float(np.mean((yh - y.astype(np.float64)) ** 2))


def loss_and_grad(p: np.ndarray, x: np.ndarray, y: np.ndarray):
    """Backpropagation of the mean squared error through the three affine maps."""
    W1, b1, W2, b2, W3, b3 = unpack(p.astype(np.float64))
    yh, (x, z1, h1, z2, h2) = forward(p, x)
    n = x.size
    d = 2.0 * (yh - y.astype(np.float64)) / n        # dL/dyhat
    g = np.zeros(N_PARAMS, dtype=np.float64)
    g[OFF_W3:OFF_W3 + 64] = h2.T @ d
    g[OFF_B3] = d.sum()
    dh2 = np.outer(d, W3)
    dz2 = dh2 * (z2 > 0)
    g[OFF_W2:OFF_W2 + 4096] = (dz2.T @ h1).reshape(-1)
    g[OFF_B2:OFF_B2 + 64] = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    g[OFF_W1:OFF_W1 + 64] = dz1.T @ x
    g[OFF_B1:OFF_B1 + 64] = dz1.sum(axis=0)
    return float(np.mean((yh - y) ** 2)), g


def adam_step(p, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    p = p - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def bit_length_u64(k: np.ndarray) -> np.ndarray:
    """Exact bit length of every uint64 (0 for 0)."""
    k = k.astype(np.uint64)
    e = np.zeros(k.shape, dtype=np.int64)
    for sh in (32, 16, 8, 4, 2, 1):
        hit = (k >> (e + sh).astype(np.uint64)) != 0
        e = np.where(hit, e + sh, e)
    return np.where(k != 0, e + 1, 0)


def loglinear(k: np.ndarray, key_bits: int) -> np.ndarray:
    """Monotone key transform t(k) = (e + 1 + (k - 2^e) / 2^e) / (key_bits + 1)
    with e = floor(log2 k), t(0) = 0: one unit per binary order of magnitude,
    linear inside it, so that narrow dense ranges near zero and the full word
    range both get resolution in float32."""
    k = k.astype(np.uint64)
    bl = bit_length_u64(k)
    e = np.maximum(bl - 1, 0)
    p = np.left_shift(np.uint64(1), e.astype(np.uint64))
    frac = (k - p).astype(np.float64) / p.astype(np.float64)
    return np.where(k != 0, (e + 1 + frac) / (key_bits + 1), 0.0)


def training_data(sorted_keys: np.ndarray, key_bits: int | None = None):
    """x = (t(k) - t(kmin)) / (t(kmax) - t(kmin)) in float64 (0 if equal), with t the
    log-linear transform; y = (i + 0.5) / N for the i-th sorted sample key."""
    kb = 8 * sorted_keys.dtype.itemsize if key_bits is None else key_bits
    t = loglinear(sorted_keys, kb)
    n = t.size
    span = t[-1] - t[0]
    x = (t - t[0]) / span if span > 0 else np.zeros(n)
    y = (np.arange(n, dtype=np.float64) + 0.5) / n
    return x, y


def batch_indices(n: int, batch: int, step: int) -> np.ndarray:
    stride = n // batch
    return np.arange(batch, dtype=np.int64) * stride + (step % stride)


def train(sorted_keys: np.ndarray, seed: int, steps: int, batch: int, lr: float):
    x, y = training_data(sorted_keys)
    p = init_params(seed)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for s in range(steps):
        idx = batch_indices(x.size, batch, s)
        l, g = loss_and_grad(p, x[idx], y[idx])
        p, m, v = adam_step(p, m, v, g, s + 1, lr)
        losses.append(l)
    return p, losses


def splitters(sorted_keys: np.ndarray, pred: np.ndarray, n_zones: int) -> np.ndarray:
    mono = np.maximum.accumulate(pred.astype(np.float64))
    out = np.zeros(n_zones - 1, dtype=np.uint64)
    last = 0
    for b in range(1, n_zones):
        q = b / n_zones
        i = int(np.searchsorted(mono, q, side="left"))
        if i < sorted_keys.size:
            s = int(sorted_keys[i])
        else:
            s = min(int(sorted_keys[-1]) + 1, (1 << (8 * sorted_keys.dtype.itemsize)) - 1)
        s = max(s, last)
        out[b - 1] = s
        last = s
    return out.astype(sorted_keys.dtype)


def zone_by_splitters(keys: np.ndarray, spl: np.ndarray) -> np.ndarray:
    return np.searchsorted(spl, keys, side="right")


def balance_error(zone_of_key: np.ndarray, n_zones: int) -> float:
    if zone_of_key.size == 0:
        return 1.0
    c = np.bincount(zone_of_key, minlength=n_zones)
    return float(c.max() / (zone_of_key.size / n_zones))
