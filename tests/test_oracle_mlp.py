"""Pins of the learned partitioner's float64 oracle (not part of the paper).

Forward pass against a hand-computed tiny case, backpropagation against
central finite differences, Adam's first step against its closed form, and
the splitter / balance definitions against direct counting.
"""
import math

import numpy as np
import pytest

from oracle import mlp


def test_forward_hand_computed():
    p = np.zeros(mlp.N_PARAMS)
    # unit 0: relu(2x - 0.5); unit 1: relu(-x + 1)
    p[mlp.OFF_W1 + 0], p[mlp.OFF_B1 + 0] = 2.0, -0.5
    p[mlp.OFF_W1 + 1], p[mlp.OFF_B1 + 1] = -1.0, 1.0
    W2 = np.zeros((64, 64)); W2[0, 0] = 1.5; W2[0, 1] = -2.0; W2[3, 1] = 1.0
    p[mlp.OFF_W2:mlp.OFF_W2 + 4096] = W2.reshape(-1)
    p[mlp.OFF_B2 + 3] = -0.25
    p[mlp.OFF_W3 + 0], p[mlp.OFF_W3 + 3] = 0.5, 3.0
    p[mlp.OFF_B3] = 0.125
    x = np.array([0.0, 0.2, 0.6, 1.0])
    y, _ = mlp.forward(p, x)
    exp = []
    for xi in x:
        a, b = max(2 * xi - 0.5, 0), max(-xi + 1, 0)
        u0 = max(1.5 * a - 2.0 * b, 0)
        u3 = max(b - 0.25, 0)
        exp.append(0.5 * u0 + 3.0 * u3 + 0.125)
    assert np.allclose(y, exp, rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    rs = np.random.default_rng(seed)
    p = mlp.init_params(seed)
    x = np.sort(rs.random(300))
    y = (np.arange(300) + 0.5) / 300
    _, g = mlp.loss_and_grad(p, x, y)
    idx = list(rs.choice(mlp.N_PARAMS, 40, replace=False)) + [mlp.OFF_B3, mlp.OFF_W1, mlp.OFF_B2, mlp.OFF_W3]
    for i in idx:
        e = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += e; pm[i] -= e
        fd = (mlp.loss(pp, x, y) - mlp.loss(pm, x, y)) / (2 * e)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_closed_form():
    # After one step from zero moments: m^ = g, v^ = g^2, so p moves by lr * g / (|g| + eps).
    g = np.array([0.3, -2.0, 0.0, 1e-3])
    p0 = np.array([1.0, 1.0, 1.0, 1.0])
    p1, m, v = mlp.adam_step(p0, np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_init_is_deterministic_and_kinks_in_unit_interval():
    a, b = mlp.init_params(5), mlp.init_params(5)
    assert (a == b).all() and not (a == mlp.init_params(6)).all()
    W1, b1 = a[mlp.OFF_W1:mlp.OFF_W1 + 64], a[mlp.OFF_B1:mlp.OFF_B1 + 64]
    kink = -b1 / W1
    assert (kink >= 0).all() and (kink < 1).all()
    assert (np.abs(W1) >= math.sqrt(6) * 0.5).all() and (np.abs(W1) <= math.sqrt(6)).all()


def test_loglinear_transform_exact_points():
    k = np.array([0, 1, 2, 3, 4, 6, 8, 2 ** 40, 3 * 2 ** 40, 2 ** 63], dtype=np.uint64)
    t = mlp.loglinear(k, 64) * 65
    assert list(t) == [0, 1, 2, 2.5, 3, 3.5, 4, 41, 42.5, 64]
    rs = np.random.default_rng(0)
    r = np.sort(rs.integers(0, 2 ** 63, 10000, dtype=np.uint64))
    tr = mlp.loglinear(r, 64)
    assert (np.diff(tr) >= 0).all()
    assert list(mlp.bit_length_u64(k)) == [int(v).bit_length() for v in k.tolist()]


def test_training_reduces_loss():
    rs = np.random.default_rng(1)
    keys = np.sort(rs.exponential(1e6, 4096).astype(np.uint64))
    p, losses = mlp.train(keys, 0, 200, 256, 3e-3)
    assert losses[-1] < 0.1 * losses[0]


def test_splitters_monotone_and_balance():
    keys = np.arange(1000, dtype=np.uint64) * np.uint64(7)
    pred = (np.arange(1000) + 0.5) / 1000                      # a perfect CDF
    spl = mlp.splitters(keys, pred, 10)
    assert list(spl) == [int(k) for k in keys[[100 * b for b in range(1, 10)]]]
    noisy = pred + 0.3 * np.sin(np.arange(1000))                # non-monotone predictions
    s2 = mlp.splitters(keys, noisy, 16)
    assert (np.diff(s2.astype(np.int64)) >= 0).all()
    z = mlp.zone_by_splitters(keys, spl)
    assert mlp.balance_error(z, 10) == 1.0
    assert mlp.balance_error(np.zeros(50, np.int64), 10) == 10.0
