"""Pins of the FP64 network oracle: finite-difference gradients, the closed
form of Adam's first step, scaler and R^2 on hand-computable data, mixed-radix
decoding, and the composition of the training loop."""
import math

import numpy as np
import pytest

from oracle import mlp
from paper_2306_14011_amd import inputs


def small_problem(n=37, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 14))
    y = np.sin(X[:, 0]) + 0.3 * X[:, 3] * X[:, 5] + 0.1 * rng.standard_normal(n)
    return X, y


def test_parameter_count():
    assert mlp.NPARAM == 9345 == inputs.mlp_init(0).size


@pytest.mark.parametrize("alpha", [0.0, 1e-4, 0.3])
def test_gradient_matches_central_differences(alpha):
    X, y = small_problem()
    theta = inputs.mlp_init(3)
    L, g = mlp.loss_grad(theta, X, y, alpha)
    rng = np.random.default_rng(1)
    h = 1e-6
    # random coordinates, including biases and every layer
    idx = np.concatenate([rng.choice(mlp.NPARAM, 60, replace=False), [0, 896, 960, 9280, 9344]])
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        fd = (mlp.loss_grad(theta + e, X, y, alpha)[0] - mlp.loss_grad(theta - e, X, y, alpha)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])
    # directional derivative along a random direction
    d = rng.standard_normal(mlp.NPARAM)
    fd = (mlp.loss_grad(theta + h * d, X, y, alpha)[0] - mlp.loss_grad(theta - h * d, X, y, alpha)[0]) / (2 * h)
    assert abs(fd - g @ d) <= 1e-7 * abs(g @ d)


def test_l2_term_closed_form():
    # zero weights: prediction is b4 for every row, and the penalty vanishes
    theta = np.zeros(mlp.NPARAM)
    theta[-1] = 0.5
    X, y = small_problem(10)
    L, g = mlp.loss_grad(theta, X, y, 0.7)
    assert abs(L - 0.5 * np.mean((0.5 - y) ** 2)) < 1e-15
    assert abs(g[-1] - np.mean(0.5 - y)) < 1e-15
    # penalty alone: loss grows by alpha/(2B) |W|^2 with gradient alpha/B W on weights only
    theta = inputs.mlp_init(5)
    L0, g0 = mlp.loss_grad(theta, X, y, 0.0)
    L1, g1 = mlp.loss_grad(theta, X, y, 0.7)
    w = theta * mlp.weight_mask()
    assert abs((L1 - L0) - 0.35 * (w @ w) / 10) < 1e-12
    assert np.allclose(g1 - g0, 0.07 * w, rtol=0, atol=1e-15)


def test_first_adam_step_closed_form():
    # from m = v = 0: step = -lr g / (|g| + eps / sqrt(1 - beta2))
    rng = np.random.default_rng(2)
    g = rng.standard_normal(50) * np.logspace(-12, 2, 50)
    th0 = rng.standard_normal(50)
    lr, b1, b2, eps = 9e-4, 0.95, 0.90, 1e-9
    th, m, v, t = mlp.adam_step(th0, np.zeros(50), np.zeros(50), 0, g, lr, b1, b2, eps)
    expect = th0 - lr * g / (np.abs(g) + eps / math.sqrt(1 - b2))
    assert t == 1
    assert np.allclose(th, expect, rtol=0, atol=1e-15)
    assert np.allclose(m, 0.05 * g) and np.allclose(v, 0.1 * g * g)


def test_standard_scaler_and_r2_toys():
    F = np.array([[1.0, 2.0], [3.0, 2.0], [5.0, 2.0]])
    mean, std = mlp.standard_scaler(F)
    assert np.allclose(mean, [3.0, 2.0]) and np.allclose(std, [math.sqrt(8.0 / 3.0), 1.0])
    y = np.array([1.0, 2.0, 3.0, 4.0])
    assert mlp.r2(y, y) == 1.0
    assert mlp.r2(y, np.full(4, 2.5)) == 0.0
    # residuals (0.5, -0.5, 0, 0): 1 - 0.5 / 5
    assert abs(mlp.r2(y, [0.5, 2.5, 3.0, 4.0]) - 0.9) < 1e-15


def test_decode_mixed_radix():
    radix = [3, 1, 4, 2]
    seen = set()
    for idx in range(24):
        d = mlp.decode(idx, radix)
        assert all(0 <= d[s] < radix[s] for s in range(4))
        assert d[0] + 3 * (d[1] + 1 * (d[2] + 4 * d[3])) == idx
        seen.add(tuple(d))
    assert len(seen) == 24


def test_full_batch_epoch_is_one_adam_step_on_the_full_gradient():
    X, y = small_problem(20)
    theta = inputs.mlp_init(7)
    order = inputs.epoch_orders(20, 1, 0)
    th, losses, ne, m, v, t = mlp.train(theta, X, y, order, batch=200, max_epochs=1)
    L, g = mlp.loss_grad(theta, X, y, 1e-4)
    th2, _, _, _ = mlp.adam_step(theta, np.zeros_like(theta), np.zeros_like(theta), 0, g, 9e-4, 0.95, 0.90, 1e-9)
    assert ne == 1 and t == 1
    assert np.allclose(th, th2, rtol=0, atol=1e-15)
    assert abs(losses[0] - L) < 1e-14


def test_minibatch_epoch_loss_is_size_weighted_mean():
    # n = 5 rows, batch 2: minibatches of 2, 2, 1 in the epoch's order
    X, y = small_problem(5)
    theta = inputs.mlp_init(8)
    order = inputs.epoch_orders(5, 1, 3)
    _, losses, _, _, _, t = mlp.train(theta, X, y, order, batch=2, max_epochs=1)
    th = theta.copy()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    tt = 0
    acc = 0.0
    for rows in (order[0][0:2], order[0][2:4], order[0][4:5]):
        L, g = mlp.loss_grad(th, X[rows], y[rows], 1e-4)
        acc += L * len(rows)
        th, m, v, tt = mlp.adam_step(th, m, v, tt, g, 9e-4, 0.95, 0.90, 1e-9)
    assert t == 3 and abs(losses[0] - acc / 5) < 1e-15


def test_early_stop_rule():
    # a constant target that the bias reaches at once: the loss stops improving
    X, y = small_problem(30)
    theta = inputs.mlp_init(9)
    order = inputs.epoch_orders(30, 400, 1)
    _, losses, ne, _, _, _ = mlp.train(theta, X, np.zeros(30), order, batch=30, max_epochs=400, tol=1e-1,
                                       n_iter_no_change=3)
    # with tol 0.1 no epoch improves enough after the first: stops after 1 + 4 epochs
    assert ne == 5, losses


def test_training_reduces_loss():
    X, y = small_problem(200, seed=4)
    theta = inputs.mlp_init(10)
    order = inputs.epoch_orders(200, 50, 2)
    _, losses, ne, _, _, _ = mlp.train(theta, X, y, order, batch=50, max_epochs=50)
    assert losses[-1] < 0.5 * losses[0]


# ---------------------------------------------------------------------------
# The problem-size-conditioned network: 16 inputs, the launch features then
# two problem features.

def test_sized_parameter_count():
    assert mlp.nparam(16) == 9473 == inputs.mlp_init(0, 16).size
    assert mlp.n_in_of(np.zeros(9473)) == 16 and mlp.n_in_of(np.zeros(9345)) == 14
    with pytest.raises(ValueError):
        mlp.n_in_of(np.zeros(9400))


def test_sized_network_with_zero_extra_columns_is_the_launch_network():
    # W1 rows are [launch features | problem features]: zeroing the two last
    # columns of every row gives the 14-input network of the same weights for
    # any problem features (a transposed or misplaced W1 block fails this)
    rng = np.random.default_rng(4)
    th14 = inputs.mlp_init(7)
    th16 = inputs.mlp_init(8, 16)
    W1 = th14[:896].reshape(64, 14)
    th16[:1024] = np.hstack([W1, np.zeros((64, 2))]).ravel()
    th16[1024:] = th14[896:]
    X = rng.standard_normal((50, 14))
    E = rng.standard_normal((50, 2)) * 3.0
    assert np.array_equal(mlp.predict(th16, np.hstack([X, E])), mlp.predict(th14, X))
    # the penalty sees the same weights, the gradient's extra columns are the
    # inputs' correlation with the first-layer deltas
    y = rng.standard_normal(50)
    L14, g14 = mlp.loss_grad(th14, X, y, 0.2)
    L16, g16 = mlp.loss_grad(th16, np.hstack([X, E]), y, 0.2)
    assert abs(L14 - L16) <= 1e-14 * abs(L14)
    G1 = g16[:1024].reshape(64, 16)
    assert np.allclose(G1[:, :14].ravel(), g14[:896], rtol=1e-13, atol=1e-16)
    assert np.allclose(g16[1024:], g14[896:], rtol=1e-13, atol=1e-16)
    # with one problem feature set to zero its column's gradient is zero too
    _, gz = mlp.loss_grad(th16, np.hstack([X, np.zeros((50, 1)), E[:, 1:]]), y, 0.0)
    assert np.all(gz[:1024].reshape(64, 16)[:, 14] == 0.0)


@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_sized_gradient_matches_central_differences(alpha):
    rng = np.random.default_rng(6)
    X = rng.standard_normal((29, 16))
    y = np.cos(X[:, 14]) + 0.2 * X[:, 15] * X[:, 2] + 0.1 * rng.standard_normal(29)
    theta = inputs.mlp_init(9, 16)
    L, g = mlp.loss_grad(theta, X, y, alpha)
    h = 1e-6
    cols = np.arange(64) * 16
    idx = np.concatenate([rng.choice(9473, 40, replace=False), cols[:8] + 14, cols[8:16] + 15, [1023, 1024, 9472]])
    for k in idx:
        e = np.zeros(9473)
        e[k] = h
        fd = (mlp.loss_grad(theta + e, X, y, alpha)[0] - mlp.loss_grad(theta - e, X, y, alpha)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])
