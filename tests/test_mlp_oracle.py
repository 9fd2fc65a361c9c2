"""Pins for the FP64 reference of the selector network (no GPU).

The analytic gradient is checked against central finite differences of the
loss (independent of the chain-rule code), the first Adam step against its
closed form (with zero initial moments the bias-corrected update is
lr * g / (|g| + eps)), and training against a target the network can fit.
"""

import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.n_params() == 10392
    th = mlp.init(0)
    assert th.size == 10392
    layers = mlp.unpack(th)
    assert [W.shape for W, _ in layers] == [(7, 64), (64, 64), (64, 64), (64, 24)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    sizes = (7, 9, 8, 6, 5)  # a smaller net of the same structure
    th = mlp.init(seed, sizes) + rng.normal(0, 0.1, mlp.n_params(sizes))
    X = rng.normal(size=(13, 7))
    T = rng.normal(size=(13, 5))
    M = (rng.random((13, 5)) < 0.8).astype(float)
    M[0, 0] = 1.0
    Y, acts = mlp.forward(th, X, sizes)
    g = mlp.backward(th, acts, mlp.loss_grad(Y, T, M), sizes)
    h = 1e-6
    num = np.empty_like(th)
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = h
        lp = mlp.loss(mlp.forward(th + e, X, sizes)[0], T, M)
        lm = mlp.loss(mlp.forward(th - e, X, sizes)[0], T, M)
        num[i] = (lp - lm) / (2 * h)
    assert np.max(np.abs(num - g)) <= 1e-6 * max(1.0, np.max(np.abs(g)))


def test_loss_is_masked_mean_square():
    Y = np.array([[1.0, 2.0], [3.0, 5.0]])
    T = np.array([[0.0, 2.0], [1.0, 0.0]])
    M = np.array([[1.0, 1.0], [1.0, 0.0]])
    assert mlp.loss(Y, T, M) == pytest.approx((1 + 0 + 4) / 3)


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(5)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 0.01, 1e-8
    new, m, v = mlp.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=lr, eps=eps)
    assert np.allclose(new, th - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_fits_a_learnable_target():
    rng = np.random.default_rng(7)
    X = rng.normal(size=(256, 7))
    teacher = mlp.init(99)
    T, _ = mlp.forward(teacher, X)
    M = np.ones_like(T)
    th, hist = mlp.train(mlp.init(3), X, T, M, steps=300, lr=3e-3)
    assert hist[-1] < 0.1 * hist[0]
