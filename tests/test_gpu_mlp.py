"""GPU: the selector network's FP32 kernels against the FP64 oracle."""

import numpy as np
import pytest

from oracle import mlp as ref

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def learn():
    from paper_1407_2889_amd import learn as L
    return L


def data(seed, B=300):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, 7))
    T = rng.normal(size=(B, 24))
    M = (rng.random((B, 24)) < 0.85).astype(np.float64)
    return X, T, M


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("seed", [0, 1])
def test_forward_loss_gradient_match_oracle(learn, seed):
    X, T, M = data(seed)
    th = learn.init_params(seed).astype(np.float64) + np.random.default_rng(9).normal(0, 0.05, 10392)
    net = learn.Net(theta=th.astype(np.float32))
    th32 = th.astype(np.float32).astype(np.float64)  # the GPU sees rounded parameters
    Y, acts = ref.forward(th32, X.astype(np.float32).astype(np.float64))
    y_gpu = net.forward(dev(X)).cpu().numpy()
    assert np.max(np.abs(y_gpu - Y)) <= 1e-4 * max(1.0, np.max(np.abs(Y)))
    loss, grad = net.gradient(dev(X), dev(T), dev(M))
    want_loss = ref.loss(Y, T.astype(np.float32), M)
    assert abs(float(loss.item()) - want_loss) <= 1e-4 * max(1.0, want_loss)
    g_ref = ref.backward(th32, acts, ref.loss_grad(Y, T.astype(np.float32).astype(np.float64), M))
    g_gpu = grad.cpu().numpy()
    assert np.max(np.abs(g_gpu - g_ref)) <= 1e-4 * np.max(np.abs(g_ref))


def test_adam_matches_oracle(learn):
    rng = np.random.default_rng(3)
    net = learn.Net(seed=3)
    th0 = net.theta.cpu().numpy().astype(np.float64)
    m = np.zeros(10392)
    v = np.zeros(10392)
    th = th0.copy()
    for t in range(1, 4):
        g = rng.normal(size=10392)
        net.grad.copy_(torch.from_numpy(g.astype(np.float32)))
        net.adam(lr=1e-2)
        th, m, v = ref.adam_step(th, g.astype(np.float32).astype(np.float64), m, v, t, lr=1e-2)
    assert np.max(np.abs(net.theta.cpu().numpy() - th)) <= 1e-5


def test_training_tracks_oracle(learn):
    X, _, _ = data(11, B=512)
    teacher = ref.init(99)
    T, _ = ref.forward(teacher, X)
    M = np.ones_like(T)
    th0 = learn.init_params(5)
    net = learn.Net(theta=th0)
    hist = net.train(dev(X), dev(T), dev(M), steps=200, lr=3e-3, log_every=50)
    _, ref_hist = ref.train(th0.astype(np.float64), X.astype(np.float32).astype(np.float64),
                            T.astype(np.float32).astype(np.float64), M, steps=200, lr=3e-3)
    assert hist[-1][1] < 0.2 * hist[0][1]
    # same trajectory within FP32 drift
    for s, l in hist:
        assert abs(l - ref_hist[s]) <= 0.05 * ref_hist[s] + 1e-6, (s, l, ref_hist[s])
