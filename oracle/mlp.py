"""FP64 reference of the variant-selector network (test infrastructure only).

TEST INFRASTRUCTURE ONLY: used by tests to check the GPU training kernels; the
product path never imports it.

The network maps a request's 7 features to a predicted log-throughput for each
of 24 scan variants: three hidden layers of 64 units with ReLU, and a linear
output layer (7 -> 64 -> 64 -> 64 -> 24, 10,392 parameters). Training
minimises the masked mean squared error

    L = sum_{b,j} M_bj (Y_bj - T_bj)^2 / sum_{b,j} M_bj

(mask M excludes variants that could not be timed for a request) with Adam
(Kingma and Ba, 2015: moments with bias correction).

Parameter vector layout (row-major, float): W1[7,64] b1[64] W2[64,64] b2[64]
W3[64,64] b3[64] W4[64,24] b4[24]; layer l computes Z = A_prev @ W_l + b_l.
"""

from __future__ import annotations

import numpy as np

SIZES = (7, 64, 64, 64, 24)


def layer_shapes(sizes=SIZES):
    out = []
    for k, n in zip(sizes[:-1], sizes[1:]):
        out.append(((k, n), (n,)))
    return out


def n_params(sizes=SIZES) -> int:
    return sum(k * n + n for (k, n), _ in layer_shapes(sizes))


def unpack(theta: np.ndarray, sizes=SIZES):
    """Views (W, b) per layer into the flat parameter vector."""
    layers = []
    o = 0
    for (k, n), _ in layer_shapes(sizes):
        W = theta[o:o + k * n].reshape(k, n)
        o += k * n
        b = theta[o:o + n]
        o += n
        layers.append((W, b))
    assert o == theta.size
    return layers


def init(seed: int, sizes=SIZES) -> np.ndarray:
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for (k, n), _ in layer_shapes(sizes):
        lim = np.sqrt(6.0 / k)
        parts.append(rng.uniform(-lim, lim, k * n))
        parts.append(np.zeros(n))
    return np.concatenate(parts)


def forward(theta: np.ndarray, X: np.ndarray, sizes=SIZES):
    """Returns the output and the activations of every layer (A0 = X)."""
    acts = [np.asarray(X, np.float64)]
    layers = unpack(np.asarray(theta, np.float64), sizes)
    for li, (W, b) in enumerate(layers):
        Z = acts[-1] @ W + b
        acts.append(np.maximum(Z, 0.0) if li < len(layers) - 1 else Z)
    return acts[-1], acts


def loss(Y: np.ndarray, T: np.ndarray, M: np.ndarray) -> float:
    return float(np.sum(M * (Y - T) ** 2) / np.sum(M))


def loss_grad(Y, T, M):
    """dL/dY of the masked mean squared error."""
    return 2.0 * M * (Y - T) / np.sum(M)


def backward(theta: np.ndarray, acts, dY: np.ndarray, sizes=SIZES) -> np.ndarray:
    """Gradient of the loss w.r.t. the flat parameter vector (chain rule
    through each linear layer and ReLU)."""
    layers = unpack(np.asarray(theta, np.float64), sizes)
    grads = []
    g = np.asarray(dY, np.float64)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        A_prev = acts[li]
        dW = A_prev.T @ g
        db = g.sum(axis=0)
        grads.append((dW, db))
        if li > 0:
            g = (g @ W.T) * (A_prev > 0)  # A_prev = ReLU(Z_prev)
    grads.reverse()
    return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])


def adam_step(theta, grad, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta, X, T, M, steps: int, lr=1e-3):
    """Full-batch Adam; returns (theta, loss history)."""
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    hist = []
    for t in range(1, steps + 1):
        Y, acts = forward(theta, X)
        hist.append(loss(Y, T, M))
        g = backward(theta, acts, loss_grad(Y, T, M))
        theta, m, v = adam_step(theta, g, m, v, t, lr)
    return theta, hist
