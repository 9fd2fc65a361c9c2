"""Learned variant selector.

A small dense network (7 -> 64 -> 64 -> 64 -> 24, ReLU) predicts, from a
request's features, the standardised log-throughput of each of the 24 scan
variants. It is trained on the exhaustive autotuner's timings with the
library's own GPU kernels (forward, masked mean squared error, backward,
Adam); this module only moves tensors and calls them. At selection time the
variant with the highest prediction among those that can run is taken; when
the predicted best beats the runner-up by less than ``margin`` (5% in
throughput), the request falls back to the exhaustive autotuner.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _check, _L, _stream_handle, _torch

N_IN, N_HIDDEN, N_OUT, N_PARAMS = 7, 64, 24, 10392


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (same layout as the kernels)."""
    rng = np.random.default_rng(seed)
    sizes = (N_IN, N_HIDDEN, N_HIDDEN, N_HIDDEN, N_OUT)
    parts = []
    for k, n in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / k)
        parts.append(rng.uniform(-lim, lim, k * n))
        parts.append(np.zeros(n))
    th = np.concatenate(parts).astype(np.float32)
    assert th.size == N_PARAMS
    return th


class Net:
    """Parameters and Adam state on the device, plus the kernels' buffers."""

    def __init__(self, theta: np.ndarray | None = None, seed: int = 0, device="cuda"):
        torch = _torch()
        self.torch = torch
        self.device = device
        th = init_params(seed) if theta is None else np.asarray(theta, np.float32)
        self.theta = torch.from_numpy(th.copy()).to(device)
        self.m = torch.zeros(N_PARAMS, dtype=torch.float32, device=device)
        self.v = torch.zeros(N_PARAMS, dtype=torch.float32, device=device)
        self.grad = torch.zeros(N_PARAMS, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.t = 0
        self._batch = 0

    def _buffers(self, batch: int):
        if batch != self._batch:
            t = self.torch
            self.act = t.empty(int(_L.mpm_mlp_act_floats(batch)), dtype=t.float32, device=self.device)
            self.y = t.empty((batch, N_OUT), dtype=t.float32, device=self.device)
            self.dy = t.empty((batch, N_OUT), dtype=t.float32, device=self.device)
            self.tmp = t.empty(2 * batch * N_HIDDEN, dtype=t.float32, device=self.device)
            self._batch = batch

    def forward(self, x):
        """x: float32 [B, 7] device tensor -> [B, 24] (a view of a reused buffer)."""
        B = x.shape[0]
        self._buffers(B)
        _check(_L.mpm_mlp_forward(_ptr(self.theta), _ptr(x), B, _ptr(self.act), _ptr(self.y),
                                  _stream_handle()), "mpm_mlp_forward")
        return self.y

    def gradient(self, x, target, mask):
        """Loss and gradient (device) for one full batch."""
        B = x.shape[0]
        self.forward(x)
        _check(_L.mpm_mlp_loss_grad(_ptr(self.y), _ptr(target), _ptr(mask), B, _ptr(self.dy),
                                    _ptr(self.loss), _stream_handle()), "mpm_mlp_loss_grad")
        _check(_L.mpm_mlp_backward(_ptr(self.theta), _ptr(x), _ptr(self.act), _ptr(self.dy), B,
                                   _ptr(self.grad), _ptr(self.tmp), _stream_handle()),
               "mpm_mlp_backward")
        return self.loss, self.grad

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        _check(_L.mpm_mlp_adam(_ptr(self.theta), _ptr(self.grad), _ptr(self.m), _ptr(self.v),
                               N_PARAMS, self.t, lr, b1, b2, eps, _stream_handle()), "mpm_mlp_adam")

    def train(self, x, target, mask, steps: int, lr=1e-3, log_every: int = 0):
        hist = []
        for s in range(steps):
            loss, _ = self.gradient(x, target, mask)
            self.adam(lr)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(loss.item())))
        return hist


class Selector:
    """Feature / target normalisation around a trained Net."""

    def __init__(self, net: Net, x_mean, x_std, y_mean, y_std):
        self.net = net
        self.x_mean, self.x_std = np.asarray(x_mean), np.asarray(x_std)
        self.y_mean, self.y_std = float(y_mean), float(y_std)

    @classmethod
    def fit(cls, feats: np.ndarray, gbs: np.ndarray, steps: int = 3000, lr: float = 2e-3,
            seed: int = 0, device="cuda"):
        """feats [R, 7]; gbs [R, 24] measured GB/s (0 where a variant cannot run)."""
        torch = _torch()
        valid = gbs > 0
        logy = np.where(valid, np.log(np.maximum(gbs, 1e-12)), 0.0)
        x_mean = feats.mean(0)
        x_std = feats.std(0) + 1e-6
        y_mean = float(logy[valid].mean())
        y_std = float(logy[valid].std() + 1e-6)
        X = torch.from_numpy(((feats - x_mean) / x_std).astype(np.float32)).to(device)
        T = torch.from_numpy(((logy - y_mean) / y_std * valid).astype(np.float32)).to(device)
        M = torch.from_numpy(valid.astype(np.float32)).to(device)
        net = Net(seed=seed, device=device)
        hist = net.train(X, T, M, steps, lr, log_every=max(1, steps // 10))
        sel = cls(net, x_mean, x_std, y_mean, y_std)
        sel.history = hist
        return sel

    def predict_gbps(self, feats: np.ndarray) -> np.ndarray:
        torch = _torch()
        X = torch.from_numpy(((np.atleast_2d(feats) - self.x_mean) / self.x_std)
                             .astype(np.float32)).to(self.net.device)
        y = self.net.forward(X).cpu().numpy().astype(np.float64)
        return np.exp(y * self.y_std + self.y_mean)

    def choose(self, feats: np.ndarray, valid: np.ndarray, margin: float = 0.05):
        """Per request: (variant, needs_fallback). valid [R, 24] booleans."""
        pred = self.predict_gbps(feats)
        pred = np.where(valid, pred, -np.inf)
        order = np.argsort(-pred, axis=1)
        best = order[:, 0]
        top = pred[np.arange(len(best)), best]
        second = pred[np.arange(len(best)), order[:, 1]]
        fallback = (top - second) / np.maximum(top, 1e-30) < margin
        return best, fallback

    def save(self, path: str):
        np.savez(path, theta=self.net.theta.cpu().numpy(), x_mean=self.x_mean, x_std=self.x_std,
                 y_mean=self.y_mean, y_std=self.y_std)

    @classmethod
    def load(cls, path: str, device="cuda"):
        z = np.load(path)
        return cls(Net(theta=z["theta"], device=device), z["x_mean"], z["x_std"],
                   float(z["y_mean"]), float(z["y_std"]))
