"""Learned variant selector.

A small dense network (7 -> 64 -> 64 -> 64 -> 24, ReLU) maps a request's
features to one standardised value per scan variant. It is trained on the
exhaustive autotuner's timings with the library's own GPU kernels (forward,
masked mean squared error, backward, Adam); this module only moves tensors
and calls them.

The selector holds two ensembles of such nets (different seeds, predictions
averaged). The ranking ensemble predicts each variant's log slowdown against
the request's fastest variant; the variant with the lowest prediction among
those that can run is taken, and when the runner-up is predicted within
``margin`` (5% in time) of it, the request falls back to the exhaustive
autotuner. The timing ensemble predicts log milliseconds per request, which
the batch planner uses to queue long requests first.
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


class _Ensemble:
    """Nets trained on the same standardised data from different seeds; their
    predictions are averaged."""

    def __init__(self, nets, x_mean, x_std, y_mean, y_std):
        self.nets = nets
        self.x_mean, self.x_std = np.asarray(x_mean), np.asarray(x_std)
        self.y_mean, self.y_std = float(y_mean), float(y_std)

    @classmethod
    def fit(cls, feats, target, valid, n_nets, steps, lr, seed, device):
        torch = _torch()
        x_mean = feats.mean(0)
        x_std = feats.std(0) + 1e-6
        y_mean = float(target[valid].mean())
        y_std = float(target[valid].std() + 1e-6)
        X = torch.from_numpy(((feats - x_mean) / x_std).astype(np.float32)).to(device)
        T = torch.from_numpy((np.where(valid, (target - y_mean) / y_std, 0.0)).astype(np.float32)).to(device)
        M = torch.from_numpy(valid.astype(np.float32)).to(device)
        nets, hist = [], []
        for k in range(n_nets):
            net = Net(seed=seed + k, device=device)
            hist.append(net.train(X, T, M, steps, lr, log_every=max(1, steps // 4)))
            nets.append(net)
        ens = cls(nets, x_mean, x_std, y_mean, y_std)
        ens.history = hist
        return ens

    def predict(self, feats):
        torch = _torch()
        X = torch.from_numpy(((np.atleast_2d(feats) - self.x_mean) / self.x_std)
                             .astype(np.float32)).to(self.nets[0].device)
        ys = [net.forward(X).cpu().numpy().astype(np.float64) for net in self.nets]
        return np.mean(ys, axis=0) * self.y_std + self.y_mean

    def state(self, prefix):
        d = {f"{prefix}_x_mean": self.x_mean, f"{prefix}_x_std": self.x_std,
             f"{prefix}_y": np.array([self.y_mean, self.y_std])}
        for k, net in enumerate(self.nets):
            d[f"{prefix}_theta{k}"] = net.theta.cpu().numpy()
        return d

    @classmethod
    def from_state(cls, z, prefix, device):
        nets = []
        k = 0
        while f"{prefix}_theta{k}" in z:
            nets.append(Net(theta=z[f"{prefix}_theta{k}"], device=device))
            k += 1
        y = z[f"{prefix}_y"]
        return cls(nets, z[f"{prefix}_x_mean"], z[f"{prefix}_x_std"], float(y[0]), float(y[1]))


class Selector:
    """Two ensembles over the request features: `rank` predicts each variant's
    log slowdown relative to the request's fastest variant (what the choice
    needs), `time` predicts each variant's log milliseconds per request (what
    the batch planner's queue order needs)."""

    def __init__(self, rank: _Ensemble, timing: _Ensemble, chunk_factor=None,
                 chunk_safety: float = 1.0):
        self.rank = rank
        self.timing = timing
        # per variant: a request's longest chunk time ~ its cost x factor /
        # its number of chunks (fitted on the timing database)
        self.chunk_factor = (np.ones(N_OUT) if chunk_factor is None
                             else np.asarray(chunk_factor, np.float64))
        # predicted costs are multiplied by this before they estimate the
        # longest chunks a plan waits for: a batch ends with its longest
        # chunk, the maximum over many requests, which an underestimated
        # cost would let the scheduler accept
        self.chunk_safety = float(chunk_safety)

    @classmethod
    def fit(cls, feats: np.ndarray, ms: np.ndarray, n_nets: int = 5, steps: int = 2000,
            lr: float = 2e-3, seed: int = 0, device="cuda", chunk_factor=None):
        """feats [R, 7]; ms [R, 24] per-request milliseconds (inf where a
        variant cannot run); chunk_factor [24] (see __init__)."""
        valid = np.isfinite(ms) & (ms > 0)
        safe = np.where(valid, ms, 1.0)
        rel = np.log(safe / np.min(np.where(valid, ms, np.inf), axis=1, keepdims=True))
        rank = _Ensemble.fit(feats, np.where(valid, rel, 0.0), valid, n_nets, steps, lr, seed, device)
        timing = _Ensemble.fit(feats, np.log(safe), valid, max(1, n_nets // 2), steps, lr,
                               seed + 100, device)
        # the 99th percentile of measured / predicted cost over the timing
        # database (clipped to [1, 3]): on requests it was not trained on the
        # ensemble errs more than on these
        pred = np.exp(np.clip(timing.predict(feats), -30.0, 30.0))
        ratio = (safe / pred)[valid]
        safety = float(np.clip(np.quantile(ratio, 0.99), 1.0, 3.0)) if ratio.size else 1.0
        sel = cls(rank, timing, chunk_factor, safety)
        sel.history = {"rank": rank.history, "time": timing.history}
        return sel

    def predict_ms(self, feats: np.ndarray) -> np.ndarray:
        # log-milliseconds clipped to a sane range before exponentiating
        return np.exp(np.clip(self.timing.predict(feats), -30.0, 30.0))

    def predict_gbps(self, feats: np.ndarray, n: np.ndarray) -> np.ndarray:
        return np.asarray(n, np.float64)[:, None] / (self.predict_ms(feats) * 1e-3) / 1e9

    def choose(self, feats: np.ndarray, valid: np.ndarray, margin: float = 0.05):
        """Per request: (variant, needs_fallback). The predicted best must beat
        the predicted runner-up by `margin` (relative time) or the request
        falls back to the exhaustive autotuner."""
        score = np.where(valid, self.rank.predict(feats), np.inf)
        order = np.argsort(score, axis=1)
        r = np.arange(len(order))
        best = order[:, 0]
        # a runner-up that cannot run (score inf) leaves an infinite gap
        diff = np.minimum(score[r, order[:, 1]] - score[r, best], 30.0)
        gap = np.exp(diff) - 1.0
        return best, gap < margin

    def save(self, path: str):
        d = self.rank.state("rank")
        d.update(self.timing.state("time"))
        d["chunk_factor"] = self.chunk_factor
        d["chunk_safety"] = np.array([self.chunk_safety])
        np.savez(path, **d)

    @classmethod
    def load(cls, path: str, device="cuda"):
        z = np.load(path)
        return cls(_Ensemble.from_state(z, "rank", device), _Ensemble.from_state(z, "time", device),
                   z["chunk_factor"] if "chunk_factor" in z else None,
                   float(z["chunk_safety"][0]) if "chunk_safety" in z else 1.0)
