"""Batched scans: many texts, each with its own index and launch variant,
run as one replayable HIP graph (binding of the mpm_batch_* entry points).

Texts are packed into one device arena at 256-byte aligned offsets; every
request gets its own output region and total. Requests that share an index
and a variant form one persistent launch whose workgroups take chunks of all
the group's texts from a shared ticket counter.
"""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import (MPM_OK, Index, MpmError, Request, Variant, _check, _L, _stream_handle,
               _torch)


def _align(x: int, a: int = 256) -> int:
    return (x + a - 1) // a * a


def pack_texts(texts, device="cuda"):
    """Copy host texts into one device arena; returns (arena, offsets, lens)."""
    torch = _torch()
    lens = np.array([len(t) for t in texts], np.int64)
    offs = np.zeros(len(texts) + 1, np.int64)
    for i, n in enumerate(lens):
        offs[i + 1] = offs[i] + _align(int(n) + 1)
    host = np.zeros(int(offs[-1]) + 256, np.uint8)
    for i, t in enumerate(texts):
        host[offs[i]:offs[i] + lens[i]] = np.asarray(t, np.uint8)
    arena = torch.from_numpy(host).to(device)
    return arena, offs[:-1], lens


class BatchScan:
    """A planned batch bound to device buffers.

    indexes[i], variants[i], capacities[i] belong to text i of the arena.
    """

    def __init__(self, arena, offsets, lens, indexes, variants, capacities, device="cuda",
                 cost_hints=None, timed: bool = False):
        torch = _torch()
        self.count = len(lens)
        self.lens = np.asarray(lens, np.int64)
        self.caps = np.asarray(capacities, np.int64)
        self.out_offs = np.zeros(self.count + 1, np.int64)
        self.out_offs[1:] = np.cumsum(np.maximum(self.caps, 0))
        self.arena = arena
        self.out = torch.empty((max(1, int(self.out_offs[-1])), 2), dtype=torch.int32, device=device)
        self.totals = torch.zeros(max(1, self.count), dtype=torch.int64, device=device)
        # timed: every run adds each request's share of its launch and raises
        # its longest chunk time (us), costs[i] = (share, longest chunk)
        self.costs = (torch.zeros((max(1, self.count), 2), dtype=torch.float32, device=device)
                      if timed else None)
        self._indexes = list(indexes)
        reqs = (Request * max(1, self.count))()
        base_t, base_o, base_tot = arena.data_ptr(), self.out.data_ptr(), self.totals.data_ptr()
        for i in range(self.count):
            ix = indexes[i]
            if not ix.uploaded:
                ix.upload(device)
            r = reqs[i]
            r.idx = ix.handle
            r.d_text = base_t + int(offsets[i])
            r.n = int(self.lens[i])
            r.d_out = base_o + 8 * int(self.out_offs[i])
            r.capacity = int(self.caps[i])
            r.d_total = base_tot + 8 * i
            v = variants[i]
            r.variant = Variant(v.lane_bytes, v.block_threads, v.placement, v.grid, v.flags)
            r.cost_hint = float(cost_hints[i]) if cost_hints is not None else 0.0
            r.d_cost = self.costs.data_ptr() + 8 * i if timed else None
        h = C.c_void_p()
        _check(_L.mpm_batch_plan(reqs, self.count, C.byref(h)), "mpm_batch_plan")
        self._h = h
        nb = int(_L.mpm_batch_device_bytes(h))
        self.dev = torch.zeros(max(256, nb), dtype=torch.uint8, device=device)
        _check(_L.mpm_batch_upload(h, C.c_void_p(self.dev.data_ptr()), self.dev.numel(),
                                   _stream_handle()), "mpm_batch_upload")
        self.captured = False

    @property
    def groups(self) -> int:
        return int(_L.mpm_batch_groups(self._h))

    def run(self, stream=None):
        _check(_L.mpm_batch_run(self._h, _stream_handle(stream)), "mpm_batch_run")

    def capture(self, stream=None):
        torch = _torch()
        s = stream or torch.cuda.Stream()
        torch.cuda.current_stream().synchronize()
        _check(_L.mpm_batch_capture(self._h, _stream_handle(s)), "mpm_batch_capture")
        s.synchronize()
        self.captured = True

    def replay(self, stream=None):
        _check(_L.mpm_batch_replay(self._h, _stream_handle(stream)), "mpm_batch_replay")

    def totals_host(self) -> np.ndarray:
        return self.totals[: self.count].cpu().numpy()

    def result(self, i: int, totals: np.ndarray | None = None):
        """(pos, id) uint32 arrays of request i (after the batch completed)."""
        tot = int((totals if totals is not None else self.totals_host())[i])
        if tot > self.caps[i]:
            raise MpmError(-2, f"batch request {i}: {tot} matches > capacity {self.caps[i]}")
        a = self.out[int(self.out_offs[i]): int(self.out_offs[i]) + tot].cpu().numpy().view(np.uint32)
        return a[:, 0].copy(), a[:, 1].copy()

    def close(self):
        if getattr(self, "_h", None) and self._h:
            _L.mpm_batch_free(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["pack_texts", "BatchScan", "MPM_OK"]
_ = Index
