"""Exhaustive autotuner for batched scans.

Every request (one text, one pattern set) can be scanned by 24 launch
variants: the algorithm (Aho-Corasick or Wu-Manber), the starting positions
per lane (64, 256 or 1024), the workgroup size (256 or 512 threads) and the
placement of the matching tables (LDS or global memory). All variants return
the same matches; they differ only in speed. The exhaustive autotuner times
all of them for a request the way it runs inside a batched launch
(``mpm_tune_time``: the request is queued several times in one persistent
launch so that small texts get a measurable, batch-realistic cost) and keeps
the fastest. Variants that cannot run (tables too large for LDS) are marked
invalid.

Request features (inputs of the learned selector):
    log2 n, log2 d, m, alphabet size (distinct pattern bytes), log2 of the
    Aho-Corasick state count, Wu-Manber mean SHIFT, sampled match density
    (matches per byte over the first 64 KiB of the text).
"""

from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np

from . import (MPM_EUNSUPPORTED, MPM_OK, MpmError, PLACE_AUTO, PLACE_GLOBAL, Index, Variant,
               _check, _L, _stream_handle, _torch, build_ac, build_wm)

ALGOS = ("ac", "wm")
LANE_BYTES = (64, 256, 1024)
BLOCK_THREADS = (256, 512)
# Placement of the matching tables: in LDS as far as they go (all of them when
# they fit, else the hot part: the shallow Aho-Corasick states or the
# Wu-Manber SHIFT table), or all in global memory.
PLACEMENTS = (PLACE_AUTO, PLACE_GLOBAL)

# (algo, lane_bytes, block_threads, placement), 24 entries in a fixed order.
VARIANTS = [(a, L, W, P) for a in ALGOS for L in LANE_BYTES for W in BLOCK_THREADS
            for P in PLACEMENTS]
DEFAULT_VARIANT = VARIANTS.index(("ac", 1024, 512, PLACE_AUTO))

FEATURES = ("log2_n", "log2_d", "m", "alphabet", "log2_states", "wm_mean_shift", "density")


def variant_struct(k: int) -> Variant:
    _, L, W, P = VARIANTS[k]
    return Variant(L, W, P, 0, 0)


@dataclass
class PatternSetIndexes:
    """Both indexes of one pattern set, uploaded."""
    ac: Index
    wm: Index
    d: int
    m: int

    @classmethod
    def build(cls, patterns, device="cuda"):
        P = np.ascontiguousarray(patterns, np.uint8)
        return cls(build_ac(P).upload(device), build_wm(P).upload(device), P.shape[0], P.shape[1])

    def index(self, k: int) -> Index:
        return self.ac if VARIANTS[k][0] == "ac" else self.wm

    def launch_key(self, k: int):
        """The batched launch a request of this set joins under variant k
        (None where the variant cannot run)."""
        keys = self.__dict__.setdefault("_keys", {})
        if k not in keys:
            from . import launch_key
            try:
                keys[k] = launch_key(self.index(k), variant_struct(k)) if self.lds_fits(k) else None
            except MpmError as e:
                if e.status != MPM_EUNSUPPORTED:
                    raise
                keys[k] = None
        return keys[k]

    def lds_fits(self, k: int) -> bool:
        """Whether variant k can run (LDS placement needs the tables to fit)."""
        if VARIANTS[k][3] != PLACEMENTS[0]:
            return True
        from . import workspace_bytes
        try:
            workspace_bytes(self.index(k), 1 << 20, variant_struct(k))
            return True
        except MpmError as e:
            if e.status == MPM_EUNSUPPORTED:
                return False
            raise


class Tuner:
    """Times requests on all variants; keeps reusable device buffers."""

    def __init__(self, device="cuda", target_chunks: int = 2048, max_bytes: int = 32 << 20,
                 max_copies: int = 4096, reps: int = 3):
        torch = _torch()
        self.torch = torch
        self.device = device
        self.target_chunks = target_chunks
        self.max_bytes = max_bytes
        self.max_copies = max_copies
        self.reps = reps
        self.work = torch.empty(0, dtype=torch.uint8, device=device)
        self.out = torch.empty((1, 2), dtype=torch.int32, device=device)
        self.total = torch.zeros(1, dtype=torch.int64, device=device)
        self._ws = {}

    def _workspace(self, nbytes: int):
        if self.work.numel() < nbytes:
            self.work = self.torch.empty(max(nbytes, 2 * self.work.numel()), dtype=self.torch.uint8,
                                         device=self.device)
        return self.work

    def count(self, sets: PatternSetIndexes, text, n: int | None = None) -> int:
        """Number of matches (scan with output capacity 0)."""
        from . import Scanner
        n = text.numel() if n is None else n
        key = id(sets)
        sc = self._ws.get(key)
        if sc is None or sc.ws.numel() * 8 < _ws_bytes(sets.ac, n):
            sc = Scanner(sets.ac, max(n, 1 << 16), capacity=0, var=Variant(256, 256, 0, 0, 0))
            self._ws[key] = sc
        tot = C.c_uint64()
        st = _L.mpm_scan_sync(sets.ac.handle, C.c_void_p(text.data_ptr()), n, None, 0,
                              C.c_void_p(sc.ws.data_ptr()), sc.ws.numel() * 8,
                              C.c_void_p(sc.total.data_ptr()), C.byref(sc.var), _stream_handle(),
                              C.byref(tot))
        if st not in (MPM_OK, -2):
            _check(st, "count")
        return int(tot.value)

    def density(self, sets: PatternSetIndexes, text) -> float:
        n = min(text.numel(), 1 << 16)
        return self.count(sets, text[:n], n) / max(1, n)

    def features(self, sets: PatternSetIndexes, text) -> np.ndarray:
        ia, iw = sets.ac.info(), sets.wm.info()
        n = text.numel()
        return np.array([math.log2(max(n, 1)), math.log2(sets.d), sets.m, ia["n_classes"],
                         math.log2(max(ia["n_states"], 1)), iw["wm_mean_shift"],
                         self.density(sets, text)], np.float64)

    def time_variant(self, sets: PatternSetIndexes, text, k: int, matches: int,
                     reps: int | None = None) -> float:
        """Per-request milliseconds of variant k inside a batched launch."""
        n = text.numel()
        ix = sets.index(k)
        v = variant_struct(k)
        # enough copies to keep every workgroup busy (steady-state cost per
        # request, which is what a request adds to a large batch), within a
        # byte budget per timing launch
        _, L, W, _ = VARIANTS[k]
        chunks = max(1, math.ceil(max(n - sets.m + 1, 1) / (L * W)))
        copies = math.ceil(self.target_chunks / chunks)
        copies = int(max(1, min(copies, self.max_copies, self.max_bytes // max(n, 1))))
        wb = int(_L.mpm_tune_work_bytes(ix.handle, n, copies, C.byref(v)))
        if wb == 0:
            return math.inf
        work = self._workspace(wb + 256)
        if self.out.shape[0] < max(1, matches):
            self.out = self.torch.empty((max(1, matches), 2), dtype=self.torch.int32,
                                        device=self.device)
        ms = C.c_float()
        base = (work.data_ptr() + 255) // 256 * 256
        st = _L.mpm_tune_time(ix.handle, C.c_void_p(text.data_ptr()), n, copies, C.byref(v),
                              C.c_void_p(self.out.data_ptr()), matches,
                              C.c_void_p(self.total.data_ptr()), C.c_void_p(base),
                              work.numel() - (base - work.data_ptr()), reps or self.reps,
                              _stream_handle(),
                              C.byref(ms))
        if st == MPM_EUNSUPPORTED:
            return math.inf
        _check(st, "mpm_tune_time")
        return float(ms.value) / copies

    def time_all(self, sets: PatternSetIndexes, text, refine: int = 4) -> np.ndarray:
        """Per-request milliseconds of all 24 variants (inf where invalid):
        every runnable variant once, then the `refine` fastest again with
        more repetitions (their times replace the first ones)."""
        matches = self.count(sets, text)
        out = np.full(len(VARIANTS), math.inf)
        for k in range(len(VARIANTS)):
            if sets.lds_fits(k):
                out[k] = self.time_variant(sets, text, k, matches, reps=1)
        for k in np.argsort(out)[:refine]:
            if np.isfinite(out[k]):
                out[k] = self.time_variant(sets, text, int(k), matches)
        return out


def time_batch(arena, offs, lens, sets: list, counts, reps: int = 2):
    """Per-request costs of all 24 variants (inf where a variant cannot run),
    measured where requests run: for each variant, every request that can
    take it goes into one batched launch (launches one after another), and
    each chunk's workgroup adds its wall-clock time divided by the launch's
    workgroup count to the request's cost (its share of a launch that has
    the device to itself) and raises the request's longest chunk time. One
    warm-up run, then `reps` runs. Request i is bytes [offs[i], offs[i] +
    lens[i]) of the device arena, scanned with sets[i], with counts[i]
    matches. Returns (share ms [R, 24] (mean per run), longest chunk ms
    [R, 24])."""
    from . import batch as _batch
    offs = np.asarray(offs, np.int64)
    lens = np.asarray(lens, np.int64)
    caps = np.asarray(counts, np.int64)
    R = len(lens)
    share = np.full((R, len(VARIANTS)), math.inf)
    chunk = np.full((R, len(VARIANTS)), math.inf)
    for k in range(len(VARIANTS)):
        ok = np.array([i for i in range(R) if sets[i].lds_fits(k)], np.int64)
        if ok.size == 0:
            continue
        v = variant_struct(k)
        bs = _batch.BatchScan(arena, offs[ok], lens[ok], [sets[i].index(k) for i in ok],
                              [v] * ok.size, caps[ok], timed=True)
        bs.run()
        bs.costs.zero_()
        for _ in range(reps):
            bs.run()
        c = bs.costs[: ok.size].cpu().numpy().astype(np.float64)
        share[ok, k] = c[:, 0] / reps / 1e3
        chunk[ok, k] = c[:, 1] / 1e3
        bs.close()
    return share, chunk


def chunks_of(n: int, m: int, k: int) -> int:
    """Chunks a text of n bytes forms under variant k (patterns of length m)."""
    _, L, W, _ = VARIANTS[k]
    return max(1, math.ceil(max(n - m + 1, 0) / (L * W)))


def _ws_bytes(ix: Index, n: int) -> int:
    from . import workspace_bytes
    return workspace_bytes(ix, max(n, 1 << 16), Variant(256, 256, 0, 0, 0))


def chunk_cost_hint(k: int, ms_per_request: float, n: int, m: int) -> float:
    """Expected duration of one chunk of a request under variant k (its
    steady-state time per starting position times the positions per
    chunk): the batch planner queues long chunks first."""
    _, L, W, _ = VARIANTS[k]
    starts = max(n - m + 1, 1)
    if not np.isfinite(ms_per_request):
        return 0.0
    return float(ms_per_request / starts * min(starts, L * W) * 1e3)


def gbps(n: int, ms: np.ndarray) -> np.ndarray:
    with np.errstate(divide="ignore"):
        return np.where(np.isfinite(ms) & (ms > 0), n / (ms * 1e-3) / 1e9, 0.0)


__all__ = ["VARIANTS", "DEFAULT_VARIANT", "FEATURES", "PatternSetIndexes", "Tuner", "gbps",
           "variant_struct", "time_batch", "chunks_of"]
