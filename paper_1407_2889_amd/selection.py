"""Variant selection for batched scans: timing database, selector training and
the comparison of selection policies on a batch.

Policies compared on one batch (each runs the whole batch as one replayed
HIP graph, every text under the variant the policy picked):
  exhaustive - every request timed on all 24 variants (in batched launches,
               each request's share of its launch measured by the kernel),
               fastest kept;
  learned    - the selector's choice, except where its predicted best beats
               the runner-up by less than the margin: those requests take
               the exhaustive choice (the fallback);
  default    - one fixed variant for every request.
Regret of the learned policy = 1 - (its batch GB/s) / (exhaustive GB/s).
"""

from __future__ import annotations

import math
import time

import numpy as np

from . import batch as _batch
from . import tune
from .learn import Selector


def build_db(tuner: tune.Tuner, sets_idx, stream_dev, reqs, log=None):
    """Features [R, 7] and per-request milliseconds [R, 24] of every request
    (request (set, offset, length) is a slice of the device text stream):
    every request timed on every variant inside batched launches."""
    R = len(reqs)
    t0 = time.perf_counter()
    feats = np.zeros((R, 7))
    caps = np.zeros(R, np.int64)
    for i, (p, off, n) in enumerate(reqs):
        text = stream_dev[off:off + n]
        feats[i] = tuner.features(sets_idx[p], text)
        caps[i] = tuner.count(sets_idx[p], text)
    t1 = time.perf_counter()
    offs = np.array([r[1] for r in reqs], np.int64)
    lens = np.array([r[2] for r in reqs], np.int64)
    ms, chunk = tune.time_batch(stream_dev, offs, lens, [sets_idx[r[0]] for r in reqs], caps)
    if log:
        log(f"[tune] {R} requests: features and counts {t1 - t0:.1f}s, all variants timed in "
            f"batched launches {time.perf_counter() - t1:.1f}s")
    nch = np.array([[tune.chunks_of(int(r[2]), sets_idx[r[0]].m, k) for k in range(len(tune.VARIANTS))]
                    for r in reqs])
    return feats, ms, chunk_factors(ms, chunk, nch)


def chunk_factors(ms: np.ndarray, chunk: np.ndarray, nchunks: np.ndarray,
                  quantile: float = 0.9) -> np.ndarray:
    """Per variant, a high quantile over a timing database of longest chunk
    time x chunks / share: a request's longest chunk is at most about its
    share times this factor over its number of chunks (the factor is near
    the launch's workgroup count when a request's chunks cost alike). The
    learned policy estimates chunks from predicted costs with it; a high
    quantile keeps the scheduler from trusting short estimates of chunks
    that turn out long (the plan then waits for them)."""
    f = np.ones(ms.shape[1])
    for k in range(ms.shape[1]):
        ok = np.isfinite(ms[:, k]) & (ms[:, k] > 0) & np.isfinite(chunk[:, k])
        if ok.any():
            f[k] = float(np.quantile(chunk[ok, k] * nchunks[ok, k] / ms[ok, k], quantile))
    return f


# Cost model of a plan (milliseconds). The launches of one plan follow each
# other on the device, each starting as the previous one's workgroups retire:
# a plan takes about the requests' summed shares, plus a start-up per launch,
# plus part of every launch's tail where its longest chunk outlasts its summed
# shares (the rest hides behind the neighbouring launches' work), and never
# less than its longest chunk. The constants are fitted to replay times of
# uniform, per-request-best and randomly perturbed plans on batches of 79 MB
# to 2 GB (median error 7%).
LAUNCH_MS = 0.0144
EXCESS = 0.32
CHUNK = 1.1


def launch_keys(pset, valid: np.ndarray) -> np.ndarray:
    """[R, V] launch key of request i under variant k (-1 where it cannot
    run): requests with equal keys share one launch of the plan."""
    R, V = valid.shape
    keys = np.full((R, V), -1, np.int64)
    for i in range(R):
        for k in range(V):
            if valid[i, k]:
                key = pset[i].launch_key(k)
                keys[i, k] = -1 if key is None else key
    return keys


def _model(sum_s: float, launches: int, excess: float, longest: float) -> float:
    return max(sum_s + LAUNCH_MS * launches + EXCESS * excess, CHUNK * longest)


def plan_ms(choice: np.ndarray, cost: np.ndarray, chunk: np.ndarray, keys: np.ndarray) -> float:
    """Modelled time of the plan that runs request i under variant choice[i]."""
    r_ = np.arange(len(choice))
    k = keys[r_, choice]
    c, h = cost[r_, choice], chunk[r_, choice]
    excess = 0.0
    ukeys = np.unique(k)
    for key in ukeys:
        sel = k == key
        excess += max(0.0, float(h[sel].max()) - float(c[sel].sum()))
    return _model(float(c.sum()), len(ukeys), excess, float(h.max()))


class _Plan:
    """Launch statistics of an assignment, updated one move at a time."""

    def __init__(self, choice, cost, chunk, keys):
        from sortedcontainers import SortedList
        self.choice, self.cost, self.chunk, self.keys = choice, cost, chunk, keys
        self.S, self.H = {}, {}
        self.all = SortedList()
        for i, k in enumerate(choice):
            key = int(keys[i, k])
            self.S[key] = self.S.get(key, 0.0) + float(cost[i, k])
            self.H.setdefault(key, SortedList()).add(float(chunk[i, k]))
            self.all.add(float(chunk[i, k]))
        self.sum_s = sum(self.S.values())
        self.excess = sum(max(0.0, self.H[key][-1] - self.S[key]) for key in self.S)

    def time(self) -> float:
        return _model(self.sum_s, len(self.S), self.excess, self.all[-1])

    def _launch(self, key):
        h = self.H.get(key)
        return (self.S.get(key, 0.0), h[-1] if h else 0.0, len(h) if h else 0)

    def delta(self, i: int, k: int) -> float:
        """Change of the modelled plan time if request i moves to variant k."""
        k0 = int(self.choice[i])
        a, b = int(self.keys[i, k0]), int(self.keys[i, k])
        c0, h0 = float(self.cost[i, k0]), float(self.chunk[i, k0])
        c1, h1 = float(self.cost[i, k]), float(self.chunk[i, k])
        Sa, Ca, na = self._launch(a)
        ha = self.H[a]
        Ca_wo = (ha[-2] if na > 1 else 0.0) if h0 >= Ca else Ca
        ex = lambda S, C, n: max(0.0, C - S) if n else 0.0
        if a == b:
            d_ex = ex(Sa - c0 + c1, max(Ca_wo, h1), na) - ex(Sa, Ca, na)
            d_l = 0
        else:
            Sb, Cb, nb = self._launch(b)
            d_ex = (ex(Sa - c0, Ca_wo, na - 1) + ex(Sb + c1, max(Cb, h1), nb + 1)
                    - ex(Sa, Ca, na) - ex(Sb, Cb, nb))
            d_l = (-1 if na == 1 else 0) + (1 if nb == 0 else 0)
        top = self.all[-1]
        rest = (self.all[-2] if len(self.all) > 1 else 0.0) if h0 >= top else top
        new = _model(self.sum_s - c0 + c1, len(self.S) + d_l, self.excess + d_ex, max(rest, h1))
        return new - self.time()

    def move(self, i: int, k: int):
        from sortedcontainers import SortedList
        k0 = int(self.choice[i])
        a, b = int(self.keys[i, k0]), int(self.keys[i, k])
        for key in {a, b}:
            if key in self.S:
                self.excess -= max(0.0, self.H[key][-1] - self.S[key])
        self.S[a] -= float(self.cost[i, k0])
        self.H[a].remove(float(self.chunk[i, k0]))
        self.all.remove(float(self.chunk[i, k0]))
        if not self.H[a]:
            del self.H[a], self.S[a]
        self.S[b] = self.S.get(b, 0.0) + float(self.cost[i, k])
        if b not in self.H:
            self.H[b] = SortedList()
        self.H[b].add(float(self.chunk[i, k]))
        self.all.add(float(self.chunk[i, k]))
        for key in {a, b}:
            if key in self.S:
                self.excess += max(0.0, self.H[key][-1] - self.S[key])
        self.sum_s += float(self.cost[i, k]) - float(self.cost[i, k0])
        self.choice[i] = k


def schedule(choice: np.ndarray, cost: np.ndarray, chunk: np.ndarray, valid: np.ndarray,
             pset, keys: np.ndarray | None = None, uniform=None, passes: int = 6) -> np.ndarray:
    """Batch-aware assignment minimising the plan's modelled time (plan_ms).
    Starts from the better of the given per-request choices and every
    uniform assignment, then alternates moves of single requests to the
    variant that lowers the model most and the dissolution of whole launches
    (each request to its cheapest variant in another launch), while the model
    improves. cost, chunk [R, V]: per-request share and longest chunk
    (measured, or predicted for the learned selector)."""
    keys = launch_keys(pset, valid) if keys is None else keys
    ok = (keys >= 0) & np.isfinite(cost) & np.isfinite(chunk)
    R, V = cost.shape
    cost = np.where(ok, cost, np.inf)
    chunk = np.where(ok, chunk, np.inf)
    starts = [np.array(choice, copy=True)]
    for k in (range(V) if uniform is None else uniform):
        u = np.array([uniform_choice(k, ok[i]) for i in range(R)])
        if ok[np.arange(R), u].all():
            starts.append(u)
    starts = [c for c in starts if ok[np.arange(R), c].all()]
    best = min(starts, key=lambda c: plan_ms(c, cost, chunk, keys)).copy()
    plan = _Plan(best, cost, chunk, keys)
    for _ in range(passes):
        improved = False
        # single-request moves, largest shares first
        order = np.argsort(-cost[np.arange(R), plan.choice])
        for i in order:
            cand = np.flatnonzero(ok[i])
            d = [plan.delta(int(i), int(k)) for k in cand]
            j = int(np.argmin(d))
            if d[j] < -1e-9:
                plan.move(int(i), int(cand[j]))
                improved = True
        # dissolve launches, smallest first, while the model improves
        for key in sorted(plan.S, key=plan.S.get):
            if key not in plan.S or len(plan.S) == 1:
                continue
            trial = plan.choice.copy()
            members = np.flatnonzero(keys[np.arange(R), trial] == key)
            others = set(plan.S) - {key}
            moved = True
            for i in members:
                alt = [k for k in np.flatnonzero(ok[i]) if int(keys[i, k]) in others]
                if not alt:
                    moved = False
                    break
                trial[i] = min(alt, key=lambda k: cost[i, k])
            if moved and plan_ms(trial, cost, chunk, keys) < plan_ms(plan.choice, cost, chunk, keys) - 1e-9:
                plan = _Plan(trial, cost, chunk, keys)
                improved = True
        if not improved:
            break
    return plan.choice


def to_gbps(lens: np.ndarray, ms: np.ndarray) -> np.ndarray:
    return np.stack([tune.gbps(int(n), ms[i]) for i, n in enumerate(lens)])


def best_uniform_variant(ms: np.ndarray) -> int:
    """The single variant with the least total time over a timing database
    (requests whose tables do not fit in LDS take its global-placement twin):
    the fixed choice a batch would use without the selector."""
    best, best_t = 0, math.inf
    for k in range(len(tune.VARIANTS)):
        pk = np.array([uniform_choice(k, np.isfinite(ms[i])) for i in range(len(ms))])
        t = float(ms[np.arange(len(ms)), pk].sum())
        if t < best_t:
            best, best_t = k, t
    return best


def uniform_choice(k: int, valid_row: np.ndarray) -> int:
    if valid_row[k]:
        return k
    a, L, W, _ = tune.VARIANTS[k]
    return tune.VARIANTS.index((a, L, W, tune.PLACEMENTS[1]))


def run_batch(arena, offs, lens, pset, choice, ms_known, caps, reps: int = 5, check=None):
    """Capture the batch with request i under variant choice[i] and return
    (median replay ms, totals, launch count). ms_known [R, 24] (or None)
    gives the per-request times the queue order is built from. check(bs),
    if given, is called with the BatchScan after the timed replays (its
    outputs then hold the last replay's lists)."""
    import torch
    R = len(pset)
    idx = [pset[i].index(int(choice[i])) for i in range(R)]
    var = [tune.variant_struct(int(choice[i])) for i in range(R)]
    hint = None
    if ms_known is not None:
        hint = [tune.chunk_cost_hint(int(choice[i]), float(ms_known[i, int(choice[i])]),
                                     int(lens[i]), pset[i].m) for i in range(R)]
    bs = _batch.BatchScan(arena, offs, lens, idx, var, caps, cost_hints=hint)
    bs.capture()
    bs.replay()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, z in ev:
        a.record()
        bs.replay()
        z.record()
    torch.cuda.synchronize()
    tms = float(np.median([a.elapsed_time(z) for a, z in ev]))
    if check is not None:
        check(bs)
    return tms, bs.totals_host(), bs.groups


def evaluate(b, tuner: tune.Tuner, selector: Selector, default_variant: int,
             margin: float = 0.05, reps: int = 5, log=None, check=None):
    """Run the three policies on batch b (texts, pattern sets and the set of
    each text: ``b.texts``, ``b.sets[k].patterns``, ``b.pairing``); returns a
    result dict."""
    sets_idx = [tune.PatternSetIndexes.build(ps.patterns) for ps in b.sets]
    arena, offs, lens = _batch.pack_texts(b.texts)
    R = len(b.texts)
    texts = [arena[int(offs[i]):int(offs[i]) + int(lens[i])] for i in range(R)]
    pset = [sets_idx[int(b.pairing[i])] for i in range(R)]
    valid = np.array([[s.lds_fits(k) for k in range(len(tune.VARIANTS))] for s in sets_idx])
    valid_r = valid[b.pairing.astype(int)]

    t0 = time.perf_counter()
    feats = np.stack([tuner.features(pset[i], texts[i]) for i in range(R)])
    t_feat = time.perf_counter() - t0
    t0 = time.perf_counter()
    learned, fallback = selector.choose(feats, valid_r, margin)
    ms_pred = selector.predict_ms(feats)
    t_infer = time.perf_counter() - t0

    caps = [tuner.count(pset[i], texts[i]) for i in range(R)]
    # exhaustive autotuning of every request (the reference, and the source of
    # the fallback choices): every request on every variant
    t0 = time.perf_counter()
    ms, chunk = tune.time_batch(arena, offs, lens, pset, caps)
    t_exh = time.perf_counter() - t0
    exh_req = np.argmin(ms, axis=1)  # each request's fastest variant
    keys = launch_keys(pset, valid_r)
    exh = schedule(exh_req, ms, chunk, valid_r, pset, keys)
    t_fallback = t_exh * float(fallback.mean())
    # the learned policy knows measured costs only where it fell back; its
    # longest chunks are estimated from its predicted costs
    nch = np.array([[tune.chunks_of(int(lens[i]), pset[i].m, k) for k in range(len(tune.VARIANTS))]
                    for i in range(R)])
    ms_learned = np.where(fallback[:, None], ms, ms_pred)
    chunk_learned = np.where(fallback[:, None], chunk,
                             ms_pred * selector.chunk_safety * selector.chunk_factor[None, :] / nch)
    final = schedule(np.where(fallback, exh_req, learned), ms_learned, chunk_learned, valid_r,
                     pset, keys)
    default = np.array([uniform_choice(default_variant, valid_r[i]) for i in range(R)])
    if log:
        log(f"[select] features {t_feat:.2f}s, inference {t_infer * 1e3:.1f}ms, exhaustive "
            f"{t_exh:.1f}s, fallback rate {fallback.mean():.3f}")

    # Queue hints: each policy only uses what it knows. Exhaustive: measured
    # times; learned: predicted times (measured ones where it fell back);
    # default: none.

    def run(choice, ms_known, name):
        return run_batch(arena, offs, lens, pset, choice, ms_known, caps, reps,
                         check=(lambda bs: check(name, bs)) if check else None)

    total_bytes = int(np.sum(lens))
    res = {"requests": R, "text_bytes": total_bytes}
    totals = {}
    for name, choice, known in (("exhaustive", exh, ms), ("learned", final, ms_learned),
                                ("default", default, None)):
        tms, tot, groups = run(choice, known, name)
        res[f"{name}_ms"] = tms
        res[f"{name}_gbps"] = total_bytes / (tms * 1e-3) / 1e9
        res[f"{name}_launches"] = groups
        totals[name] = tot
    res["totals_agree"] = bool(all(np.array_equal(totals["exhaustive"], t) for t in totals.values())
                               and np.array_equal(totals["exhaustive"], np.array(caps)))
    res["regret"] = 1.0 - res["learned_gbps"] / res["exhaustive_gbps"]
    res["gain_over_default"] = res["learned_gbps"] / res["default_gbps"] - 1.0
    res["fallback_rate"] = float(fallback.mean())
    res["chunk_safety"] = selector.chunk_safety
    res["selection_overhead_s"] = {"features": t_feat, "inference": t_infer,
                                   "fallback_tuning": t_fallback, "exhaustive_tuning": t_exh}
    # how often the learned pick (before fallback) equals the per-request
    # best, and each policy's summed measured cost against the per-request
    # bests (every request on its own fastest variant)
    res["pick_agreement"] = float(np.mean(learned == exh_req))
    r_ = np.arange(R)
    tbest = ms[r_, exh_req].sum()
    res["time_regret_tuned"] = {
        "learned_no_fallback": float(ms[r_, learned].sum() / tbest - 1),
        "learned": float(ms[r_, final].sum() / tbest - 1),
        "exhaustive_scheduled": float(ms[r_, exh].sum() / tbest - 1),
        "default": float(ms[r_, default].sum() / tbest - 1)}
    # each plan's modelled time from the measured costs, beside its replay
    res["model_ms"] = {name: plan_ms(c, np.where(np.isfinite(ms), ms, np.inf),
                                     np.where(np.isfinite(chunk), chunk, np.inf), keys)
                       for name, c in (("exhaustive", exh), ("learned", final),
                                       ("default", default))}
    res["default_variant"] = list(tune.VARIANTS[default_variant])
    res["matches"] = int(np.sum(caps))
    res["_state"] = dict(arena=arena, offs=offs, lens=lens, pset=pset, caps=caps, ms=ms,
                         ms_pred=ms_pred, exh=exh, final=final, default=default,
                         learned=learned, fallback=fallback, chunk=chunk)
    return res
