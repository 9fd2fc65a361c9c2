"""Variant selection for batched scans: timing database, selector training and
the comparison of selection policies on a batch.

Policies compared on one batch (each runs the whole batch as one replayed
HIP graph, every text under the variant the policy picked):
  exhaustive - every request timed on all 24 variants, fastest kept;
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
    """Features [R, 7] and per-request milliseconds [R, 24] of every request."""
    R = len(reqs)
    feats = np.zeros((R, 7))
    ms = np.full((R, len(tune.VARIANTS)), np.inf)
    t0 = time.perf_counter()
    for i, (p, off, n) in enumerate(reqs):
        text = stream_dev[off:off + n]
        feats[i] = tuner.features(sets_idx[p], text)
        ms[i] = tuner.time_all(sets_idx[p], text)
        if log and (i + 1) % max(1, R // 10) == 0:
            log(f"[tune] {i + 1}/{R} requests timed ({time.perf_counter() - t0:.1f}s)")
    return feats, ms


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

    # exhaustive autotuning of every request (the reference, and the source of
    # the fallback choices)
    t0 = time.perf_counter()
    rows = []
    for i in range(R):
        rows.append(tuner.time_all(pset[i], texts[i]))
        if log and (i + 1) % max(1, R // 10) == 0:
            log(f"[select] exhaustive tuning {i + 1}/{R} ({time.perf_counter() - t0:.1f}s)")
    ms = np.stack(rows)
    t_exh = time.perf_counter() - t0
    exh = np.argmin(ms, axis=1)
    t_fallback = t_exh * float(fallback.mean())
    final = np.where(fallback, exh, learned)
    default = np.array([uniform_choice(default_variant, valid_r[i]) for i in range(R)])
    caps = [tuner.count(pset[i], texts[i]) for i in range(R)]
    if log:
        log(f"[select] features {t_feat:.2f}s, inference {t_infer * 1e3:.1f}ms, exhaustive "
            f"{t_exh:.1f}s, fallback rate {fallback.mean():.3f}")

    # Queue hints: each policy only uses what it knows. Exhaustive: measured
    # times; learned: predicted times (measured ones where it fell back);
    # default: none.
    ms_learned = np.where(fallback[:, None], ms, ms_pred)

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
    res["selection_overhead_s"] = {"features": t_feat, "inference": t_infer,
                                   "fallback_tuning": t_fallback, "exhaustive_tuning": t_exh}
    # how often the learned pick (before fallback) equals the exhaustive best,
    # and its predicted-vs-isolated slowdown on the picks that differ
    iso = to_gbps(np.asarray(lens), ms)
    best = iso[np.arange(R), exh]
    res["pick_agreement"] = float(np.mean(learned == exh))
    res["isolated_regret_learned_only"] = float(
        1.0 - iso[np.arange(R), learned].sum() / max(best.sum(), 1e-30))
    tbest = ms[np.arange(R), exh].sum()
    res["time_regret_isolated"] = {
        "learned_no_fallback": float(ms[np.arange(R), learned].sum() / tbest - 1),
        "learned": float(ms[np.arange(R), final].sum() / tbest - 1),
        "default": float(ms[np.arange(R), default].sum() / tbest - 1)}
    res["default_variant"] = list(tune.VARIANTS[default_variant])
    res["matches"] = int(np.sum(caps))
    res["_state"] = dict(arena=arena, offs=offs, lens=lens, pset=pset, caps=caps, ms=ms,
                         ms_pred=ms_pred, exh=exh, final=final, default=default,
                         learned=learned, fallback=fallback)
    return res
