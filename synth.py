"""Seeded synthetic inputs for exact multiple pattern matching.

This module only draws random bytes: texts and pattern sets shaped like the
paper's workload (Section 5: a DNA string over a four-letter alphabet, pattern
sets made of substrings of the text). It holds none of the matching method's
arithmetic, so both the CPU oracle and the GPU path can take their inputs from
it without sharing any code with each other.

Workloads (all seeded, numpy PCG64):

* ``uniform_dna(n, seed)``: i.i.d. uniform bytes over ``ACGT``.
* ``est_text(n, seed)``: EST-shaped text. Records have log-normal lengths with
  arithmetic mean 500 (mu = ln 500 - sigma^2/2, sigma = 0.5, rounded, at least
  1). Record bytes are A/C/G/T with probability 0.2475 each and N with 0.01.
  Each record is followed by a newline; the last record is cut to hit ``n``.
* ``pattern_set(text, d, m, n_planted, seed)``: ids ``0..n_planted-1`` are
  windows of the text at uniform random starts (a start whose window holds a
  newline is drawn again), the remaining ids are uniform random ``ACGT``
  strings. Planted starts are returned so tests can check each occurrence.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)
ACGTN = np.frombuffer(b"ACGTN", dtype=np.uint8)
NEWLINE = 10
MiB = 1 << 20
GiB = 1 << 30


def uniform_dna(n: int, seed: int) -> np.ndarray:
    """i.i.d. uniform text over ACGT (uint8[n])."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.uint8)
    step = 64 * MiB
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        out[lo:hi] = ACGT[rng.integers(0, 4, hi - lo, dtype=np.uint8)]
    return out


def est_text(n: int, seed: int, mean_len: float = 500.0, sigma: float = 0.5,
             p_n: float = 0.01) -> np.ndarray:
    """EST-shaped DNA text (uint8[n]): log-normal records, 1% N, newline separators."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.uint8)
    # byte = LUT[uniform integer in [0, 400)]: 99/400 = 0.2475 for each base,
    # 4/400 = 0.01 for N (p_n is fixed at 0.01 by this table)
    assert abs(p_n - 0.01) < 1e-12, "the lookup table encodes 1% N"
    lut = np.empty(400, dtype=np.uint8)
    lut[0:99], lut[99:198], lut[198:297], lut[297:396], lut[396:400] = ACGTN
    step = 64 * MiB
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        out[lo:hi] = lut[rng.integers(0, 400, hi - lo, dtype=np.uint16)]
    mu = math.log(mean_len) - 0.5 * sigma * sigma
    # record lengths until the text is covered; '\n' follows each record
    pos = 0
    newlines = []
    while pos < n:
        k = max(1024, int((n - pos) / (mean_len + 1) * 1.05) + 64)
        lens = np.maximum(1, np.rint(rng.lognormal(mu, sigma, k))).astype(np.int64)
        ends = pos + np.cumsum(lens + 1) - 1  # index of the '\n' after each record
        ends = ends[ends < n]
        newlines.append(ends)
        if len(ends) < k:
            break
        pos = int(ends[-1]) + 1
    if newlines:
        nl = np.concatenate(newlines)
        out[nl] = NEWLINE
    return out


@dataclass
class PatternSet:
    patterns: np.ndarray          # uint8[d, m]
    planted_starts: np.ndarray    # int64[n_planted]; pattern i == text[s : s + m]
    m: int
    d: int
    seed: int


def pattern_set(text: np.ndarray, d: int, m: int, n_planted: int, seed: int,
                texts: list | None = None) -> PatternSet:
    """d patterns of length m: n_planted text windows first, then uniform ACGT.

    If ``texts`` is given (a list of uint8 arrays), each planted pattern is cut
    from one of them chosen uniformly; ``planted_starts`` then refer to that
    text and ``planted_text`` records which one.
    """
    rng = np.random.default_rng(seed)
    pats = np.empty((d, m), dtype=np.uint8)
    starts = np.empty(n_planted, dtype=np.int64)
    srcs = np.zeros(n_planted, dtype=np.int64)
    pool = texts if texts is not None else [text]
    for i in range(n_planted):
        for _ in range(10000):
            t = int(rng.integers(0, len(pool))) if len(pool) > 1 else 0
            src = pool[t]
            if len(src) < m:
                continue
            s = int(rng.integers(0, len(src) - m + 1))
            w = src[s:s + m]
            if not (w == NEWLINE).any():
                break
        else:
            raise ValueError("could not plant a newline-free window")
        pats[i] = w
        starts[i] = s
        srcs[i] = t
    if d > n_planted:
        pats[n_planted:] = ACGT[rng.integers(0, 4, (d - n_planted, m), dtype=np.uint8)]
    ps = PatternSet(pats, starts, m, d, seed)
    ps.planted_text = srcs  # type: ignore[attr-defined]
    return ps


def mixed_pattern_set(text: np.ndarray, d: int, lo: int, hi: int, n_planted: int, seed: int,
                      n_prefix: int = 0, n_suffix: int = 0, n_dup: int = 0) -> list:
    """d patterns (bytes) of lengths drawn uniformly from [lo, hi]: n_planted
    newline-free text windows, then n_prefix leading parts and n_suffix
    trailing parts (at least lo long) of planted ones, n_dup copies of planted
    ones, and uniform ACGT strings for the rest, in a seeded shuffled order."""
    rng = np.random.default_rng(seed)
    pats = []
    for _ in range(n_planted):
        m = int(rng.integers(lo, hi + 1))
        for _ in range(10000):
            s = int(rng.integers(0, len(text) - m + 1))
            w = text[s:s + m]
            if not (w == NEWLINE).any():
                break
        else:
            raise ValueError("could not plant a newline-free window")
        pats.append(w.tobytes())
    base = list(pats)
    for _ in range(n_prefix):
        p = base[int(rng.integers(0, len(base)))]
        pats.append(p[:int(rng.integers(lo, len(p) + 1))])
    for _ in range(n_suffix):
        p = base[int(rng.integers(0, len(base)))]
        pats.append(p[len(p) - int(rng.integers(lo, len(p) + 1)):])
    for _ in range(n_dup):
        pats.append(base[int(rng.integers(0, len(base)))])
    while len(pats) < d:
        m = int(rng.integers(lo, hi + 1))
        pats.append(ACGT[rng.integers(0, 4, m)].tobytes())
    order = rng.permutation(len(pats))
    return [pats[i] for i in order[:d]]


# ---------------------------------------------------------------------------
# Named workloads. Sizes follow the paper's problem shape (Section 5: a 1 GiB
# DNA string, m = 8, d in the thousands) scaled to the cases used here.
# ---------------------------------------------------------------------------

def workload_small():
    """1 MiB uniform ACGT (seed 0); d=100, m=8, 50 planted + 50 random (seed 1)."""
    text = uniform_dna(MiB, seed=0)
    ps = pattern_set(text, d=100, m=8, n_planted=50, seed=1)
    return text, ps


def workload_est256(n: int = 256 * MiB):
    """256 MiB EST-shaped text (seed 2); d=1000, m=16, 300 planted (seed 3)."""
    text = est_text(n, seed=2)
    ps = pattern_set(text, d=1000, m=16, n_planted=300, seed=3)
    return text, ps


SWEEP_D = (1000, 10000, 100000)
SWEEP_M = (8, 16, 32)


def workload_sweep_text(n: int = GiB):
    """1 GiB EST-shaped text (seed 4) for the pattern-set sweep."""
    return est_text(n, seed=4)


def workload_sweep_set(text: np.ndarray, d: int, m: int) -> PatternSet:
    """Sweep pattern set (d, m) with 10% planted; seeds 10..18 in (d, m) order."""
    k = SWEEP_D.index(d) * len(SWEEP_M) + SWEEP_M.index(m)
    return pattern_set(text, d=d, m=m, n_planted=d // 10, seed=10 + k)


@dataclass
class Batch:
    texts: list                    # list of uint8 arrays
    sets: list                     # list of PatternSet
    pairing: np.ndarray            # int64[len(texts)]: set index per text
    meta: dict = field(default_factory=dict)


BATCH_M_CHOICES = (8, 12, 16, 24, 32)


def batch_request_shapes(n_texts: int, n_sets: int, seed_len: int, seed_sets: int,
                         min_len: int = 1024, max_len: int = 4 * MiB,
                         d_lo: int = 100, d_hi: int = 50000):
    """Text lengths (log-uniform) and per-set (d, m) for a batched workload."""
    rng = np.random.default_rng(seed_len)
    lens = np.exp(rng.uniform(math.log(min_len), math.log(max_len), n_texts))
    lens = np.rint(lens).astype(np.int64)
    rs = np.random.default_rng(seed_sets)
    ds = np.rint(np.exp(rs.uniform(math.log(d_lo), math.log(d_hi), n_sets))).astype(np.int64)
    ms = np.array(BATCH_M_CHOICES)[rs.integers(0, len(BATCH_M_CHOICES), n_sets)]
    return lens, ds, ms


def workload_batch(n_texts: int = 4096, n_sets: int = 64, max_len: int = 4 * MiB,
                   d_hi: int = 50000, seed: int = 20) -> Batch:
    """Batched workload: EST-shaped texts of log-uniform length, each paired with
    one of ``n_sets`` pattern sets (d log-uniform, m from {8,12,16,24,32}, 10%
    planted from the texts that use the set). Seeds: lengths/texts ``seed``,
    sets ``seed+1``, pairing ``seed+2``."""
    lens, ds, ms = batch_request_shapes(n_texts, n_sets, seed, seed + 1,
                                        max_len=max_len, d_hi=d_hi)
    # one long EST stream cut into the texts keeps generation cheap and seeded
    total = int(lens.sum())
    stream = est_text(total, seed=seed)
    offs = np.concatenate([[0], np.cumsum(lens)])
    texts = [stream[offs[i]:offs[i + 1]] for i in range(n_texts)]
    pairing = np.random.default_rng(seed + 2).integers(0, n_sets, n_texts)
    sets = []
    for k in range(n_sets):
        users = [texts[i] for i in np.nonzero(pairing == k)[0] if len(texts[i]) >= ms[k]]
        pool = users if users else [texts[0]]
        d = int(ds[k])
        sets.append(pattern_set(pool[0], d=d, m=int(ms[k]), n_planted=d // 10,
                                seed=seed + 100 + k, texts=pool))
    return Batch(texts, sets, pairing, {"lens": lens, "offsets": offs, "stream": stream})


def selector_training_requests(n_req: int, n_sets: int, seed: int,
                                stream_bytes: int = 256 << 20, max_len: int = 4 << 20,
                                d_hi: int = 50000):
    """Seeded requests for the variant selector's timing database, drawn from
    the batched workload's distributions: text slices of one EST-shaped stream
    (256-byte aligned starts, log-uniform lengths) paired with a pool of
    pattern sets. Returns (stream, sets, [(set, offset, length), ...])."""
    lens, ds, ms = batch_request_shapes(n_req, n_sets, seed, seed + 1, max_len=max_len,
                                        d_hi=d_hi)
    stream = est_text(stream_bytes, seed=seed + 2)
    rng = np.random.default_rng(seed + 3)
    offs = (rng.integers(0, stream_bytes - lens + 1) // 256 * 256).astype(np.int64)
    pair = rng.integers(0, n_sets, n_req)
    sets = []
    for k in range(n_sets):
        d = int(ds[k])
        sets.append(pattern_set(stream, d=d, m=int(ms[k]), n_planted=d // 10,
                                seed=seed + 100 + k))
    return stream, sets, list(zip(pair.tolist(), offs.tolist(), lens.tolist()))
