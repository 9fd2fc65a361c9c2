"""Write the full-size expected values of the sweep and batch workloads.

Calls only the CPU oracle (``oracle/``) and the seeded input generator
(``synth``): no value here comes from the GPU library. For every list it
stores the total number of pairs, an order-sensitive 64-bit digest of the
whole sorted (position, id) list (``listdigest``), and, for the sweep, the
per-pattern occurrence counts (their SHA-256 plus summary values) and the
first and last pairs. The lists are those of the Definition in Section 1 of
the paper, computed by the oracle's sorted-window scan over contiguous ranges
of starting positions (the paper's split between workers, Section 4.4) and
concatenated in range order.

    python tests/golden/make_digests.py sweep   # 1 GiB text, nine pattern sets
    python tests/golden/make_digests.py batch   # 4,096 texts, 64 pattern sets
"""

from __future__ import annotations

import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import oracle  # noqa: E402
import synth  # noqa: E402
from listdigest import digest_np  # noqa: E402

WORKERS = min(16, os.cpu_count() or 1)
RANGE = 32 << 20  # starting positions per piece of the streamed compare
EDGE = 64         # pairs kept from each end of a list
SPOTS = 16        # per-pattern counts kept by value


def say(*a):
    print(*a, flush=True)


def sha256_bytes(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def list_summary(win, text: np.ndarray, d: int, m: int) -> dict:
    """Streamed summary of the oracle's list for the whole text."""
    n = len(text)
    ns = max(0, n - m + 1)
    counts = np.zeros(d, np.int64)
    digest, total = 0, 0
    head, tail = [], []
    for lo in range(0, ns, RANGE):
        hi = min(ns, lo + RANGE)
        pos, ids = oracle.parallel_scan(win, text, lo, hi, workers=WORKERS)
        counts += np.bincount(ids, minlength=d)[:d]
        digest = (digest + digest_np(pos, ids, total)) & ((1 << 64) - 1)
        if len(head) < EDGE:
            head += [[int(p), int(i)] for p, i in zip(pos[:EDGE - len(head)], ids)]
        if len(pos):
            tail = (tail + [[int(p), int(i)] for p, i in zip(pos[-EDGE:], ids[-EDGE:])])[-EDGE:]
        total += len(pos)
    rng = np.random.default_rng(d * 1000 + m)
    spot_ids = sorted({0, d - 1, *rng.integers(0, d, SPOTS - 2).tolist()})
    return {
        "total": int(total),
        "digest": f"{digest:016x}",
        "counts_sha256": sha256_bytes(counts.astype("<u4")),
        "patterns_hit": int((counts > 0).sum()),
        "max_count": int(counts.max()) if d else 0,
        "spot_counts": {str(i): int(counts[i]) for i in spot_ids},
        "head": head,
        "tail": tail,
    }


def make_sweep(path: str):
    t0 = time.perf_counter()
    say("[golden] sweep text (1 GiB EST-shaped, seed 4)")
    text = synth.workload_sweep_text()
    rec = {"what": "pattern-set sweep, 1 GiB EST-shaped text (seed 4), d in {1000, 10000, "
                   "100000} x m in {8, 16, 32}, 10% planted (seeds 10-18)",
           "n": len(text), "text_sha256": sha256_bytes(text), "sets": []}
    for d in synth.SWEEP_D:
        for m in synth.SWEEP_M:
            ps = synth.workload_sweep_set(text, d, m)
            s0 = time.perf_counter()
            with oracle.Win(ps.patterns) as win:
                summ = list_summary(win, text, d, m)
            summ.update({"d": d, "m": m, "patterns_sha256": sha256_bytes(ps.patterns)})
            rec["sets"].append(summ)
            say(f"[golden] d={d} m={m}: {summ['total']} pairs, digest {summ['digest']} "
                f"({time.perf_counter() - s0:.1f}s)")
            with open(path, "w") as f:
                json.dump(rec, f, indent=1)
    say(f"[golden] sweep done in {time.perf_counter() - t0:.0f}s -> {path}")


def make_batch(path: str):
    t0 = time.perf_counter()
    say("[golden] batch (4,096 texts, 64 sets, seeds 20-22)")
    b = synth.workload_batch(n_texts=4096, n_sets=64, seed=20)
    wins = [oracle.Win(ps.patterns) for ps in b.sets]
    R = len(b.texts)

    def one(i):
        win = wins[int(b.pairing[i])]
        t = b.texts[i]
        pos, ids = win.scan(t)
        return len(pos), digest_np(pos, ids, 0)

    with ThreadPoolExecutor(WORKERS) as ex:
        res = list(ex.map(one, range(R)))
    rec = {"what": "batched workload: 4,096 EST-shaped texts, log-uniform 1 KiB-4 MiB (seed "
                   "20), 64 pattern sets d log-uniform 100-50k, m in {8,12,16,24,32}, 10% "
                   "planted (seed 21), pairing seed 22",
           "texts": R,
           "stream_sha256": sha256_bytes(b.meta["stream"]),
           "patterns_sha256": [sha256_bytes(ps.patterns) for ps in b.sets],
           "pairing": [int(x) for x in b.pairing],
           "total": int(sum(c for c, _ in res)),
           "counts": [int(c) for c, _ in res],
           "digests": [f"{g:016x}" for _, g in res]}
    with open(path, "w") as f:
        json.dump(rec, f)
    say(f"[golden] batch: {rec['total']} pairs in {R} lists ({time.perf_counter() - t0:.0f}s) "
        f"-> {path}")


if __name__ == "__main__":
    which = sys.argv[1:] or ["sweep", "batch"]
    if "sweep" in which:
        make_sweep(os.path.join(HERE, "sweep_digests.json"))
    if "batch" in which:
        make_batch(os.path.join(HERE, "batch_digests.json"))
