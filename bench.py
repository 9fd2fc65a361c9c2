"""Benchmark: text GB/s of the HIP multi-pattern scan on one MI355X.

Default workload (one step = one Aho-Corasick scan plus one Wu-Manber scan of
the same text, each producing the full sorted (position, id) list):
256 MiB EST-shaped DNA text (log-normal records of mean 500, 1% N, newline
separators; seed 2) against d = 1000 patterns of m = 16 (300 planted text
windows + 700 random; seed 3). Inputs are resident in HBM before timing.

Prints one JSON line. `value` is whole-step text throughput: 2 n bytes
scanned (n by AC, n by WM) per second. The line also carries the roofline of
the dominant kernel (HIP events on the launch stream), the batched workload's
learned-versus-exhaustive selection (batch_* keys; 4,096 texts, 64 pattern
sets, every policy's lists checked against the oracle's) and the CPU oracle's
throughput on the same text (one thread per usable host CPU, at most one
GPU's share of the host: 16).

Other workloads (one JSON line each):
  --workload sweep   1 GiB EST-shaped text against nine pattern sets
                     (d in {1k, 10k, 100k} x m in {8, 16, 32}), AC and WM;
  --workload batch   4,096 texts with 64 pattern sets run as one replayed
                     graph per selection policy (exhaustive autotune, learned
                     selector with fallback, fixed default), after a timing
                     database of --train-requests requests trains the selector.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--workload est256|small|sweep|batch]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s

DEFAULT_VARIANTS = {
    "ac": dict(lane_bytes=1024, block_threads=1024, placement=0),
    "wm": dict(lane_bytes=1024, block_threads=1024, placement=0),
}
# Dense output (MPM_VARIANT_DENSE): for sets with many occurrences per position.
DENSE_VARIANT = dict(block_threads=1024, placement=0, flags=8)

METRIC = "text GB/s scanned (AC, WM) + %HBM roofline; learned vs exhaustive-tuned GB/s"


# The sources the single-text AC and WM scan kernels and their launches are
# built from (the kernels' template code, its launch and workspace set-up).
SCAN_SOURCES = ("mpm_internal.h", "mpm_scan_impl.h", "mpm_scan.hip", "mpm_scan_ac16_lds.hip",
                "mpm_scan_wm.hip", "mpm_host.cpp")


def kernel_digest() -> str:
    """Hash of the sources of the single-text scan kernels and their launch:
    counter records taken from an older build stop applying once it
    changes."""
    import hashlib
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1407_2889_amd", "csrc")
    h = hashlib.sha256()
    for f in SCAN_SOURCES:
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str, algo: str):
    """HBM bytes per launch of the `algo` scan kernel on `workload` from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE record (each scaled by the
    same counter's reading for a kernel of known traffic), or None when there
    is no record or the kernels changed since it was taken."""
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                     f"scan_{workload}_hbm_counters.md")
    try:
        with open(p) as f:
            rec = next(json.loads(l[len("counters: "):]) for l in f if l.startswith("counters: "))
    except (OSError, StopIteration, ValueError):
        return None
    if rec.get("digest") != kernel_digest() or algo not in rec.get("kernels", {}):
        return None
    k = rec["kernels"][algo]
    return int(round(1024 * (k["fetch_kib"] * rec["fetch_factor"] + k["write_kib"] * rec["write_factor"])))


# MI355X compute units and engine clock (GHz) for the LDS ceiling.
CUS, CLOCK_GHZ = 256, 2.4


def recorded_lds(workload: str, algo: str):
    """LDS-active cycles per wave-wide LDS read and LDS reads per 64 text
    bytes of the `algo` scan kernel on `workload`, from the committed
    rocprofv3 record (SQ_LDS_IDX_ACTIVE / SQ_INSTS_LDS, bank conflicts
    included), or None when absent or taken from older kernel sources."""
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                     f"scan_{workload}_lds_counters.md")
    try:
        with open(p) as f:
            rec = next(json.loads(l[len("lds: "):]) for l in f if l.startswith("lds: "))
    except (OSError, StopIteration, ValueError):
        return None
    if rec.get("digest") != kernel_digest() or algo not in rec.get("kernels", {}):
        return None
    return rec["kernels"][algo]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden")


def golden(name: str):
    """Expected values of a full-size workload written from the CPU oracle
    alone (tests/golden/make_digests.py), or None when absent."""
    try:
        with open(os.path.join(GOLDEN_DIR, f"{name}_digests.json")) as f:
            return json.load(f)
    except OSError:
        return None


def listdigest():
    """The order-sensitive list digest the expected values use."""
    if GOLDEN_DIR not in sys.path:
        sys.path.insert(0, GOLDEN_DIR)
    import listdigest as ld
    return ld


def workload(name: str):
    import synth
    if name == "est256":
        text, ps = synth.workload_est256()
        desc = ("EST-shaped DNA text 256 MiB (log-normal records mean 500, 1% N, '\\n' "
                "separators), d=1000 patterns m=16 (30% planted)")
    elif name == "small":
        text, ps = synth.workload_small()
        desc = "uniform ACGT text 1 MiB, d=100 patterns m=8 (50% planted)"
    else:
        raise SystemExit(f"unknown workload {name}")
    return text, ps, desc


# Host threads one GPU's share of the GPU host gives a process (the host runs
# one such share per GPU, whatever the operating system reports as online).
HOST_SHARE_THREADS = 16


def host_cpus() -> dict:
    """What the host reports: online CPUs, CPUs this process may run on."""
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = os.cpu_count() or 1
    return {"online": os.cpu_count() or 1, "affinity": aff}


def cpu_baseline(text, P, sample_bytes: int):
    """The CPU oracle (literal AC and WM, as written) on the host cores: the
    text split into contiguous ranges with the m - 1 overlap (the paper's
    split between nodes, Section 4.4) on one thread per CPU this process may
    use, capped at one GPU's share of the host; single-thread rates of a
    smaller prefix are given in `sample`."""
    import oracle
    s = text[:sample_bytes]
    cpus = host_cpus()
    workers = max(1, min(HOST_SHARE_THREADS, cpus["affinity"]))
    ac, wm = oracle.AC(P), oracle.WM(P)
    t0 = time.perf_counter()
    oracle.parallel_scan(ac, s, workers=workers)
    t1 = time.perf_counter()
    oracle.parallel_scan(wm, s, workers=workers)
    t2 = time.perf_counter()
    one = s[: min(len(s), 32 << 20)]
    u0 = time.perf_counter()
    ac.scan(one)
    u1 = time.perf_counter()
    wm.scan(one)
    u2 = time.perf_counter()
    return {
        "value": round(2 * len(s) / (t2 - t0) / 1e9, 5),
        "unit": "GB/s",
        "cores": workers,
        "host_cpus_online": cpus["online"],
        "host_cpus_affinity": cpus["affinity"],
        "kind": "oracle",
        "sample": f"first {len(s)} bytes of the same text on {workers} threads (contiguous "
                  f"ranges with the m-1 overlap): oracle AC (Algorithms 1-3) "
                  f"{len(s) / (t1 - t0) / 1e9:.4f} GB/s, oracle WM (Algorithms 4-5, B=3) "
                  f"{len(s) / (t2 - t1) / 1e9:.4f} GB/s; one thread on the first {len(one)} "
                  f"bytes: AC {len(one) / (u1 - u0) / 1e9:.4f}, WM {len(one) / (u2 - u1) / 1e9:.4f} GB/s",
    }


def time_scans(sc, dev_text, steps: int, warmup: int, stream) -> float:
    """Mean kernel milliseconds of `steps` scans (HIP events on the stream)."""
    import torch
    for _ in range(warmup):
        sc.scan_async(dev_text)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record(stream)
        sc.scan_async(dev_text)
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def run_sweep(args):
    """Pattern-set sweep: 1 GiB EST-shaped text, d in {1k, 10k, 100k} x m in
    {8, 16, 32}, 10% planted; every (set, algorithm) scanned with the full
    sorted list written. One JSON line with one record per (set, algorithm):
    text GB/s, the HBM roofline fraction of the algorithmic bytes, the match
    count, and a digest of the per-pattern counts (counted on the device from
    the list, timed separately as count_ms)."""
    import torch
    import paper_1407_2889_amd as mpm
    import synth
    log("[bench] generating 1 GiB EST-shaped text")
    text = synth.workload_sweep_text()
    n = len(text)
    gold = golden("sweep")
    if gold is not None:
        import hashlib
        if hashlib.sha256(text.tobytes()).hexdigest() != gold["text_sha256"]:
            gold = None  # the generator changed: no expected values for this text
    dev = torch.from_numpy(text).cuda()
    stream = torch.cuda.current_stream()
    rows = []
    t_all = 0.0
    only = ({tuple(int(x) for x in dm.split(":")) for dm in args.sweep_sets.split(",")}
            if args.sweep_sets else None)
    for d in synth.SWEEP_D:
        for m in synth.SWEEP_M:
            if only is not None and (d, m) not in only:
                continue
            ps = synth.workload_sweep_set(text, d, m)
            lists = {}
            for algo in ("ac", "wm"):
                t0 = time.perf_counter()
                ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(ps.patterns, upload=True)
                build_s = time.perf_counter() - t0
                info = ix.info()
                v0 = mpm.variant(**DEFAULT_VARIANTS[algo])
                count = mpm.Scanner(ix, n, 0, v0)
                count.scan_async(dev)
                torch.cuda.synchronize()
                M = int(count.total.item())
                del count
                by_variant, best = {}, None
                for vname, vdict in (("default", DEFAULT_VARIANTS[algo]), ("dense", DENSE_VARIANT)):
                    v = mpm.variant(**vdict)
                    sc = mpm.Scanner(ix, n, M, v)
                    kms = time_scans(sc, dev, args.steps, args.warmup, stream)
                    t_all += kms * args.steps
                    if int(sc.total.item()) != M:
                        raise SystemExit(f"d={d} m={m} {algo} {vname}: {int(sc.total.item())} "
                                         f"pairs, the counting scan found {M}")
                    cbuf = torch.empty(d, dtype=torch.int32, device=dev.device)
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                    mpm.count_ids(sc.out[:M], d, out=cbuf)
                    ev[0].record(stream)
                    for _ in range(args.steps):
                        mpm.count_ids(sc.out[:M], d, out=cbuf)
                    ev[1].record(stream)
                    torch.cuda.synchronize()
                    count_ms = ev[0].elapsed_time(ev[1]) / args.steps
                    counts = cbuf.to(torch.int64) & 0xFFFFFFFF
                    if int(counts.sum()) != M:
                        raise SystemExit(f"per-pattern counts do not sum to the list length at d={d} m={m}")
                    parity = None
                    if gold is not None:
                        import hashlib
                        g = next(r for r in gold["sets"] if r["d"] == d and r["m"] == m)
                        dig = f"{listdigest().digest_torch(sc.out[:M]):016x}"
                        csha = hashlib.sha256(cbuf.cpu().numpy().view(np.uint32).astype("<u4")
                                              .tobytes()).hexdigest()
                        parity = bool(M == g["total"] and dig == g["digest"] and
                                      csha == g["counts_sha256"])
                        if not parity:
                            raise SystemExit(f"d={d} m={m} {algo} {vname}: list differs from the "
                                             f"oracle's ({M} vs {g['total']} pairs)")
                    by_variant[vname] = {"gbps": round(n / (kms * 1e-3) / 1e9, 2),
                                         "kernel_ms": round(kms, 4), "equals_oracle": parity}
                    if best is None or kms < best[1]:
                        if best is not None:
                            del best[2]
                        best = [vname, kms, sc, count_ms, counts, parity]
                    else:
                        del sc
                vname, kms, sc, count_ms, counts, parity = best
                lists[algo] = sc.out[:M]
                alg_bytes = n + 8 * M + info["table_bytes"]
                rows.append({
                    "d": d, "m": m, "algo": algo, "gbps": round(n / (kms * 1e-3) / 1e9, 2),
                    "kernel_ms": round(kms, 4), "variant": vname, "by_variant": by_variant,
                    "matches": M,
                    "roofline_frac": round(alg_bytes / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "table_bytes": info["table_bytes"],
                    "states": info["n_states"] if algo == "ac" else None,
                    "wm_block": info["wm_block"] if algo == "wm" else None,
                    "placement": "lds" if info["table_bytes"] + 1536 <= 160 * 1024 else "hot",
                    "patterns_hit": int((counts > 0).sum()), "max_count": int(counts.max()),
                    "count_ms": round(count_ms, 4),
                    "equals_oracle": parity,
                    "build_s": round(build_s, 3)})
                log(f"[bench] d={d} m={m} {algo}: {rows[-1]['gbps']} GB/s ({vname}; "
                    f"{ {k: x['gbps'] for k, x in by_variant.items()} }), {M} matches")
                del sc, ix, best
            if not torch.equal(lists["ac"], lists["wm"]):
                raise SystemExit(f"AC and WM disagree at d={d} m={m}")
            del lists
            torch.cuda.empty_cache()
    line = {"metric": METRIC, "workload": "sweep",
            "config": {"workload": "1 GiB EST-shaped DNA text (seed 4); d in {1000, 10000, 100000} x "
                                   "m in {8, 16, 32}, 10% planted (seeds 10-18)", "n_bytes": n,
                       "variants": dict(DEFAULT_VARIANTS, dense=DENSE_VARIANT)},
            "steps": args.steps, "warmup": args.warmup, "dtype": "u8", "data": "synthetic",
            "rows": rows}
    print(json.dumps(line), flush=True)


def run_stream(args):
    """Host-resident text: the 256 MiB EST-shaped text in pinned host memory,
    scanned chunk by chunk through two device staging buffers with the copies
    overlapping the scans. Text GB/s here include the host-to-device copies;
    the plain copy rate of the same text is reported beside them. One JSON
    line."""
    import torch
    import paper_1407_2889_amd as mpm
    text, ps, desc = workload("est256")
    n = len(text)
    host = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    host.numpy()[:] = text
    dev = torch.empty(n, dtype=torch.uint8, device="cuda")
    for _ in range(2):
        dev.copy_(host, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dev.copy_(host, non_blocking=True)
    torch.cuda.synchronize()
    h2d = n * args.steps / (time.perf_counter() - t0) / 1e9
    rows = []
    for algo in ("ac", "wm"):
        ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(ps.patterns, upload=True)
        v = mpm.variant(**DEFAULT_VARIANTS[algo])
        want = mpm.scan(ix, dev, var=v)
        for chunk_mib in (16, 64):
            chunk = chunk_mib << 20
            got = mpm.scan_host(ix, host, chunk=chunk, var=v)
            if not torch.equal(got, want):
                raise SystemExit(f"host-streamed {algo} list differs from the device-resident scan")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                mpm.scan_host(ix, host, chunk=chunk, var=v)
            wall = (time.perf_counter() - t0) / args.steps
            rows.append({"algo": algo, "chunk_mib": chunk_mib, "ms": round(wall * 1e3, 3),
                         "gbps_with_copies": round(n / wall / 1e9, 2)})
            log(f"[bench] stream {algo} chunk {chunk_mib} MiB: {rows[-1]['gbps_with_copies']} GB/s")
        del ix
    line = {"metric": "text GB/s scanned from host memory (copies included)", "workload": "stream",
            "config": {"workload": desc + "; text in pinned host memory", "n_bytes": n,
                       "variants": DEFAULT_VARIANTS},
            "steps": args.steps, "dtype": "u8", "data": "synthetic",
            "h2d_copy_gbps": round(h2d, 2), "rows": rows}
    print(json.dumps(line), flush=True)


def run_ablation(args):
    """The paper's kernel ladder (Section 4.2.2: unoptimised, texture-cached
    tables, coalesced reads into shared memory, 16-byte reads, coalesced
    writes) rebuilt for gfx950 on the 256 MiB EST text (d=1000, m=16): text
    read a byte at a time from global memory, with the tables in global
    memory then in LDS; the chunk's text staged in LDS by coalesced 16-byte
    loads; 16-byte line streaming through registers (byte-class table, then
    register byte classes); the benchmark's launch shape; then the other
    table placements and the goto function with supply links. Writes: the
    same scan counting only, writing the ordered list lane by lane, and
    writing it in dense mode, on a dense set (d=100k, m=8). Kernel time from
    HIP events; every row's list is checked against its group's first. One
    JSON line."""
    import torch
    import paper_1407_2889_amd as mpm
    import synth
    text, ps, desc = workload("est256")
    n = len(text)
    dev = torch.from_numpy(text).cuda()
    stream = torch.cuda.current_stream()
    ix = mpm.build_ac(ps.patterns, upload=True, goto=True)
    L, W = DEFAULT_VARIANTS["ac"]["lane_bytes"], DEFAULT_VARIANTS["ac"]["block_threads"]
    # Two launch shapes, both 1024 threads per workgroup: the benchmark's
    # 1 KiB lanes (a 1 MiB chunk, too large to stage in LDS), and 16-byte
    # lanes (a 16 KiB chunk, the largest whose text fits in LDS beside the
    # 142 KB table) for the staged-text rung.
    TB, TL, NS = mpm.VARIANT_TEXT_BYTES, mpm.VARIANT_TEXT_LDS, mpm.VARIANT_NO_SWAR
    rows_spec = [
        ("U: bytes one at a time from global memory, tables in global memory", L, W,
         mpm.PLACE_GLOBAL, TB),
        ("TC: tables in LDS (the paper's texture-cached tables), bytes from global memory", L, W,
         mpm.PLACE_LDS, TB),
        ("R16: 16-byte loads into registers, whole lines, byte-class table in LDS", L, W,
         mpm.PLACE_LDS, NS),
        ("R16 + register byte classes (the benchmark kernel)", L, W, mpm.PLACE_LDS, 0),
        ("16-byte lanes, U: bytes from global memory, tables in global memory", 16, W,
         mpm.PLACE_GLOBAL, TB),
        ("16-byte lanes, TC: tables in LDS, bytes from global memory", 16, W, mpm.PLACE_LDS, TB),
        ("16-byte lanes, CR: chunk text staged in LDS by coalesced 16-byte loads", 16, W,
         mpm.PLACE_LDS, TL),
        ("16-byte lanes, R16: 16-byte loads into registers, byte-class table", 16, W,
         mpm.PLACE_LDS, NS),
        ("16-byte lanes, R16 + register byte classes", 16, W, mpm.PLACE_LDS, 0),
        ("benchmark launch shape, hot rows in LDS", L, W, mpm.PLACE_HOT, 0),
        ("benchmark launch shape, tables in global memory", L, W, mpm.PLACE_GLOBAL, 0),
        ("goto + supply links (not flattened), tables in global memory", L, W, mpm.PLACE_GLOBAL,
         mpm.VARIANT_SUPPLY)]
    rows, ref = [], None
    for name, l, w, pl, fl in rows_spec:
        v = mpm.variant(lane_bytes=l, block_threads=w, placement=pl, flags=fl)
        sc = mpm.Scanner(ix, n, capacity=1 << 20, var=v)
        got = sc.scan(dev)
        if ref is None:
            ref = got.clone()
        elif not torch.equal(got, ref):
            raise SystemExit(f"ablation row '{name}' reports a different list")
        kms = time_scans(sc, dev, args.steps, args.warmup, stream)
        rows.append({"kernel": name, "lane_bytes": l, "block_threads": w, "kernel_ms": round(kms, 4),
                     "gbps": round(n / (kms * 1e-3) / 1e9, 2)})
        log(f"[bench] ablation {name}: {rows[-1]['gbps']} GB/s")
        del sc
    del ix
    # writes: a dense set on the same text
    dset = synth.workload_sweep_set(text, 100_000, 8)
    dix = mpm.build_ac(dset.patterns, upload=True)
    wrows, wref, M = [], None, None
    for name, cap_full, fl in (("CW: count only (capacity 0), per-lane counts", False, 0),
                               ("ordered list, lane by lane", True, 0),
                               ("ordered list, dense mode (waves write consecutive slots)", True,
                                mpm.VARIANT_DENSE)):
        v = mpm.variant(lane_bytes=L if not fl else 0, block_threads=W, flags=fl)
        if M is None:
            c0 = mpm.Scanner(dix, n, capacity=0, var=v)
            c0.scan_async(dev)
            torch.cuda.synchronize()
            M = int(c0.total.item())
            del c0
        sc = mpm.Scanner(dix, n, capacity=M if cap_full else 0, var=v)
        sc.scan_async(dev)
        torch.cuda.synchronize()
        assert int(sc.total.item()) == M
        if cap_full:
            got = sc.out[:M]
            if wref is None:
                wref = got.clone()
            elif not torch.equal(got, wref):
                raise SystemExit(f"write row '{name}' reports a different list")
        kms = time_scans(sc, dev, args.steps, args.warmup, stream)
        wrows.append({"kernel": name, "kernel_ms": round(kms, 4),
                      "gbps": round(n / (kms * 1e-3) / 1e9, 2),
                      "list_bytes": 8 * M if cap_full else 0})
        log(f"[bench] ablation {name}: {wrows[-1]['gbps']} GB/s")
        del sc
    line = {"metric": "text GB/s scanned (AC kernel designs)", "workload": "ablation",
            "config": {"workload": desc, "n_bytes": n, "matches": int(ref.shape[0]),
                       "states": mpm.build_ac(ps.patterns).info()["n_states"],
                       "write_set": "d=100000, m=8, 10% planted (the sweep's set) on the same text",
                       "write_matches": M},
            "steps": args.steps, "warmup": args.warmup, "dtype": "u8", "data": "synthetic",
            "rows": rows, "write_rows": wrows}
    print(json.dumps(line), flush=True)


MIXED_DESC = ("EST-shaped DNA text 256 MiB (seed 51), d=1000 patterns of lengths 8-32: 500 text "
              "windows, 200 of their prefixes, 100 suffixes, 50 duplicates, 150 random (seed 52)")


def run_mixed(args):
    """Pattern sets of different lengths: the reversed-automaton AC scan and
    the shortest-length WM scan of the 256 MiB EST text, each with its
    default launch variant, the whole list written; text GB/s, the HBM
    roofline fraction of the algorithmic bytes (text read once, list written
    once), and the list's count and digest against the oracle's. One JSON
    line."""
    import torch
    import paper_1407_2889_amd as mpm
    import synth
    import oracle
    text = synth.est_text(256 << 20, seed=51)
    P = synth.mixed_pattern_set(text, 1000, 8, 32, 500, seed=52, n_prefix=200, n_suffix=100,
                                n_dup=50)
    n = len(text)
    dev = torch.from_numpy(text).cuda()
    stream = torch.cuda.current_stream()
    log("[bench] mixed lengths: oracle list")
    want = oracle.parallel_scan(oracle.AC(P), text, workers=HOST_SHARE_THREADS)
    M = len(want[0])
    dg = listdigest()
    want_digest = dg.digest_np(want[0], want[1])
    rows = []
    for algo in ("ac", "wm"):
        ix = (mpm.build_ac_var if algo == "ac" else mpm.build_wm_var)(P, upload=True)
        inf = ix.info()
        for pl in (mpm.PLACE_AUTO, mpm.PLACE_HOT, mpm.PLACE_GLOBAL):
            v = dict(DEFAULT_VARIANTS[algo], placement=pl)
            sc = mpm.Scanner(ix, n, capacity=M + 64, var=mpm.variant(**v))
            got = sc.scan(dev)
            equal = int(got.shape[0]) == M and dg.digest_torch(got) == want_digest
            kms = time_scans(sc, dev, args.steps, args.warmup, stream)
            alg = n + 8 * M
            rows.append({"algo": algo, "variant": v, "kernel_ms": round(kms, 4),
                         "gbps": round(n / (kms * 1e-3) / 1e9, 2),
                         "roofline_frac": round(alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "matches": M, "equals_oracle": bool(equal),
                         "table_bytes": int(inf["table_bytes"]), "m_min": inf["m"],
                         "m_max": inf["m_max"]})
            log(f"[bench] mixed {algo} placement {pl}: {rows[-1]['gbps']} GB/s, equals oracle {equal}")
            del sc
        del ix
    if not all(r["equals_oracle"] for r in rows):
        raise SystemExit("mixed-length lists differ from the oracle's")
    line = {"metric": "text GB/s scanned (pattern sets of different lengths)", "workload": "mixed",
            "config": {"workload": MIXED_DESC, "n_bytes": n}, "steps": args.steps,
            "warmup": args.warmup, "dtype": "u8", "data": "synthetic", "rows": rows}
    print(json.dumps(line), flush=True)


def run_scaling(args):
    """Kernel time against the number of busy CUs: the AC and WM scans of the
    first k MiB of the 256 MiB EST text in the benchmark's launch
    configuration (one 1 MiB chunk per workgroup, one workgroup per CU), k
    from 1 to 256, and the same text read in the scans' lane layout without
    the walk (1 KiB lanes, and 128-byte lanes for comparison). One JSON
    line."""
    import torch
    import paper_1407_2889_amd as mpm
    text, ps, desc = workload("est256")
    dev = torch.from_numpy(text).cuda()
    stream = torch.cuda.current_stream()
    rows = []
    for algo in ("ac", "wm"):
        ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(ps.patterns, upload=True)
        v = mpm.variant(**DEFAULT_VARIANTS[algo])
        for k in (1, 8, 64, 128, 192, 224, 240, 256):
            n = min(len(text), k << 20)
            sc = mpm.Scanner(ix, n, capacity=1 << 16, var=v)
            kms = time_scans(sc, dev[:n], args.steps, args.warmup, stream)
            rows.append({"algo": algo, "chunks": k, "kernel_us": round(kms * 1e3, 2),
                         "gbps": round(n / (kms * 1e-3) / 1e9, 2)})
            log(f"[bench] scaling {algo} {k} chunks: {rows[-1]['kernel_us']} us")
            del sc
        del ix
    # the same lane layout read without the table walk: the memory system's
    # rate for the scans' access pattern
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    for lane in (1024, 128):
        for k in (1, 8, 64, 128, 192, 256):
            n = min(len(text), k << 20)
            buf = dev[:n]
            for _ in range(args.warmup):
                mpm.read_probe_lanes(buf, lane, sink)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)]
            torch.cuda.synchronize()
            for a, b in ev:
                a.record(stream)
                mpm.read_probe_lanes(buf, lane, sink)
                b.record(stream)
            torch.cuda.synchronize()
            kms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
            rows.append({"algo": f"read_lanes_{lane}", "chunks": n // (1024 * lane),
                         "mib": n >> 20, "kernel_us": round(kms * 1e3, 2),
                         "gbps": round(n / (kms * 1e-3) / 1e9, 2)})
            log(f"[bench] scaling read lanes {lane} B, {n >> 20} MiB: {rows[-1]['kernel_us']} us")
    line = {"metric": "kernel time against busy CUs", "workload": "scaling",
            "config": {"workload": desc, "variants": DEFAULT_VARIANTS}, "steps": args.steps,
            "warmup": args.warmup, "dtype": "u8", "data": "synthetic", "rows": rows}
    print(json.dumps(line), flush=True)


BATCH_DESC = ("4,096 EST-shaped texts, log-uniform 1 KiB-4 MiB (seed 20), 64 pattern sets d "
              "log-uniform 100-50k, m in {8,12,16,24,32}, 10% planted (seed 21), pairing seed 22")


def batch_selection(args) -> dict:
    """Batched workload with variant selection: a timing database of seeded
    training requests (every request timed on all 24 variants inside batched
    launches), the selector trained on it with the library's kernels, then the
    4,096-text batch run as one replayed graph per policy (exhaustive
    autotune, learned with fallback, fixed default), every policy's lists
    checked against the oracle's. Returns the result keys."""
    import torch
    import synth
    from paper_1407_2889_amd import learn, selection, tune
    t_start = time.perf_counter()
    log(f"[bench] timing database: {args.train_requests} requests")
    stream, sets, reqs = synth.selector_training_requests(args.train_requests, 48, seed=1000,
                                                          stream_bytes=256 << 20)
    sd = torch.from_numpy(stream).cuda()
    sidx = [tune.PatternSetIndexes.build(p.patterns) for p in sets]
    tuner = tune.Tuner()
    t0 = time.perf_counter()
    feats, ms, cfac = selection.build_db(tuner, sidx, sd, reqs, log=log)
    t_db = time.perf_counter() - t0
    del sd, sidx
    t0 = time.perf_counter()
    sel = learn.Selector.fit(feats, ms, chunk_factor=cfac)
    t_fit = time.perf_counter() - t0
    kdef = selection.best_uniform_variant(ms)
    log(f"[bench] db {t_db:.1f}s, fit {t_fit:.1f}s, default variant {tune.VARIANTS[kdef]}")
    log(f"[bench] batch: {args.batch_texts} texts")
    b = synth.workload_batch(n_texts=args.batch_texts, n_sets=64, seed=20)
    gold = golden("batch") if args.batch_texts == 4096 else None
    parity = {}

    def check(name, bs):
        """Every text's list of this policy's last replay against the
        oracle's (pair count and order-sensitive digest)."""
        if gold is None:
            return
        tot = bs.totals_host()
        ok = bool(np.array_equal(tot, np.array(gold["counts"], np.int64)))
        if ok:
            dg = listdigest().segment_digests_torch(
                bs.out, torch.from_numpy(bs.out_offs[:-1].astype(np.int64)).cuda(),
                torch.from_numpy(tot.astype(np.int64)).cuda())
            ok = dg == [int(x, 16) for x in gold["digests"]]
        parity[name] = ok
        log(f"[bench] batch policy {name}: lists {'equal' if ok else 'DIFFER FROM'} the oracle's")

    res = selection.evaluate(b, tuner, sel, kdef, log=log, check=check)
    res.pop("_state")
    if gold is not None and not all(parity.values()):
        raise SystemExit(f"batched lists differ from the oracle's: {parity}")
    return {
        "learned_gbps": round(res["learned_gbps"], 2),
        "exhaustive_gbps": round(res["exhaustive_gbps"], 2),
        "default_gbps": round(res["default_gbps"], 2),
        "regret": round(res["regret"], 4), "fallback_rate": round(res["fallback_rate"], 4),
        "gain_over_default": round(res["gain_over_default"], 4),
        "totals_agree": res["totals_agree"], "matches": res["matches"],
        "equals_oracle": parity or None,
        "text_bytes": res["text_bytes"],
        "launches": {k: res[f"{k}_launches"] for k in ("exhaustive", "learned", "default")},
        "pick_agreement": round(res["pick_agreement"], 4),
        "chunk_safety": round(res["chunk_safety"], 3),
        "time_regret_tuned": {k: round(v, 4) for k, v in res["time_regret_tuned"].items()},
        "selection_overhead_s": {k: round(v, 4) for k, v in res["selection_overhead_s"].items()},
        "train_requests": args.train_requests,
        "timing_db_s": round(t_db, 1), "fit_s": round(t_fit, 1),
        "default_variant": res["default_variant"],
        "wall_s": round(time.perf_counter() - t_start, 1)}


def run_batched(args):
    """--workload batch: the batched selection result as its own JSON line."""
    res = batch_selection(args)
    line = {"metric": METRIC, "workload": "batch", "value": res["learned_gbps"], "unit": "GB/s",
            "higher_is_better": True, "dtype": "u8", "data": "synthetic",
            "config": {"workload": BATCH_DESC if args.batch_texts == 4096 else
                       f"{args.batch_texts} texts of the batched workload's distributions"}}
    line.update(res)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="est256")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-workload selection keys of the default line")
    ap.add_argument("--cpu-sample-mib", type=int, default=256)
    ap.add_argument("--ac", default=None, help="AC variant as L,W,placement[,flags]")
    ap.add_argument("--wm", default=None, help="WM variant as L,W,placement[,flags]")
    ap.add_argument("--train-requests", type=int, default=5000, help="batch: timing database size")
    ap.add_argument("--batch-texts", type=int, default=4096, help="batch: texts in the batch")
    ap.add_argument("--sweep-sets", default=None,
                    help="sweep: only these sets, as d:m pairs separated by commas")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the scan shards by contiguous text ranges across GPUs, but this benchmark "
              "measures one GPU", file=sys.stderr)
        sys.exit(2)
    if args.workload == "sweep":
        return run_sweep(args)
    if args.workload == "batch":
        return run_batched(args)
    if args.workload == "stream":
        return run_stream(args)
    if args.workload == "ablation":
        return run_ablation(args)
    if args.workload == "scaling":
        return run_scaling(args)
    if args.workload == "mixed":
        return run_mixed(args)

    import torch
    import paper_1407_2889_amd as mpm

    variants = dict(DEFAULT_VARIANTS)
    for k in ("ac", "wm"):
        s = getattr(args, k)
        if s:
            f = [int(x) for x in s.split(",")]
            variants[k] = dict(lane_bytes=f[0], block_threads=f[1], placement=f[2],
                               **({"flags": f[3]} if len(f) > 3 else {}))

    log(f"[bench] generating workload {args.workload}")
    text, ps, desc = workload(args.workload)
    n = len(text)
    dev_text = torch.from_numpy(text).cuda()
    P = ps.patterns
    log("[bench] building indexes")
    t0 = time.perf_counter()
    ix = {"ac": mpm.build_ac(P, upload=True), "wm": mpm.build_wm(P, upload=True)}
    build_s = time.perf_counter() - t0
    scanners = {}
    for k in ("ac", "wm"):
        v = mpm.variant(**variants[k])
        scanners[k] = mpm.Scanner(ix[k], n, capacity=max(1 << 20, n // 64), var=v)

    # correctness guard: both algorithms report the same list
    res = {k: mpm.pairs_numpy(scanners[k].scan(dev_text)) for k in ("ac", "wm")}
    M = len(res["ac"][0])
    if not (np.array_equal(res["ac"][0], res["wm"][0]) and np.array_equal(res["ac"][1], res["wm"][1])):
        raise SystemExit("AC and WM disagree")
    log(f"[bench] matches={M}")

    stream = torch.cuda.current_stream()
    # Streaming-read ceiling of this device: a coalesced read of a 1 GiB buffer.
    probe = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    probe.fill_(1)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    for _ in range(2):
        mpm.read_probe(probe, sink)
    pe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    for a, b in pe:
        a.record(stream)
        mpm.read_probe(probe, sink)
        b.record(stream)
    torch.cuda.synchronize()
    probe_ms = float(np.median([a.elapsed_time(b) for a, b in pe]))
    read_ceiling = probe.numel() / (probe_ms * 1e-3) / 1e9
    del probe

    for _ in range(args.warmup):
        for k in ("ac", "wm"):
            scanners[k].scan_async(dev_text)
    torch.cuda.synchronize()

    ev = {k: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)] for k in ("ac", "wm")}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        for k in ("ac", "wm"):
            ev[k][s][0].record(stream)
            scanners[k].scan_async(dev_text)
            ev[k][s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = {k: float(np.mean([a.elapsed_time(b) for a, b in ev[k]])) for k in ("ac", "wm")}
    for k in ("ac", "wm"):
        assert int(scanners[k].total.item()) == M
    ms_step = wall / args.steps * 1e3
    gbs = {k: n / (kms[k] * 1e-3) / 1e9 for k in ("ac", "wm")}
    dom = max(kms, key=kms.get)
    info = ix[dom].info()
    alg_bytes = n + 8 * M + info["table_bytes"]
    achieved = alg_bytes / (kms[dom] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": round(2 * n / (wall / args.steps) / 1e9, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": desc, "n_bytes": n, "d": int(P.shape[0]), "m": int(P.shape[1]),
                   "matches": M, "variants": variants},
        "ac_gbps": round(gbs["ac"], 2),
        "wm_gbps": round(gbs["wm"], 2),
        "ac_kernel_ms": round(kms["ac"], 4),
        "wm_kernel_ms": round(kms["wm"], 4),
        "ac_roofline_frac": round((n + 8 * M + ix["ac"].info()["table_bytes"]) / (kms["ac"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "wm_roofline_frac": round((n + 8 * M + ix["wm"].info()["table_bytes"]) / (kms["wm"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "index_build_s": round(build_s, 3),
        "hbm_read_ceiling_gbs": round(read_ceiling, 1),
        "frac_of_read_ceiling": {k: round(gbs[k] / read_ceiling, 4) for k in ("ac", "wm")},
        "roofline": {"bound": "hbm", "kernel": f"scan_kernel ({dom.upper()})",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(args.workload, dom),
                     "alg_bytes_per_launch": alg_bytes},
    }
    lds = recorded_lds(args.workload, dom)
    if lds is not None and ix[dom].info()["table_bytes"] + 1536 <= 160 * 1024:
        # The walk makes one dependent table lookup per text byte from LDS:
        # its ceiling is the rate at which the CUs' LDS serves the kernel's
        # wave-wide reads at their measured cost (bank conflicts included).
        ceiling = CUS * CLOCK_GHZ * 64 / (lds["lds_cycles_per_instr"] * lds["lds_instr_per_64_bytes"])
        hbm = line["roofline"]
        line["roofline"] = {
            "bound": "lds", "kernel": hbm["kernel"], "achieved": round(gbs[dom], 2),
            "peak": round(ceiling, 1), "unit": "GB/s", "frac": round(gbs[dom] / ceiling, 4),
            "traffic": hbm["traffic"], "alg_bytes_per_launch": alg_bytes,
            "peak_basis": (f"text bytes per second at one LDS table lookup per byte: {CUS} CUs x "
                           f"{CLOCK_GHZ} GHz x 64 lanes per wave-wide LDS read / "
                           f"({lds['lds_cycles_per_instr']} LDS-active cycles per read x "
                           f"{lds['lds_instr_per_64_bytes']} reads per 64 text bytes), both "
                           "from rocprofv3 SQ_LDS_IDX_ACTIVE and SQ_INSTS_LDS"),
            "hbm": {"achieved": hbm["achieved"], "peak": HBM_PEAK_GBS, "frac": hbm["frac"]}}
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(text, P, min(n, args.cpu_sample_mib << 20))
    if not args.no_batch:
        # the metric's second half: learned against exhaustive-tuned selection
        # on the batched workload (untimed by the step loop above)
        del scanners, ix, dev_text
        torch.cuda.empty_cache()
        bres = batch_selection(args)
        line["batch"] = dict(bres, workload=BATCH_DESC)
        for k in ("learned_gbps", "exhaustive_gbps", "default_gbps", "regret", "fallback_rate"):
            line[f"batch_{k}"] = bres[k]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
