"""GPU parity at the pattern-set sweep's full size: 1 GiB EST-shaped text,
d in {1k, 10k, 100k} x m in {8, 16, 32} (10% planted), in the benchmark's
launch configuration. Each case checks, at full size:

  - the whole list against the oracle's, streamed: the pair count, an
    order-sensitive 64-bit digest of the whole sorted list, the per-pattern
    occurrence counts (SHA-256 of the vector, counted on the device from the
    list) and the first and last pairs, all written by
    tests/golden/make_digests.py from the CPU oracle alone;
  - the oracle's exact list on sampled ranges of starting positions (the
    first and last ranges of the text included) against the GPU list
    restricted to the same ranges, element by element;
  - Aho-Corasick and Wu-Manber lists equal to each other, element by element;
  - every planted pattern reported at its planted start.
"""

import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import listdigest  # noqa: E402

N_RANGES = 24
RANGE = 4096


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mpm():
    import paper_1407_2889_amd as m
    assert torch.cuda.is_available()
    return m


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(GOLDEN, "sweep_digests.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def sweep_text(golden):
    say("[sweep] generating 1 GiB text")
    text = synth.workload_sweep_text()
    assert hashlib.sha256(text.tobytes()).hexdigest() == golden["text_sha256"], \
        "the generator no longer reproduces the text the expected values were computed on"
    return text, torch.from_numpy(text).cuda()


def ranges(n: int, m: int, seed: int):
    ns = n - m + 1
    rng = np.random.default_rng(seed)
    los = [0, ns - RANGE] + sorted(rng.integers(0, ns - RANGE, N_RANGES - 2).tolist())
    return [(int(lo), int(lo) + RANGE) for lo in los]


def device_keys(pairs):
    """int64 key pos * 2^32 + id of an int32 [M, 2] (pos, id) tensor."""
    p = pairs[:, 0].to(torch.int64) & 0xFFFFFFFF
    i = pairs[:, 1].to(torch.int64) & 0xFFFFFFFF
    return (p << 32) | i


@pytest.mark.parametrize("d", synth.SWEEP_D)
@pytest.mark.parametrize("m", synth.SWEEP_M)
def test_sweep_full_size(mpm, sweep_text, golden, d, m):
    import bench
    text, dev = sweep_text
    ps = synth.workload_sweep_set(text, d, m)
    P = ps.patterns
    g = next(r for r in golden["sets"] if r["d"] == d and r["m"] == m)
    assert hashlib.sha256(P.tobytes()).hexdigest() == g["patterns_sha256"]
    lists = {}
    for algo in ("ac", "wm"):
        ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(P, upload=True)
        v = mpm.variant(**bench.DEFAULT_VARIANTS[algo])
        say(f"[sweep d={d} m={m}] {algo} {ix.info()['table_bytes']} table bytes, variant {v}")
        lists[algo] = mpm.scan(ix, dev, var=v)
        del ix
    a, w = lists["ac"], lists["wm"]
    say(f"[sweep d={d} m={m}] {a.shape[0]} pairs (oracle {g['total']})")
    # the whole list against the oracle's (streamed summary)
    assert a.shape[0] == g["total"], f"AC {a.shape[0]} pairs vs oracle {g['total']}"
    dig = listdigest.digest_torch(a)
    assert f"{dig:016x}" == g["digest"], "AC list digest differs from the oracle's"
    head = a[: len(g["head"])].cpu().numpy().view(np.uint32).tolist()
    tail = a[a.shape[0] - len(g["tail"]):].cpu().numpy().view(np.uint32).tolist()
    assert head == g["head"] and tail == g["tail"]
    counts = mpm.count_ids(a, d).cpu().numpy().view(np.uint32)
    assert hashlib.sha256(counts.astype("<u4").tobytes()).hexdigest() == g["counts_sha256"], \
        "per-pattern counts differ from the oracle's"
    assert int((counts > 0).sum()) == g["patterns_hit"] and int(counts.max()) == g["max_count"]
    assert {str(i): int(counts[int(i)]) for i in g["spot_counts"]} == g["spot_counts"]
    # Wu-Manber: the same list
    assert a.shape == w.shape, f"AC {a.shape[0]} vs WM {w.shape[0]} pairs"
    assert torch.equal(a, w), "AC and WM lists differ"
    # dense output, both algorithms: the same list again
    for algo in ("ac", "wm"):
        ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(P, upload=True)
        say(f"[sweep d={d} m={m}] {algo} dense output")
        dn = mpm.scan(ix, dev, capacity=g["total"], var=mpm.variant(**bench.DENSE_VARIANT))
        assert torch.equal(dn, a), f"{algo} dense output differs"
        del ix, dn
    key = device_keys(a)
    # sampled exact comparison with the oracle
    orc = oracle.Win(P)
    pos = a[:, 0].to(torch.int64) & 0xFFFFFFFF
    for lo, hi in ranges(len(text), m, seed=1000 * d + m):
        want = orc.scan(text, lo, hi)
        b0 = int(torch.searchsorted(pos, lo))
        b1 = int(torch.searchsorted(pos, hi))
        got = a[b0:b1].cpu().numpy().view(np.uint32)
        assert len(got) == len(want[0]), f"range [{lo}, {hi}): {len(got)} vs oracle {len(want[0])}"
        assert np.array_equal(got[:, 0], want[0]) and np.array_equal(got[:, 1], want[1]), \
            f"range [{lo}, {hi}) differs"
    # planted occurrences
    planted = torch.from_numpy(
        (ps.planted_starts.astype(np.int64) << 32) | np.arange(len(ps.planted_starts), dtype=np.int64)
    ).cuda()
    idx = torch.searchsorted(key, planted)
    ok = (idx < key.numel()) & (key[idx.clamp(max=key.numel() - 1)] == planted)
    assert bool(ok.all()), "a planted pattern is missing at its planted start"
    del lists, a, w, key, pos
    torch.cuda.empty_cache()
