"""GPU parity for pattern sets of different lengths: the HIP scans through the
C-ABI against the CPU oracle (the Definition with a length per pattern),
element by element. Aho-Corasick walks the automaton of the reversed strings
backwards; Wu-Manber windows on the shortest length."""

import ctypes as C
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mpm():
    import paper_1407_2889_amd as m
    assert torch.cuda.is_available()
    return m


def to_dev(text: np.ndarray, misalign: int = 0):
    buf = torch.zeros(len(text) + misalign + 64, dtype=torch.uint8, device="cuda")
    if len(text):
        buf[misalign:misalign + len(text)] = torch.from_numpy(np.array(text, np.uint8)).cuda()
    return buf[misalign:misalign + len(text)]


def assert_same(got, want, what=""):
    gp, gi = got
    wp, wi = want
    assert len(gp) == len(wp), f"{what}: {len(gp)} pairs vs oracle {len(wp)}"
    if len(wp):
        bad = np.nonzero((gp != wp) | (gi != wi))[0]
        assert bad.size == 0, (f"{what}: first mismatch at {bad[0]}: got {(gp[bad[0]], gi[bad[0]])} "
                               f"want {(wp[bad[0]], wi[bad[0]])}")


def build(mpm, algo, P):
    return (mpm.build_ac_var if algo == "ac" else mpm.build_wm_var)(P, upload=True)


VARIANTS = [dict(lane_bytes=16, block_threads=256), dict(lane_bytes=64, block_threads=1024),
            dict(lane_bytes=256, block_threads=512, placement=2),
            dict(lane_bytes=32, block_threads=256, placement=1),
            dict(lane_bytes=4096, block_threads=256)]


def variants_for(mpm, ix, algo):
    vs = list(VARIANTS) + [dict(lane_bytes=64, block_threads=512, placement=3),
                           dict(lane_bytes=1024, block_threads=1024, placement=3)]
    out = []
    for v in vs:
        var = mpm.variant(**v)
        try:
            mpm.workspace_bytes(ix, 1 << 20, var)
        except mpm.MpmError as e:  # LDS placement of a table that does not fit
            assert e.status == mpm.MPM_EUNSUPPORTED and v.get("placement") == 1
            continue
        out.append((v, var))
    return out


def cases():
    rng = np.random.default_rng(21)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    out = []
    hand = json.load(open(os.path.join(HERE, "golden", "mixed_hand_example.json")))
    for k, c in enumerate(hand["cases"]):
        out.append((f"hand{k}", np.frombuffer(c["text"].encode(), np.uint8),
                    [p.encode() for p in c["patterns"]]))
    t = acgt[rng.integers(0, 4, 100_003)]
    P = [t[s:s + int(rng.integers(3, 12))].tobytes() for s in rng.integers(0, len(t) - 12, 40)]
    P += [p[:max(1, len(p) - 2)] for p in P[:10]] + [p[2:] for p in P[10:20] if len(p) > 3]
    P += P[:5]  # duplicates
    out.append(("prefix-suffix-dup", t, P))
    out.append(("all-A nested", np.full(70_001, ord("A"), np.uint8),
                [b"A" * k for k in (1, 2, 3, 5, 8, 13)] + [b"AAB", b"A"]))
    t = synth.est_text(300_000, seed=5)
    out.append(("est lengths 8-32", t,
                synth.mixed_pattern_set(t, 600, 8, 32, 300, seed=6, n_prefix=120, n_suffix=60,
                                        n_dup=30)))
    t = synth.est_text(150_000, seed=7)
    out.append(("est lengths 4-64 dense", t,
                synth.mixed_pattern_set(t, 3000, 4, 64, 1500, seed=8, n_prefix=600, n_dup=100)))
    b = rng.integers(0, 256, 50_000).astype(np.uint8)
    P = [b[s:s + int(rng.integers(2, 9))].tobytes() for s in rng.integers(0, 50_000 - 9, 60)]
    P += [bytes(rng.permutation(256).astype(np.uint8)[:k]) for k in (3, 5, 7)]
    out.append(("all byte values", b, P))
    t = acgt[rng.integers(0, 4, 20_000)]
    out.append(("one long pattern", t, [b"AC", t[5000:5300].tobytes(), t[5000:5002].tobytes()]))
    out.append(("text shorter than the longest", acgt[rng.integers(0, 4, 10)],
                [b"A", b"C", acgt[rng.integers(0, 4, 40)].tobytes()]))
    out.append(("text shorter than the shortest", acgt[rng.integers(0, 4, 2)], [b"ACG", b"ACGTT"]))
    out.append(("empty text", np.zeros(0, np.uint8), [b"AC", b"A"]))
    return out


@pytest.mark.parametrize("case", cases(), ids=lambda c: c[0])
@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_mixed_cases(mpm, case, algo):
    name, T, P = case
    want = oracle.bf(T, P) if len(T) <= 20_000 else oracle.parallel_scan(oracle.AC(P), T)
    ix = build(mpm, algo, P)
    info = ix.info()
    assert info["m"] == min(len(p) for p in P) and info["m_max"] == max(len(p) for p in P)
    for v, var in variants_for(mpm, ix, algo):
        for mis in (0, 3):
            say(f"[mixed {name} n={len(T)} d={len(P)}] {algo} {v} misalign {mis}")
            out = mpm.scan(ix, to_dev(T, mis), var=var)
            assert_same(mpm.pairs_numpy(out), want, f"{name} {algo} {v}")


@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_mixed_capacity_prefix_and_count(mpm, algo):
    t = synth.est_text(400_000, seed=31)
    P = synth.mixed_pattern_set(t, 800, 6, 24, 500, seed=32, n_prefix=200, n_dup=40)
    want = oracle.parallel_scan(oracle.AC(P), t)
    ix = build(mpm, algo, P)
    td = to_dev(t)
    for cap in (len(want[0]) // 3, 1, 0):
        say(f"[mixed capacity] {algo} cap={cap}")
        sc = mpm.Scanner(ix, len(t), cap)
        with pytest.raises(mpm.MpmError) as e:
            sc.scan(td)
        assert e.value.status == mpm.MPM_EOVERFLOW
        assert int(sc.total.item()) == len(want[0])
        if cap:
            got = mpm.pairs_numpy(sc.out[:cap])
            assert_same(got, (want[0][:cap], want[1][:cap]), f"prefix {cap}")


@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_mixed_no_alloc_entry_point(mpm, algo):
    t = synth.est_text(200_000, seed=41)
    P = synth.mixed_pattern_set(t, 300, 8, 20, 200, seed=42, n_prefix=60)
    want = oracle.parallel_scan(oracle.AC(P), t)
    ix = build(mpm, algo, P)
    say(f"[mixed no-alloc] {algo}")
    td = to_dev(t)
    cap = len(want[0]) + 8
    out = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = mpm._L.mpm_scan_noalloc(ix.handle, C.c_void_p(td.data_ptr()), len(t),
                                 C.c_void_p(out.data_ptr()), cap, C.c_void_p(total.data_ptr()),
                                 None, mpm._stream_handle())
    assert st == mpm.MPM_OK, mpm._L.mpm_last_error()
    torch.cuda.synchronize()
    n = int(total.item())
    assert_same(mpm.pairs_numpy(out[:n]), want, "no-alloc")


def test_mixed_rejects_what_it_does_not_run(mpm):
    P = [b"ACG", b"ACGTA"]
    for algo in ("ac", "wm"):
        ix = build(mpm, algo, P)
        for flags in (mpm.VARIANT_ILP2, mpm.VARIANT_DENSE):
            with pytest.raises(mpm.MpmError) as e:
                mpm.workspace_bytes(ix, 1 << 20, mpm.variant(block_threads=1024, flags=flags))
            assert e.value.status == mpm.MPM_EUNSUPPORTED


@pytest.mark.parametrize("size", [1 << 20, 256 << 20], ids=["1MiB", "256MiB"])
@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_mixed_full_size(mpm, algo, size):
    """EST-shaped text, d = 1,000 patterns of lengths 8..32 (text windows,
    their prefixes and suffixes, duplicates and random strings): the whole
    list against the oracle's."""
    t = synth.est_text(size, seed=51)
    P = synth.mixed_pattern_set(t, 1000, 8, 32, 500, seed=52, n_prefix=200, n_suffix=100,
                                n_dup=50)
    say(f"[mixed full {size >> 20} MiB] oracle")
    want = oracle.parallel_scan(oracle.AC(P), t)
    ix = build(mpm, algo, P)
    say(f"[mixed full {size >> 20} MiB] {algo}: {len(want[0])} pairs")
    out = mpm.scan(ix, to_dev(t), capacity=len(want[0]) + 64)
    assert_same(mpm.pairs_numpy(out), want, f"{algo} {size}")
    assert len(want[0]) > size // 4096
