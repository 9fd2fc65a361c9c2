"""GPU parity: the HIP scan through the C-ABI against the CPU oracle,
element by element (bit-exact (pos, id) lists)."""

import itertools
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mpm():
    import paper_1407_2889_amd as m
    assert torch.cuda.is_available()
    return m


def to_dev(text: np.ndarray, misalign: int = 0):
    """Device copy of text starting `misalign` bytes into a 256-aligned buffer."""
    buf = torch.zeros(len(text) + misalign + 64, dtype=torch.uint8, device="cuda")
    if len(text):
        buf[misalign:misalign + len(text)] = torch.from_numpy(np.ascontiguousarray(text)).cuda()
    return buf[misalign:misalign + len(text)]


def gpu_pairs(mpm, ix, text, var=None, misalign=0, capacity=None):
    t = to_dev(text, misalign)
    out = mpm.scan(ix, t, capacity=capacity, var=var)
    return mpm.pairs_numpy(out)


def assert_same(got, want, what=""):
    gp, gi = got
    wp, wi = want
    assert len(gp) == len(wp), f"{what}: {len(gp)} pairs vs oracle {len(wp)}"
    if len(wp):
        bad = np.nonzero((gp != wp) | (gi != wi))[0]
        assert bad.size == 0, f"{what}: first mismatch at {bad[0]}: got {(gp[bad[0]], gi[bad[0]])} want {(wp[bad[0]], wi[bad[0]])}"


VARIANTS = [dict(lane_bytes=L, block_threads=W, placement=P, flags=F)
            for L, W, P, F in itertools.product((16, 64, 256), (256, 512, 1024), (1, 2), (0, 1, 2, 3))]


@pytest.fixture(scope="module")
def small():
    text, ps = synth.workload_small()
    want = oracle.parallel_scan(oracle.Win(ps.patterns), text)
    return text, ps.patterns, want


@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_small_workload_all_variants(mpm, small, algo):
    text, P, want = small
    ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(P, upload=True)
    for v in VARIANTS:
        say(f"[small 1MiB d=100 m=8] {algo} {v}")
        got = gpu_pairs(mpm, ix, text, mpm.variant(**v))
        assert_same(got, want, f"{algo} {v}")
    assert len(want[0]) > 800


def edge_cases():
    rng = np.random.default_rng(11)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    cases = []
    cases.append(("empty", np.zeros(0, np.uint8), acgt[rng.integers(0, 4, (5, 4))]))
    cases.append(("n<m", acgt[rng.integers(0, 4, 3)], acgt[rng.integers(0, 4, (5, 4))]))
    t = acgt[rng.integers(0, 4, 8)]
    cases.append(("n==m", t, np.stack([t, t, acgt[rng.integers(0, 4, 8)]])))
    t = acgt[rng.integers(0, 4, 100_003)]
    P = acgt[rng.integers(0, 4, (64, 6))]
    P[:20] = np.stack([t[s:s + 6] for s in rng.integers(0, len(t) - 6, 20)])
    cases.append(("ragged", t, P))
    cases.append(("all-A dense", np.full(70_001, ord("A"), np.uint8),
                  np.full((3, 5), ord("A"), np.uint8)))
    t = np.frombuffer(b"ACGT\n", np.uint8)[rng.integers(0, 5, 50_000)]
    cases.append(("newline-dense", t, acgt[rng.integers(0, 4, (200, 3))]))
    t = acgt[rng.integers(0, 4, 30_000)]
    P = acgt[rng.integers(0, 4, (50, 4))]
    P[10:30] = P[0]
    P[0] = t[100:104]
    cases.append(("duplicates", t, P))
    cases.append(("m=1", acgt[rng.integers(0, 4, 20_000)], np.frombuffer(b"ACX", np.uint8).reshape(3, 1)))
    t = synth.est_text(200_000, seed=5)
    ps = synth.pattern_set(t, d=300, m=32, n_planted=150, seed=6)
    cases.append(("m=32 est", t, ps.patterns))
    t = synth.est_text(150_000, seed=7)
    ps = synth.pattern_set(t, d=5000, m=8, n_planted=2500, seed=8)
    cases.append(("m=8 d=5000 dense", t, ps.patterns))
    bytes_all = rng.integers(0, 256, 40_000).astype(np.uint8)
    P = np.stack([bytes_all[s:s + 5] for s in rng.integers(0, 40_000 - 5, 30)])
    cases.append(("binary alphabet", bytes_all, P))
    # every byte value is a pattern byte: 256 symbol classes
    t = rng.integers(0, 256, 60_000).astype(np.uint8)
    P = np.concatenate([rng.permutation(256).astype(np.uint8).reshape(32, 8),
                        np.stack([t[s:s + 8] for s in rng.integers(0, 60_000 - 8, 40)])])
    cases.append(("all 256 byte values", t, P))
    return cases


@pytest.mark.parametrize("case", edge_cases(), ids=lambda c: c[0])
@pytest.mark.parametrize("algo", ["ac", "wm", "ac-supply", "ac-text"])
def test_edge_cases(mpm, case, algo):
    name, T, P = case
    want = oracle.Win(P).scan(T)
    assert_same(oracle.AC(P).scan(T), want, "oracle AC")
    if algo == "wm":
        ix = mpm.build_wm(P, upload=True)
    else:
        ix = mpm.build_ac(P, upload=True, goto=algo == "ac-supply")
    variants = (dict(lane_bytes=16, block_threads=256), dict(lane_bytes=64, block_threads=1024),
                dict(lane_bytes=256, block_threads=512, placement=2),
                dict(lane_bytes=32, block_threads=256, flags=2),
                dict(lane_bytes=128, block_threads=1024, flags=3),
                dict(block_threads=1024, flags=mpm.VARIANT_DENSE),
                dict(block_threads=1024, placement=2, flags=mpm.VARIANT_DENSE))
    if algo == "ac-supply":
        variants = tuple(dict(v, flags=mpm.VARIANT_SUPPLY) for v in variants if not v.get("flags"))
    if algo == "ac-text":
        # the text-access variants of the kernel ladder: bytes from global
        # memory, or the chunk's text staged in LDS
        variants = tuple(dict(lane_bytes=L, block_threads=W, placement=pl, flags=f)
                         for L, W in ((16, 256), (64, 1024), (48, 512))
                         for pl in (1, 2)
                         for f in (mpm.VARIANT_TEXT_BYTES, mpm.VARIANT_TEXT_LDS))
    for mis in (0, 3):
        for v in variants:
            say(f"[edge {name} n={len(T)} d={len(P)} m={P.shape[1]}] {algo} misalign={mis} {v}")
            try:
                got = gpu_pairs(mpm, ix, T, mpm.variant(**v), misalign=mis)
            except mpm.MpmError as e:
                # ladder variants: 32-bit tables, or LDS tables beside the staged text
                if algo == "ac-text" and e.status == mpm.MPM_EUNSUPPORTED:
                    continue
                raise
            assert_same(got, want, f"{name} {algo} mis={mis} {v}")


@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_dense_output_all_placements(mpm, algo):
    """Dense output (position marks in LDS, waves writing consecutive slots)
    on a set with about one occurrence per position and repeated strings
    (several id-count groups), every placement, aligned and misaligned text,
    full lists and overflowing capacities."""
    t = synth.est_text(3_000_000, seed=51)
    ps = synth.pattern_set(t, d=20000, m=8, n_planted=5000, seed=52)
    P = ps.patterns.copy()
    P[100:160] = P[0]          # one string with 61 ids
    P[200:203] = P[1]          # one with 4
    want = oracle.parallel_scan(oracle.Win(P), t)
    assert len(want[0]) > len(t) // 5
    ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(P, upload=True)
    for pl in (0, 1, 2, 3):
        v = mpm.variant(block_threads=1024, placement=pl, flags=mpm.VARIANT_DENSE)
        for mis in (0, 5):
            say(f"[dense] {algo} placement={pl} misalign={mis}")
            try:
                got = gpu_pairs(mpm, ix, t, v, misalign=mis)
            except mpm.MpmError as e:
                # the tables (or their hot part) and the marks exceed the LDS
                assert e.status == mpm.MPM_EUNSUPPORTED and pl in (1, 3)
                break
            assert_same(got, want, f"dense {algo} pl={pl} mis={mis}")
    dev = to_dev(t)
    for cap in (0, 1, 777, len(want[0]) - 1):
        say(f"[dense] {algo} capacity {cap}")
        sc = mpm.Scanner(ix, len(t), cap, mpm.variant(block_threads=1024, flags=mpm.VARIANT_DENSE))
        with pytest.raises(mpm.MpmError):
            sc.scan(dev)
        assert int(sc.total.item()) == len(want[0])
        got = mpm.pairs_numpy(sc.out[:cap])
        assert_same(got, (want[0][:cap], want[1][:cap]), f"dense prefix {cap}")


@pytest.mark.parametrize("m", [1, 5, 16, 17, 18, 33, 34])
def test_dense_output_pattern_lengths(mpm, m):
    """Dense Aho-Corasick lanes read their 16 + m - 1 bytes as two (m <= 17)
    or three (m <= 33) 16-byte pieces up front and walk them from registers;
    longer patterns, misaligned text and the lanes near the text's end take
    the byte walk. Every length boundary, at text offsets 0 and 3, for texts
    ending inside a lane and inside the last pieces."""
    t = synth.est_text(300_000, seed=60 + m)
    ps = synth.pattern_set(t, d=300, m=m, n_planted=200, seed=61 + m)
    ix = mpm.build_ac(ps.patterns, upload=True)
    for nn in (len(t), 16 * 1024 * 5 + 16 + m, 16 * 1024 * 5 + 47, 16 * 1024 * 2 + 9):
        tt = t[:nn]
        want = oracle.Win(ps.patterns).scan(tt)
        for pl in (0, 2):
            for mis in (0, 3):
                v = dict(block_threads=1024, placement=pl, flags=mpm.VARIANT_DENSE)
                say(f"[dense-m] m={m} n={nn} misalign={mis} {v}")
                got = gpu_pairs(mpm, ix, tt, mpm.variant(**v), misalign=mis)
                assert_same(got, want, f"dense m={m} n={nn} mis={mis} {v}")
        assert len(want[0]) > 0


@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_capacity_overflow_keeps_sorted_prefix(mpm, small, algo):
    text, P, want = small
    ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(P, upload=True)
    t = to_dev(text)
    cap = len(want[0]) // 3
    say(f"[overflow] {algo} cap={cap}")
    sc = mpm.Scanner(ix, len(text), cap)
    with pytest.raises(mpm.MpmError) as e:
        sc.scan(t)
    assert e.value.status == mpm.MPM_EOVERFLOW
    got = mpm.pairs_numpy(sc.out[:cap])
    assert_same(got, (want[0][:cap], want[1][:cap]), "prefix")
    assert int(sc.total.item()) == len(want[0])
    # capacity 0: count only
    sc0 = mpm.Scanner(ix, len(text), 0)
    with pytest.raises(mpm.MpmError):
        sc0.scan(t)
    assert int(sc0.total.item()) == len(want[0])


@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_repeat_determinism_and_workspace_reuse(mpm, small, algo):
    text, P, want = small
    ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(P, upload=True)
    t = to_dev(text)
    for v in (mpm.variant(lane_bytes=16, block_threads=256, grid=7),
              mpm.variant(lane_bytes=64, block_threads=1024),
              mpm.variant(lane_bytes=48, block_threads=512, grid=5, flags=2)):
        sc = mpm.Scanner(ix, len(text), len(want[0]) + 10, v)
        for rep in range(6):
            say(f"[repeat] {algo} {v} rep={rep}")
            got = mpm.pairs_numpy(sc.scan(t))
            assert_same(got, want, f"rep {rep}")
        # shorter text through the same workspace
        got = mpm.pairs_numpy(sc.scan(t[:100_000]))
        w2 = oracle.Win(P).scan(text[:100_000])
        assert_same(got, w2, "prefix text")


@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_est256_full_list(mpm, algo):
    """The 256 MiB EST-shaped text, d=1000, m=16, full match list, in the
    launch configuration the benchmark times."""
    import bench
    say(f"[est256] generating")
    text, ps = synth.workload_est256()
    want = oracle.parallel_scan(oracle.Win(ps.patterns), text)
    assert len(want[0]) >= 300
    ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(ps.patterns, upload=True)
    v = bench.DEFAULT_VARIANTS[algo]
    say(f"[est256] {algo} {v}")
    got = gpu_pairs(mpm, ix, text, mpm.variant(**v))
    assert_same(got, want, f"est256 {algo}")
    # planted patterns all occur at their recorded starts
    found = set(zip(got[0].tolist(), got[1].tolist()))
    for r, s in enumerate(ps.planted_starts.tolist()):
        assert (s, r) in found


@pytest.mark.parametrize("algo", ["ac", "ac32", "wm"])
def test_hot_placement_large_tables(mpm, algo):
    """Tables larger than LDS: the hot part in LDS (the first rows of the
    Aho-Corasick table in breadth-first order; the Wu-Manber SHIFT table), the
    rest read through the caches. Bit-exact against the oracle, alone and as
    the automatic choice, at text offsets 0 and 5."""
    t = synth.est_text(2_500_000, seed=31)
    if algo == "ac":
        ps = synth.pattern_set(t, d=3000, m=20, n_planted=1500, seed=32)
    elif algo == "ac32":
        ps = synth.pattern_set(t, d=6000, m=20, n_planted=3000, seed=34)
    else:
        ps = synth.pattern_set(t, d=20000, m=16, n_planted=2000, seed=33)
    want = oracle.Win(ps.patterns).scan(t)
    ix = (mpm.build_wm if algo == "wm" else mpm.build_ac)(ps.patterns, upload=True)
    info = ix.info()
    assert info["table_bytes"] > 160 * 1024
    if algo != "wm":
        assert info["state_bytes"] == (2 if algo == "ac" else 4)
    with pytest.raises(mpm.MpmError):  # the whole table does not fit
        mpm.workspace_bytes(ix, len(t), mpm.variant(lane_bytes=64, block_threads=256,
                                                    placement=mpm.PLACE_LDS))
    for mis in (0, 5):
        for v in (dict(lane_bytes=64, block_threads=256, placement=mpm.PLACE_HOT),
                  dict(lane_bytes=1024, block_threads=1024, placement=mpm.PLACE_HOT),
                  dict(lane_bytes=256, block_threads=512, placement=mpm.PLACE_AUTO),
                  dict(lane_bytes=128, block_threads=256, placement=mpm.PLACE_HOT, flags=1)):
            say(f"[hot] {algo} d={len(ps.patterns)} misalign={mis} {v}")
            got = gpu_pairs(mpm, ix, t, mpm.variant(**v), misalign=mis)
            assert_same(got, want, f"hot {algo} mis={mis} {v}")


def test_per_pattern_counts(mpm, small):
    """Per-pattern counts of the scan's list (the counts of Section 4.2 summed
    per pattern) against the oracle's list counted per id, on the 1 MiB
    workload and on a dense set whose id range spans two LDS histograms."""
    text, P, want = small
    ix = mpm.build_ac(P, upload=True)
    out = mpm.scan(ix, to_dev(text))
    got = mpm.count_ids(out, len(P)).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, np.bincount(want[1], minlength=len(P)))
    t = synth.est_text(1_500_000, seed=41)
    ps = synth.pattern_set(t, d=50000, m=8, n_planted=5000, seed=42)
    want = oracle.Win(ps.patterns).scan(t)
    ix = mpm.build_wm(ps.patterns, upload=True)
    out = mpm.scan(ix, to_dev(t))
    assert out.shape[0] == len(want[0]) > 100_000
    got = mpm.count_ids(out, 50000).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, np.bincount(want[1], minlength=50000))


def test_per_pattern_counts_edges(mpm):
    """Counting edge cases on synthetic lists: an empty list zeroes the
    counts, ids not below d are skipped, a list length that is not a multiple
    of the unrolled stride, and three id slices."""
    c = torch.full((100,), 7, dtype=torch.int32, device="cuda")
    mpm.count_ids(torch.empty((0, 2), dtype=torch.int32, device="cuda"), 100, out=c)
    assert int(c.abs().sum()) == 0
    rng = np.random.default_rng(43)
    for d, M in ((1, 5), (100, 1), (1000, 3_000_001), (100_000, 2_000_003)):
        ids = rng.integers(0, d + 50, M).astype(np.uint32)
        pairs = np.stack([np.arange(M, dtype=np.uint32), ids], axis=1)
        dev = torch.from_numpy(pairs.view(np.int32)).cuda()
        say(f"[counts] d={d} M={M}")
        got = mpm.count_ids(dev, d).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, np.bincount(ids[ids < d], minlength=d)), (d, M)


@pytest.mark.parametrize("case", ["small", "est", "u32"])
def test_supply_walk(mpm, small, case):
    """The goto function with supply links at run time (the paper's kernel
    design) against the oracle: tables in LDS and in global memory, 16- and
    32-bit states, several launch shapes, text offsets 0 and 3."""
    if case == "small":
        t, P, want = small
    else:
        t = synth.est_text(2_000_000, seed=61)
        d, m = (1000, 16) if case == "est" else (6000, 20)
        P = synth.pattern_set(t, d=d, m=m, n_planted=d // 3, seed=62).patterns
        want = oracle.Win(P).scan(t)
    ix = mpm.build_ac(P, upload=True, goto=True)
    assert ix.info()["state_bytes"] == (4 if case == "u32" else 2)
    sup = mpm.VARIANT_SUPPLY
    for mis in (0, 3):
        for v in (dict(lane_bytes=64, block_threads=256, placement=mpm.PLACE_AUTO, flags=sup),
                  dict(lane_bytes=1024, block_threads=1024, placement=mpm.PLACE_GLOBAL, flags=sup),
                  dict(lane_bytes=16, block_threads=512, placement=mpm.PLACE_AUTO, flags=sup)):
            say(f"[supply] {case} misalign={mis} {v}")
            got = gpu_pairs(mpm, ix, t, mpm.variant(**v), misalign=mis)
            assert_same(got, want, f"supply {case} mis={mis} {v}")


@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_persistent_grid_sizes(mpm, small, algo):
    """The same list whatever the number of persistent workgroups taking
    chunk tickets (one workgroup walking every chunk in turn, a few, a
    prime number, more than the chunks), repeated on one workspace."""
    text, P, want = small
    ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(P, upload=True)
    t = to_dev(text)
    for grid in (1, 3, 17, 256, 4096):
        v = mpm.variant(lane_bytes=64, block_threads=256, grid=grid)
        sc = mpm.Scanner(ix, len(text), capacity=len(want[0]) + 16, var=v)
        for rep in range(3):
            say(f"[grid] {algo} grid={grid} rep={rep}")
            assert_same(mpm.pairs_numpy(sc.scan(t)), want, f"{algo} grid={grid} rep={rep}")
