"""GPU: batched persistent launches (per-text parity with the oracle, HIP graph
replays) and the autotuner's timing call."""

import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def mpm():
    import paper_1407_2889_amd as m
    return m


@pytest.fixture(scope="module")
def small_batch():
    b = synth.workload_batch(n_texts=40, n_sets=5, max_len=200_000, d_hi=3000, seed=300)
    texts = list(b.texts)
    # edge texts: empty, shorter than m, exactly m
    texts[0] = texts[0][:0]
    texts[1] = texts[1][:3]
    m2 = b.sets[int(b.pairing[2])].m
    texts[2] = texts[2][:m2]
    want = [oracle.Win(b.sets[int(b.pairing[i])].patterns).scan(texts[i]) for i in range(len(texts))]
    return b, texts, want


def build_requests(mpm, b, texts, want, seed):
    from paper_1407_2889_amd import tune
    rng = np.random.default_rng(seed)
    sets = [tune.PatternSetIndexes.build(ps.patterns) for ps in b.sets]
    idx, var = [], []
    for i in range(len(texts)):
        s = sets[int(b.pairing[i])]
        while True:
            k = int(rng.integers(0, len(tune.VARIANTS)))
            if s.lds_fits(k):
                break
        idx.append(s.index(k))
        v = tune.variant_struct(k)
        if rng.random() < 0.2:
            v.flags = mpm.VARIANT_NO_SWAR
        var.append(v)
    caps = [len(w[0]) + (i % 3) for i, w in enumerate(want)]
    return sets, idx, var, caps


def check_all(bs, want, tag):
    tot = bs.totals_host()
    for i, (wp, wi) in enumerate(want):
        assert int(tot[i]) == len(wp), f"{tag} text {i}: total {int(tot[i])} vs {len(wp)}"
        gp, gi = bs.result(i, tot)
        assert np.array_equal(gp, wp) and np.array_equal(gi, wi), f"{tag} text {i}"


def test_batch_parity_and_graph_replays(mpm, small_batch):
    from paper_1407_2889_amd import batch
    b, texts, want = small_batch
    sets, idx, var, caps = build_requests(mpm, b, texts, want, seed=1)
    arena, offs, lens = batch.pack_texts(texts)
    bs = batch.BatchScan(arena, offs, lens, idx, var, caps)
    say(f"[batch] {len(texts)} texts, {bs.groups} launches, eager run")
    bs.run()
    torch.cuda.synchronize()
    check_all(bs, want, "eager")
    bs.capture()
    for rep in range(3):
        bs.out.fill_(-1)        # eager work between replays
        bs.totals.fill_(12345)
        torch.cuda.synchronize()
        say(f"[batch] graph replay {rep}")
        bs.replay()
        torch.cuda.synchronize()
        check_all(bs, want, f"replay {rep}")


def test_batch_all_variants_one_set(mpm):
    """One text through every variant of the grid in one batch."""
    from paper_1407_2889_amd import batch, tune
    t = synth.est_text(300_000, seed=41)
    ps = synth.pattern_set(t, d=400, m=12, n_planted=200, seed=42)
    want = oracle.Win(ps.patterns).scan(t)
    s = tune.PatternSetIndexes.build(ps.patterns)
    ks = [k for k in range(len(tune.VARIANTS)) if s.lds_fits(k)]
    assert len(ks) == 24
    arena, offs, lens = batch.pack_texts([t] * len(ks))
    bs = batch.BatchScan(arena, offs, lens, [s.index(k) for k in ks],
                         [tune.variant_struct(k) for k in ks], [len(want[0])] * len(ks))
    say(f"[batch] 24 variants, {bs.groups} launches")
    bs.run()
    torch.cuda.synchronize()
    check_all(bs, [want] * len(ks), "variants")


def test_tune_time_all_variants(mpm):
    from paper_1407_2889_amd import tune
    t = synth.est_text(50_000, seed=43)
    ps = synth.pattern_set(t, d=2000, m=16, n_planted=200, seed=44)
    s = tune.PatternSetIndexes.build(ps.patterns)
    tuner = tune.Tuner()
    td = torch.from_numpy(t).cuda()
    assert tuner.count(s, td) == len(oracle.Win(ps.patterns).scan(t)[0])
    say("[tune] timing 24 variants")
    ms = tuner.time_all(s, td)
    assert ms.shape == (24,)
    runnable = np.array([s.lds_fits(k) for k in range(24)])
    assert np.all(np.isfinite(ms[runnable])) and np.all(ms[runnable] > 0)
    assert np.all(np.isinf(ms[~runnable]))
    assert runnable.sum() >= 18
    f = tuner.features(s, td)
    assert f.shape == (7,) and math.isclose(f[2], 16)
    # a set whose automaton cannot live in LDS marks those variants invalid
    big = synth.pattern_set(t, d=20000, m=32, n_planted=100, seed=45)
    sb = tune.PatternSetIndexes.build(big.patterns)
    msb = tuner.time_all(sb, td[:20000])
    lds_ac = [k for k, v in enumerate(tune.VARIANTS) if v[0] == "ac" and v[3] == 1]
    assert np.all(np.isinf(msb[lds_ac]))
    assert np.isfinite(msb).sum() >= 12
