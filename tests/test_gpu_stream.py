"""GPU: scanning a text held in host memory, chunk by chunk through two
device staging buffers, against the oracle element by element: several
chunk sizes (one chunk, ragged last chunk, chunks shorter than a workgroup's
tile, chunks of one starting position), pinned and pageable host memory,
capacity overflow, and texts shorter than m."""

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


@pytest.fixture(scope="module")
def case():
    t = synth.est_text(3_000_000, seed=51)
    ps = synth.pattern_set(t, d=800, m=12, n_planted=400, seed=52)
    want = oracle.Win(ps.patterns).scan(t)
    assert len(want[0]) >= 400
    return t, ps.patterns, want


def check(mpm, got, want, what):
    gp, gi = mpm.pairs_numpy(got)
    assert len(gp) == len(want[0]), f"{what}: {len(gp)} pairs vs oracle {len(want[0])}"
    assert np.array_equal(gp, want[0]) and np.array_equal(gi, want[1]), what


@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_host_text_chunks(mpm, case, algo):
    t, P, want = case
    ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(P, upload=True)
    pinned = torch.empty(len(t), dtype=torch.uint8, pin_memory=True)
    pinned.numpy()[:] = t
    for chunk in (1 << 30, 1 << 20, 777_777, 3000):
        say(f"[stream] {algo} chunk={chunk}")
        check(mpm, mpm.scan_host(ix, pinned, chunk=chunk), want, f"{algo} chunk {chunk}")
    # pageable host memory
    check(mpm, mpm.scan_host(ix, torch.from_numpy(t), chunk=1 << 20), want, f"{algo} pageable")


def test_host_text_overflow_and_short(mpm, case):
    t, P, want = case
    ix = mpm.build_ac(P, upload=True)
    half = len(want[0]) // 2
    with pytest.raises(mpm.MpmError) as e:
        mpm.scan_host(ix, t, chunk=500_000, capacity=half)
    assert e.value.status == mpm.MPM_EOVERFLOW
    # a short text (fewer bytes than m) and chunks of one starting position
    check(mpm, mpm.scan_host(ix, t[:11], chunk=1), (want[0][:0], want[1][:0]), "n < m")
    short = t[:2000]
    w = oracle.Win(P).scan(short)
    check(mpm, mpm.scan_host(ix, short, chunk=1), w, "chunk 1")
    check(mpm, mpm.scan_host(ix, short, chunk=7), w, "chunk 7")
