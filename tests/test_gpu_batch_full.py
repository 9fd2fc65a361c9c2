"""GPU parity of the batched workload at full size: 4,096 EST-shaped texts of
log-uniform length (1 KiB to 4 MiB, 2 GB in all) paired with 64 resident
pattern sets (d log-uniform 100 to 50k, m in {8, 12, 16, 24, 32}), each text
scanned in one persistent batched launch per walker kind, captured as one
HIP graph and replayed. Every text's list is compared with the oracle's by
its pair count and its order-sensitive 64-bit digest (written by
tests/golden/make_digests.py from the CPU oracle alone), on every replay,
under three variant assignments: the default variant for every text, a
seeded random variant per text (all 24 of the autotuner's variants occur),
and Wu-Manber everywhere."""

import hashlib
import json
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import listdigest  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(GOLDEN, "batch_digests.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def batch(golden):
    from paper_1407_2889_amd import batch as B
    from paper_1407_2889_amd import tune
    say("[batch4096] generating 4,096 texts and 64 pattern sets")
    b = synth.workload_batch(n_texts=4096, n_sets=64, seed=20)
    assert hashlib.sha256(b.meta["stream"].tobytes()).hexdigest() == golden["stream_sha256"]
    assert [hashlib.sha256(ps.patterns.tobytes()).hexdigest() for ps in b.sets] == \
        golden["patterns_sha256"]
    assert b.pairing.tolist() == golden["pairing"]
    say("[batch4096] building 128 indexes")
    sets = [tune.PatternSetIndexes.build(ps.patterns) for ps in b.sets]
    arena, offs, lens = B.pack_texts(b.texts)
    return b, sets, arena, offs, lens


def check(bs, golden, what):
    counts = np.array(golden["counts"], np.int64)
    tot = bs.totals_host()
    bad = np.nonzero(tot != counts)[0]
    assert bad.size == 0, f"{what}: text {bad[0]}: {tot[bad[0]]} pairs vs oracle {counts[bad[0]]}"
    dev_counts = torch.from_numpy(tot.astype(np.int64)).cuda()
    starts = torch.from_numpy(bs.out_offs[:-1].astype(np.int64)).cuda()
    dg = listdigest.segment_digests_torch(bs.out, starts, dev_counts)
    want = [int(x, 16) for x in golden["digests"]]
    bad = [i for i in range(len(want)) if dg[i] != want[i]]
    assert not bad, f"{what}: {len(bad)} texts' lists differ from the oracle's (first: {bad[0]})"


@pytest.mark.parametrize("assign", ["default", "random", "wm"])
def test_batch_4096_graph_replays_equal_oracle(batch, golden, assign):
    from paper_1407_2889_amd import batch as B
    from paper_1407_2889_amd import selection, tune
    b, sets, arena, offs, lens = batch
    R = len(lens)
    valid = np.array([[s.lds_fits(k) for k in range(len(tune.VARIANTS))] for s in sets])
    rng = np.random.default_rng(4242)
    choice = []
    for i in range(R):
        v = valid[int(b.pairing[i])]
        if assign == "default":
            k = selection.uniform_choice(tune.DEFAULT_VARIANT, v)
        elif assign == "random":
            k = int(rng.choice(np.nonzero(v)[0]))
        else:
            k = selection.uniform_choice(tune.VARIANTS.index(("wm", 256, 256, tune.PLACEMENTS[0])), v)
        choice.append(k)
    if assign == "random":
        assert len(set(choice)) == len(tune.VARIANTS)
    idx = [sets[int(b.pairing[i])].index(choice[i]) for i in range(R)]
    var = [tune.variant_struct(choice[i]) for i in range(R)]
    caps = np.array(golden["counts"], np.int64)
    say(f"[batch4096 {assign}] planning {R} requests")
    bs = B.BatchScan(arena, offs, lens, idx, var, caps)
    say(f"[batch4096 {assign}] {bs.groups} launches; direct run")
    bs.run()
    torch.cuda.synchronize()
    check(bs, golden, f"{assign} direct")
    bs.capture()
    for rep in range(2):
        bs.totals.zero_()
        bs.out.fill_(-1)
        torch.cuda.synchronize()
        bs.replay()
        torch.cuda.synchronize()
        say(f"[batch4096 {assign}] replay {rep}")
        check(bs, golden, f"{assign} replay {rep}")
