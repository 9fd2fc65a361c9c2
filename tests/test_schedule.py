"""Host-only: the batch plan model and the scheduler that minimises it."""

import numpy as np
import pytest

from paper_1407_2889_amd import selection


class FakeSet:
    """Launch keys without a GPU: variants 2j and 2j+1 share launch j."""

    def __init__(self, shift=0):
        self.shift = shift

    def launch_key(self, k):
        return k // 2 + self.shift


def random_case(seed, R=60, V=8):
    rng = np.random.default_rng(seed)
    cost = rng.uniform(0.001, 0.05, (R, V))
    chunk = cost * rng.uniform(0.05, 2.0, (R, V))
    valid = rng.random((R, V)) < 0.9
    valid[:, 0] = True
    pset = [FakeSet() for _ in range(R)]
    return cost, chunk, valid, pset


def brute_plan_ms(choice, cost, chunk, keys):
    """The model written out per launch, as a check of plan_ms."""
    launches = {}
    for i, k in enumerate(choice):
        launches.setdefault(int(keys[i, k]), []).append((cost[i, k], chunk[i, k]))
    total, excess, longest = 0.0, 0.0, 0.0
    for members in launches.values():
        S = sum(c for c, _ in members)
        Cm = max(h for _, h in members)
        total += S
        excess += max(0.0, Cm - S)
        longest = max(longest, Cm)
    return max(total + selection.LAUNCH_MS * len(launches) + selection.EXCESS * excess,
               selection.CHUNK * longest)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_plan_ms_matches_definition(seed):
    cost, chunk, valid, pset = random_case(seed)
    keys = selection.launch_keys(pset, valid)
    rng = np.random.default_rng(seed + 100)
    for _ in range(5):
        choice = np.array([rng.choice(np.flatnonzero(valid[i])) for i in range(len(cost))])
        assert selection.plan_ms(choice, cost, chunk, keys) == pytest.approx(
            brute_plan_ms(choice, cost, chunk, keys))


@pytest.mark.parametrize("seed", [4, 5])
def test_incremental_delta_equals_recomputed_model(seed):
    cost, chunk, valid, pset = random_case(seed)
    keys = selection.launch_keys(pset, valid)
    rng = np.random.default_rng(seed)
    choice = np.array([rng.choice(np.flatnonzero(valid[i])) for i in range(len(cost))])
    plan = selection._Plan(choice.copy(), cost, chunk, keys)
    for _ in range(200):
        i = int(rng.integers(len(cost)))
        k = int(rng.choice(np.flatnonzero(valid[i])))
        before = selection.plan_ms(plan.choice, cost, chunk, keys)
        d = plan.delta(i, k)
        plan.move(i, k)
        after = selection.plan_ms(plan.choice, cost, chunk, keys)
        assert d == pytest.approx(after - before, abs=1e-12)


@pytest.mark.parametrize("seed", [6, 7, 8])
def test_schedule_no_worse_than_any_start(seed):
    cost, chunk, valid, pset = random_case(seed)
    keys = selection.launch_keys(pset, valid)
    R, V = cost.shape
    best_req = np.argmin(np.where(valid, cost, np.inf), axis=1)
    out = selection.schedule(best_req, cost, chunk, valid, pset, keys)
    assert valid[np.arange(R), out].all()
    t = selection.plan_ms(out, cost, chunk, keys)
    assert t <= selection.plan_ms(best_req, cost, chunk, keys) + 1e-12
    for k in range(V):
        u = np.array([selection.uniform_choice(k, valid[i]) if valid[i, k] else 0
                      for i in range(R)])
        if valid[np.arange(R), u].all():
            assert t <= selection.plan_ms(u, cost, chunk, keys) + 1e-12


def test_schedule_moves_a_long_chunk_out_of_a_cheap_launch():
    # request 0 is cheapest under variant 0 but one of its chunks there runs
    # far longer than the whole batch's work: the plan takes variant 2
    R, V = 20, 4
    cost = np.full((R, V), 0.01)
    cost[:, 0] = 0.005
    chunk = np.full((R, V), 0.001)
    chunk[0, 0] = 1.0
    valid = np.ones((R, V), bool)
    pset = [FakeSet() for _ in range(R)]
    keys = selection.launch_keys(pset, valid)
    out = selection.schedule(np.zeros(R, int), cost, chunk, valid, pset, keys)
    assert keys[0, out[0]] != keys[0, 0] or chunk[0, out[0]] < 1.0
    assert out[0] != 0
    assert (out[1:] <= 1).all()


def test_schedule_dissolves_small_launches():
    # every request's best is its own launch; per-launch overheads make one
    # launch cheaper overall
    R, V = 6, 12
    cost = np.full((R, V), 0.004)
    for i in range(R):
        cost[i, 2 * i] = 0.003
    chunk = cost / 100
    valid = np.ones((R, V), bool)
    pset = [FakeSet() for _ in range(R)]
    keys = selection.launch_keys(pset, valid)
    best = np.argmin(cost, axis=1)
    out = selection.schedule(best, cost, chunk, valid, pset, keys)
    assert len(set(keys[np.arange(R), out])) == 1
