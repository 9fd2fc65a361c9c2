"""Host-only: index builders for pattern sets of different lengths (no GPU)."""

import numpy as np
import pytest

import paper_1407_2889_amd as mpm
import synth


def brute_lists(P):
    """For each distinct string u: the ascending ids of every pattern that is
    a prefix of u (those occur wherever u does)."""
    distinct = sorted(set(P))
    return {u: sorted(r for r, p in enumerate(P) if u.startswith(p)) for u in distinct}


def exported_lists(ix):
    uoff, ids = ix.export_unique()
    return [list(ids[uoff[u]:uoff[u + 1]]) for u in range(len(uoff) - 1)]


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_id_lists_cover_prefix_patterns(algo, seed):
    t = synth.est_text(50_000, seed=seed)
    P = synth.mixed_pattern_set(t, 300, 3, 15, 150, seed=seed + 10, n_prefix=80, n_suffix=30,
                                n_dup=20)
    ix = (mpm.build_ac_var if algo == "ac" else mpm.build_wm_var)(P)
    inf = ix.info()
    want = brute_lists(P)
    assert inf["d"] == len(P) and inf["d_unique"] == len(want)
    assert inf["m"] == min(map(len, P)) and inf["m_max"] == max(map(len, P))
    got = exported_lists(ix)
    # the multiset of lists equals the brute force's (numbering is the builder's)
    assert sorted(map(tuple, got)) == sorted(map(tuple, want.values()))
    # numbered by list length, ascending
    lens = [len(x) for x in got]
    assert lens == sorted(lens)
    assert inf["max_dup"] == max(lens)


def test_nested_prefix_chain_lists():
    P = [b"AAAA", b"A", b"AA", b"AAA", b"AA", b"C"]
    ix = mpm.build_ac_var(P)
    got = sorted(map(tuple, exported_lists(ix)))
    assert got == sorted([(1,), (1, 2, 4), (1, 2, 3, 4), (0, 1, 2, 3, 4), (5,)])


def test_equal_lengths_give_the_fixed_index():
    rng = np.random.default_rng(4)
    P = rng.integers(0, 4, (50, 7)).astype(np.uint8)
    a = mpm.build_ac_var([p.tobytes() for p in P])
    b = mpm.build_ac(P)
    assert a.info() == b.info()
    ta, ca = a.export_ac()
    tb, cb = b.export_ac()
    assert np.array_equal(ta, tb) and np.array_equal(ca, cb)
    w = mpm.build_wm_var([p.tobytes() for p in P])
    assert w.info() == mpm.build_wm(P).info()


def test_reversed_automaton_walk_finds_longest_string_per_start():
    """Walk the exported table of the reversed strings over a text from its
    end: after the byte at q the state is the longest string that starts at q
    and ends some pattern, so it is a reporting state exactly when a pattern
    starts at q. Checked against the definition on a small text."""
    rng = np.random.default_rng(9)
    acgt = np.frombuffer(b"ACGT", np.uint8)
    t = acgt[rng.integers(0, 4, 3000)]
    P = [t[s:s + int(rng.integers(2, 7))].tobytes() for s in rng.integers(0, 2990, 25)]
    P += [p[:2] for p in P[:5]]
    ix = mpm.build_ac_var(P)
    table, classes = ix.export_ac()
    col = np.zeros(256, np.int64)
    col[classes] = np.arange(1, len(classes) + 1)
    # reporting states come last: find them as the rows reached exactly at starts
    s = 0
    states = np.empty(len(t), np.int64)
    for q in range(len(t) - 1, -1, -1):
        s = table[s, col[t[q]]]
        states[q] = s
    starts = {q for q in range(len(t)) for p in P if t[q:q + len(p)].tobytes() == p}
    reach = {q for q in range(len(t)) if states[q] >= min(states[list(starts)])} if starts else set()
    assert starts and reach == starts


def test_errors():
    with pytest.raises(mpm.MpmError) as e:
        mpm.build_ac_var([b"AC", b""])
    assert e.value.status == mpm.MPM_EINVAL
    with pytest.raises(mpm.MpmError) as e:
        mpm.build_wm_var([b"ACGT", b"AC"], B=3)
    assert e.value.status == mpm.MPM_EUNSUPPORTED
    with pytest.raises(mpm.MpmError):
        mpm.build_wm_var([])
