"""Pins for the CPU oracle (no GPU).

The oracle is only trusted once it agrees with things other than itself:
  * the values the paper prints for its worked Aho-Corasick example
    (Section 3.1; fixture tests/golden/ac_worked_example.json);
  * library routines for the special cases d = 1 (regex search with a
    look-ahead, which finds overlapping occurrences) and m = 1 (numpy equality);
  * the longest-suffix characterisation of the AC state (Section 3.1), checked
    by brute force position by position;
  * the SHIFT table's definition in words (Section 3.2), evaluated with Python
    sets;
  * exhaustive enumeration of tiny inputs, where brute force, sorted-window
    lookup, AC and WM must agree, WM for several (B, B', bitshift);
  * the contiguous split with an m-1 overlap (Section 4.4): per-range results
    concatenated in range order equal the whole-text result.
"""

import itertools
import json
import os
import re

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pairs(res):
    p, i = res
    return list(zip(p.tolist(), i.tolist()))


def rand_case(rng, alphabet=b"AC", n_max=40, d_max=6, m_max=5, m_min=1):
    m = int(rng.integers(m_min, m_max + 1))
    n = int(rng.integers(0, n_max + 1))
    d = int(rng.integers(1, d_max + 1))
    A = np.frombuffer(alphabet, np.uint8)
    T = A[rng.integers(0, len(A), n)] if n else np.zeros(0, np.uint8)
    P = A[rng.integers(0, len(A), (d, m))]
    if d > 1 and rng.random() < 0.5:  # duplicates
        P[-1] = P[0]
    if n >= m and rng.random() < 0.7:  # plant an occurrence
        s = int(rng.integers(0, n - m + 1))
        P[0] = T[s:s + m]
    return T.astype(np.uint8), P.astype(np.uint8)


# ---------------------------------------------------------------------------
# Worked example (paper-printed values)
# ---------------------------------------------------------------------------

def test_ac_worked_example_printed_values():
    with open(os.path.join(GOLDEN, "ac_worked_example.json")) as f:
        g = json.load(f)
    ac = oracle.AC([p.encode() for p in g["patterns"]])
    for q, c, want in g["printed"]["goto"]:
        assert ac.goto(q, c) == want, (q, c)
    for q, want in g["printed"]["supply"]:
        assert ac.supply(q) == want, q
    # all patterns are terminal at depth m; the example has 9 states
    assert ac.nstates == 9
    terms = [q for q in range(ac.nstates) if ac.output(q)]
    assert sorted(ac.depth(q) for q in terms) == [3, 3, 3]


def test_ac_worked_example_search():
    ac = oracle.AC([b"AAC", b"AGT", b"GTA"])
    text = b"AAGTAACGTAGT"
    got = pairs(ac.scan(text))
    # occurrences by inspection of the 12-character text
    assert got == [(1, 1), (2, 2), (4, 0), (7, 2), (9, 1)]


# ---------------------------------------------------------------------------
# Library-routine pins for the brute force (the root of trust)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(20))
def test_bf_single_pattern_matches_regex(seed):
    rng = np.random.default_rng(seed)
    T, P = rand_case(rng, alphabet=b"ACG", n_max=300, d_max=1, m_max=6)
    p = bytes(P[0])
    want = [mt.start() for mt in re.finditer(b"(?=" + re.escape(p) + b")", bytes(T))]
    pos, ids = oracle.bf(T, P)
    assert pos.tolist() == want
    assert set(ids.tolist()) <= {0}


@pytest.mark.parametrize("seed", range(10))
def test_bf_length_one_patterns_match_numpy(seed):
    rng = np.random.default_rng(100 + seed)
    T = np.frombuffer(b"ACGTN\n", np.uint8)[rng.integers(0, 6, 500)]
    P = np.frombuffer(b"ACGTNX", np.uint8)[rng.integers(0, 6, (7, 1))]
    pos, ids = oracle.bf(T, P)
    want = sorted((int(i), int(r)) for r in range(len(P)) for i in np.nonzero(T == P[r, 0])[0])
    assert pairs((pos, ids)) == want
    # per-pattern counts equal the byte histogram
    hist = np.bincount(T, minlength=256)
    for r in range(len(P)):
        assert int((ids == r).sum()) == int(hist[P[r, 0]])


def test_bf_edge_cases():
    P = np.frombuffer(b"ACGT", np.uint8).reshape(1, 4)
    assert oracle.bf(b"", P)[0].size == 0
    assert oracle.bf(b"ACG", P)[0].size == 0          # n < m
    assert pairs(oracle.bf(b"ACGT", P)) == [(0, 0)]   # n == m
    assert pairs(oracle.bf(b"AAAA", np.frombuffer(b"AA", np.uint8).reshape(1, 2))) == [(0, 0), (1, 0), (2, 0)]


# ---------------------------------------------------------------------------
# Characterisation of the AC state (Section 3.1)
# ---------------------------------------------------------------------------

def state_labels(ac):
    """L(q) for each state, recovered from the goto function by a walk from q0
    over forward (depth-increasing) edges."""
    labels = {0: b""}
    stack = [0]
    while stack:
        q = stack.pop()
        for c in range(256):
            s = ac.goto(q, c)
            if s > 0 and ac.depth(s) == ac.depth(q) + 1 and s not in labels:
                labels[s] = labels[q] + bytes([c])
                stack.append(s)
    return labels


@pytest.mark.parametrize("seed", range(12))
def test_ac_state_is_longest_suffix_that_is_a_prefix(seed):
    rng = np.random.default_rng(200 + seed)
    T, P = rand_case(rng, alphabet=b"ACG", n_max=60, d_max=5, m_max=5)
    ac = oracle.AC(P)
    labels = state_labels(ac)
    assert len(labels) == ac.nstates
    prefixes = {bytes(p[:k]) for p in P for k in range(P.shape[1] + 1)}
    tr = ac.trace(T)
    Tb = bytes(T)
    for i in range(len(Tb)):
        best = b""
        for k in range(0, i + 2):  # longest suffix first
            if Tb[k:i + 1] in prefixes:
                best = Tb[k:i + 1]
                break
        assert labels[int(tr[i])] == best, (i, best)


@pytest.mark.parametrize("seed", range(8))
def test_ac_supply_chain_has_no_other_terminal(seed):
    # Equal-length patterns: supply strictly lowers depth, so no terminal lies
    # on another terminal's supply chain (the Output merge is a no-op).
    rng = np.random.default_rng(300 + seed)
    _, P = rand_case(rng, alphabet=b"AC", n_max=0, d_max=8, m_max=6, m_min=2)
    ac = oracle.AC(P)
    m = P.shape[1]
    for q in range(1, ac.nstates):
        s = ac.supply(q)
        assert ac.depth(s) < ac.depth(q)
        while s != 0:
            assert ac.depth(s) < m and not ac.output(s)
            s = ac.supply(s)


# ---------------------------------------------------------------------------
# Wu-Manber tables against their definition (Section 3.2)
# ---------------------------------------------------------------------------

def shift_add(block, bitshift):
    h = 0
    for c in block:
        h = (h << bitshift) + c
    return h


@pytest.mark.parametrize("B,Bp,bs", [(3, 2, 2), (2, 1, 1), (1, 1, 2), (4, 3, 3)])
def test_wm_shift_table_definition(B, Bp, bs):
    rng = np.random.default_rng(400 + B)
    P = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, (30, 7))]
    wm = oracle.WM(P, B=B, Bp=Bp, bitshift=bs)
    m = P.shape[1]
    size = sum(256 * (2 ** bs) ** i for i in range(B))
    assert wm.tsize == size
    # SHIFT[h]: distance from the rightmost block with hash h to the end of
    # any pattern; m - B + 1 if no block hashes to h.
    best = {}
    for p in P:
        for q in range(B, m + 1):
            h = shift_add(bytes(p[q - B:q]), bs)
            best[h] = min(best.get(h, m - B + 1), m - q)
    table = wm.shift_table()
    for h in range(size):
        assert table[h] == best.get(h, m - B + 1), h
    # HASH[h]: ascending ids whose B-suffix hashes to h; PREFIX[r] = h2(prefix)
    for h in {shift_add(bytes(p[m - B:]), bs) for p in P}:
        want = [r for r in range(len(P)) if shift_add(bytes(P[r, m - B:]), bs) == h]
        assert wm.hash_list(h) == want
    for r in range(len(P)):
        assert wm.prefix(r) == shift_add(bytes(P[r, :Bp]), bs)


def test_wm_paper_table_size():
    # B = 3, bitshift = 2 over byte values: 256 * (1 + 4 + 16) entries, which
    # also bounds the largest hash 255 * 21.
    assert oracle.lib().orc_wm_table_size(3, 2) == 5376
    assert shift_add(b"\xff\xff\xff", 2) == 5355


def test_wm_rejects_short_patterns():
    with pytest.raises(ValueError):
        oracle.WM([b"AC"], B=3, Bp=2)


# ---------------------------------------------------------------------------
# Exhaustive and random agreement of the four oracles
# ---------------------------------------------------------------------------

def all_agree(T, P, wm_params=((3, 2, 2),)):
    want = pairs(oracle.bf(T, P))
    assert pairs(oracle.Win(P).scan(T)) == want
    assert pairs(oracle.AC(P).scan(T)) == want
    m = P.shape[1]
    for B, Bp, bs in wm_params:
        B, Bp = min(B, m), min(Bp, m)
        assert pairs(oracle.WM(P, B=B, Bp=Bp, bitshift=bs).scan(T)) == want, (B, Bp, bs)
    return want


def test_exhaustive_tiny_binary():
    # every text over {A,C} up to length 8 against a few pattern sets
    sets = [[b"A"], [b"AC", b"CA", b"AC"], [b"AAA", b"ACA", b"CCC", b"AAA"],
            [b"ACAC", b"CACA"], [b"AAAAA"]]
    for P in sets:
        Pa = np.frombuffer(b"".join(P), np.uint8).reshape(len(P), len(P[0]))
        for n in range(0, 9):
            for t in itertools.product(b"AC", repeat=n):
                all_agree(np.array(t, np.uint8), Pa, wm_params=((3, 2, 2), (1, 1, 1), (2, 2, 8)))


@pytest.mark.parametrize("seed", range(60))
def test_random_agreement(seed):
    rng = np.random.default_rng(500 + seed)
    T, P = rand_case(rng, alphabet=b"ACGTN\n" if seed % 3 == 0 else b"ACGT",
                     n_max=400, d_max=12, m_max=9)
    all_agree(T, P, wm_params=((3, 2, 2), (2, 1, 2), (1, 1, 0)))


def test_worst_case_all_same_character():
    # Section 3.2 worst case: text and m-1 characters of every pattern are the
    # same repeated character.
    T = np.full(300, ord("A"), np.uint8)
    P = np.full((6, 8), ord("A"), np.uint8)
    P[1:, 3] = np.frombuffer(b"CGTNX", np.uint8)
    want = all_agree(T, P)
    assert want == [(i, 0) for i in range(300 - 8 + 1)]


def test_newline_dense_text_and_duplicates():
    rng = np.random.default_rng(7)
    T = np.frombuffer(b"ACGT\n", np.uint8)[rng.integers(0, 5, 2000)]
    P = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, (40, 3))]
    P[10:20] = P[0]
    all_agree(T, P)


# ---------------------------------------------------------------------------
# Contiguous split with an m-1 overlap (Section 4.4) and ownership rule
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("parts", [1, 2, 3, 7, 64])
def test_split_concatenation_equals_whole(parts):
    text, ps = synth.workload_small()
    T = text[:40000]
    P = ps.patterns
    whole = oracle.Win(P).scan(T)
    for obj in (oracle.Win(P), oracle.AC(P), oracle.WM(P)):
        got = oracle.parallel_scan(obj, T, parts=parts, workers=4)
        assert np.array_equal(got[0], whole[0]) and np.array_equal(got[1], whole[1])
    n, m = len(T), P.shape[1]
    # the paper's equation: rank r reads [r n/P, (r+1) n/P + m - 1)
    acc = []
    for r in range(parts):
        start, stop = r * n // parts, (r + 1) * n // parts
        acc.append(oracle.AC(P).scan(T, start, stop))
    cat = (np.concatenate([a[0] for a in acc]), np.concatenate([a[1] for a in acc]))
    assert np.array_equal(cat[0], whole[0]) and np.array_equal(cat[1], whole[1])


# ---------------------------------------------------------------------------
# Generator sanity (not parity): planted patterns occur where recorded
# ---------------------------------------------------------------------------

def test_planted_patterns_occur():
    text, ps = synth.workload_small()
    assert len(text) == 1 << 20 and ps.patterns.shape == (100, 8)
    assert set(np.unique(text).tolist()) <= set(b"ACGT")
    pos, ids = oracle.Win(ps.patterns).scan(text)
    found = set(zip(pos.tolist(), ids.tolist()))
    for r, s in enumerate(ps.planted_starts.tolist()):
        assert (s, r) in found
    # a random 8-mer on i.i.d. uniform text: (n-m+1)/4^m ~ 16 hits on average
    rnd = np.bincount(ids, minlength=100)[50:]
    assert 8 < rnd.mean() < 24


def test_est_text_shape():
    t = synth.est_text(1 << 20, seed=2)
    vals, cnt = np.unique(t, return_counts=True)
    freq = dict(zip(bytes(vals), cnt / len(t)))
    assert set(freq) <= set(b"ACGTN\n")
    assert 0.006 < freq[ord("N")] < 0.014
    nl = np.nonzero(t == 10)[0]
    lens = np.diff(np.concatenate([[-1], nl])) - 1
    assert 440 < lens.mean() < 560
    # same seed, same bytes
    assert np.array_equal(t, synth.est_text(1 << 20, seed=2))


# ---------------------------------------------------------------------------
# Pattern sets of different lengths (the Definition with a length per pattern)
# ---------------------------------------------------------------------------

def mixed_agree(T, P, wm_params=((3, 2, 2),)):
    """bf, Win, AC and WM (for each usable (B, B', bitshift)) give one list."""
    want = pairs(oracle.bf(T, P))
    assert pairs(oracle.Win(P).scan(T)) == want
    assert pairs(oracle.AC(P).scan(T)) == want
    short = min(len(p) for p in P)
    for B, Bp, bs in wm_params:
        B, Bp = min(B, short), min(Bp, short)
        assert pairs(oracle.WM(P, B=B, Bp=Bp, bitshift=bs).scan(T)) == want, (B, Bp, bs)
    return want


def rand_mixed(rng, alphabet=b"AC", n_max=40, d_max=6, len_max=5):
    A = np.frombuffer(alphabet, np.uint8)
    n = int(rng.integers(0, n_max + 1))
    T = A[rng.integers(0, len(A), n)] if n else np.zeros(0, np.uint8)
    d = int(rng.integers(1, d_max + 1))
    P = [bytes(A[rng.integers(0, len(A), int(rng.integers(1, len_max + 1)))]) for _ in range(d)]
    if d > 1 and rng.random() < 0.4:
        P[-1] = P[0]                       # a duplicate
    if d > 1 and rng.random() < 0.5 and len(P[0]) > 1:
        P[1] = P[0][: int(rng.integers(1, len(P[0])))]   # a prefix of another
    if d > 2 and rng.random() < 0.5 and len(P[0]) > 1:
        P[2] = P[0][int(rng.integers(1, len(P[0]))):]    # a suffix of another
    if n and rng.random() < 0.7:
        L = len(P[0])
        if n >= L:
            s = int(rng.integers(0, n - L + 1))
            P[0] = bytes(T[s:s + L])
    return T.astype(np.uint8), P


def test_mixed_hand_fixture():
    with open(os.path.join(GOLDEN, "mixed_hand_example.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        T = np.frombuffer(case["text"].encode(), np.uint8)
        P = [p.encode() for p in case["patterns"]]
        want = [tuple(x) for x in case["pairs"]]
        assert mixed_agree(T, P, wm_params=((1, 1, 2), (2, 1, 1))) == want


@pytest.mark.parametrize("seed", range(10))
def test_mixed_bf_matches_regex_per_pattern(seed):
    rng = np.random.default_rng(700 + seed)
    T, P = rand_mixed(rng, alphabet=b"ACG", n_max=300, d_max=8, len_max=6)
    Tb = bytes(T)
    want = []
    for r, p in enumerate(P):
        want += [(mt.start(), r) for mt in re.finditer(b"(?=" + re.escape(p) + b")", Tb)]
    assert pairs(oracle.bf(T, P)) == sorted(want)


def test_mixed_exhaustive_tiny():
    sets = [[b"A", b"AA", b"AAA"], [b"AC", b"C", b"CAC", b"C"], [b"CA", b"ACA", b"A", b"CCA"],
            [b"AAC", b"A", b"AACA", b"AC"]]
    for P in sets:
        for n in range(0, 8):
            for t in itertools.product(b"AC", repeat=n):
                mixed_agree(np.array(t, np.uint8), P, wm_params=((3, 2, 2), (1, 1, 1), (2, 2, 8)))


@pytest.mark.parametrize("seed", range(40))
def test_mixed_random_agreement(seed):
    rng = np.random.default_rng(800 + seed)
    T, P = rand_mixed(rng, alphabet=b"ACGTN\n" if seed % 3 == 0 else b"ACGT", n_max=400,
                      d_max=12, len_max=9)
    mixed_agree(T, P, wm_params=((3, 2, 2), (2, 1, 2), (1, 1, 0)))


@pytest.mark.parametrize("seed", range(8))
def test_ac_merged_output_is_every_pattern_suffix(seed):
    """The merged output set of a state holds exactly the patterns that are
    suffixes of the state's label (Section 3.1: a state reports a pattern
    when it ends there; with several lengths a pattern can end inside a
    longer path)."""
    rng = np.random.default_rng(900 + seed)
    _, P = rand_mixed(rng, alphabet=b"ACG", n_max=0, d_max=10, len_max=6)
    ac = oracle.AC(P)
    labels = state_labels(ac)
    assert len(labels) == ac.nstates
    for q, lab in labels.items():
        want = [r for r, p in enumerate(P) if lab.endswith(p)]
        assert ac.output_all(q) == want, (lab, want)
        assert ac.output(q) == [r for r, p in enumerate(P) if lab == p]


def test_mixed_wm_shift_uses_the_shortest_length():
    """SHIFT over blocks of every pattern's first w characters, w the
    shortest length (Section 3.2 with m read as the shortest length); HASH
    keyed on the block ending those w characters."""
    rng = np.random.default_rng(31)
    A = np.frombuffer(b"ACGT", np.uint8)
    P = [bytes(A[rng.integers(0, 4, int(L))]) for L in rng.integers(4, 10, 25)]
    B, Bp, bs = 3, 2, 2
    wm = oracle.WM(P, B=B, Bp=Bp, bitshift=bs)
    w = min(len(p) for p in P)
    best = {}
    for p in P:
        for q in range(B, w + 1):
            h = shift_add(p[q - B:q], bs)
            best[h] = min(best.get(h, w - B + 1), w - q)
    table = wm.shift_table()
    for h in range(wm.tsize):
        assert table[h] == best.get(h, w - B + 1), h
    for h in {shift_add(p[w - B:w], bs) for p in P}:
        assert wm.hash_list(h) == [r for r, p in enumerate(P) if shift_add(p[w - B:w], bs) == h]


def test_equal_lengths_as_list_equal_array_form():
    text, ps = synth.workload_small()
    T = text[:50000]
    P = ps.patterns
    as_list = [bytes(p) for p in P]
    for cls in (oracle.Win, oracle.AC, oracle.WM):
        a, b = cls(P).scan(T), cls(as_list).scan(T)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("parts", [1, 3, 17])
def test_mixed_split_concatenation_equals_whole(parts):
    """Contiguous ranges of starting positions, each reading up to (longest
    length - 1) characters past its end (Section 4.4's split), concatenate to
    the whole list."""
    rng = np.random.default_rng(41)
    T = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, 20000)]
    P = [bytes(T[s:s + L]) for s, L in zip(rng.integers(0, 19000, 30), rng.integers(2, 12, 30))]
    P += [p[:3] for p in P[:5]] + [p[-2:] for p in P[5:10]]
    whole = oracle.bf(T, P)
    for obj in (oracle.Win(P), oracle.AC(P), oracle.WM(P, B=2, Bp=2)):
        got = oracle.parallel_scan(obj, T, parts=parts, workers=4)
        assert np.array_equal(got[0], whole[0]) and np.array_equal(got[1], whole[1])
