"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host-side builders produce tables whose behaviour matches the oracle
(simulated on the CPU from the exported tables; no GPU involved)."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_1407_2889_amd as mpm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "mpm.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    syms = declared_symbols()
    assert "mpm_build_ac" in syms and "mpm_scan" in syms and "mpm_free" in syms
    lib = C.CDLL(mpm.LIB_PATH)
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(mpm.EXPORTS)
    assert mpm._L.mpm_version().startswith(b"mpm")


def test_error_codes():
    P = np.frombuffer(b"ACGTACGT", np.uint8).reshape(2, 4)
    h = C.c_void_p()
    assert mpm._L.mpm_build_ac(P.ctypes.data, 0, 4, None, C.byref(h)) == mpm.MPM_EINVAL
    assert b"d must be positive" in mpm._L.mpm_last_error()
    assert mpm._L.mpm_build_ac(P.ctypes.data, 2, 0, None, C.byref(h)) == mpm.MPM_EINVAL
    assert mpm._L.mpm_build_ac(None, 2, 4, None, C.byref(h)) == mpm.MPM_EINVAL
    assert mpm._L.mpm_build_wm(P.ctypes.data, 2, 4, None, None) == mpm.MPM_EINVAL
    o = mpm.Opts()
    o.wm_block = 5
    assert mpm._L.mpm_build_wm(P.ctypes.data, 2, 4, C.byref(o), C.byref(h)) == mpm.MPM_EUNSUPPORTED
    o.wm_block = 9
    P9 = np.zeros((1, 12), np.uint8)
    assert mpm._L.mpm_build_wm(P9.ctypes.data, 1, 12, C.byref(o), C.byref(h)) == mpm.MPM_EUNSUPPORTED
    mpm._L.mpm_free(None)  # NULL-safe
    # scanning an index that was never uploaded
    ix = mpm.build_ac(P)
    tot = C.c_uint64()
    st = mpm._L.mpm_scan_sync(ix.handle, C.c_void_p(16), 8, None, 0, C.c_void_p(64), 1 << 20,
                              C.c_void_p(8), None, None, C.byref(tot))
    assert st == mpm.MPM_ESTATE
    # host-streamed scan and per-pattern counts: argument checks, no device work
    def scan_host(n, chunk):
        return mpm._L.mpm_scan_host(ix.handle, C.c_void_p(16), n, C.c_void_p(64), 1 << 20, chunk,
                                    None, 0, C.c_void_p(64), 1 << 20, C.c_void_p(8), None, None,
                                    C.byref(tot))
    assert scan_host(100, 0) == mpm.MPM_EINVAL
    assert scan_host(1 << 32, 1024) == mpm.MPM_ETOOBIG
    assert scan_host(3, 1024) == mpm.MPM_ESTATE  # n < m: a scan of nothing, index not uploaded
    assert mpm._L.mpm_count_ids(None, 0, 0, C.c_void_p(64), None) == mpm.MPM_EINVAL
    assert mpm._L.mpm_count_ids(C.c_void_p(4), 1, 10, C.c_void_p(64), None) == mpm.MPM_EINVAL
    assert mpm._L.mpm_count_ids(None, 5, 10, C.c_void_p(64), None) == mpm.MPM_EINVAL
    with pytest.raises(mpm.MpmError):
        mpm.workspace_bytes(ix, 100, mpm.variant(lane_bytes=24))
    with pytest.raises(mpm.MpmError):
        mpm.workspace_bytes(ix, 100, mpm.variant(block_threads=128))


def simulate_dfa(table, classes, m, du, text):
    """Walk the exported dense table on the CPU: column 0 for bytes in no
    pattern, column k for the k-th smallest pattern byte."""
    col = np.zeros(256, np.int64)
    for k, b in enumerate(classes):
        col[b] = k + 1
    S = table.shape[0]
    first = S - du
    s = 0
    hits = []
    for i, b in enumerate(np.asarray(text, np.uint8)):
        s = int(table[s, col[b]])
        if s >= first:
            hits.append((i - m + 1, s - first))
    return hits


def expand(hits, uoff, ids):
    out = []
    for pos, u in hits:
        for j in range(uoff[u], uoff[u + 1]):
            out.append((pos, int(ids[j])))
    return out


@pytest.mark.parametrize("seed", range(25))
def test_ac_table_walk_equals_oracle(seed):
    rng = np.random.default_rng(seed)
    alpha = np.frombuffer(b"ACGTN\n" if seed % 2 else b"ACGT", np.uint8)
    m = int(rng.integers(1, 9))
    d = int(rng.integers(1, 40))
    T = alpha[rng.integers(0, len(alpha), 3000)]
    P = alpha[rng.integers(0, len(alpha), (d, m))]
    if d > 3:
        P[1] = P[0]
        P[2] = T[10:10 + m]
    ix = mpm.build_ac(P)
    inf = ix.info()
    table, classes = ix.export_ac()
    uoff, ids = ix.export_unique()
    assert inf["d_unique"] == len({bytes(p) for p in P})
    assert list(classes) == sorted(set(P.flatten().tolist()))
    # column 0 always returns to the root; terminals are the last block
    assert (table[:, 0] == 0).all()
    assert inf["n_states"] == table.shape[0]
    got = expand(simulate_dfa(table, classes, m, inf["d_unique"], T), uoff, ids)
    pos, idv = oracle.Win(P).scan(T)
    assert got == list(zip(pos.tolist(), idv.tolist()))


@pytest.mark.parametrize("n_bytes", [255, 256])
def test_ac_over_every_byte_value(n_bytes):
    """Patterns that use all 256 byte values (256 symbol classes, 257 table
    columns) build, and the exported table walks to the oracle's list."""
    rng = np.random.default_rng(n_bytes)
    vals = rng.permutation(256)[:n_bytes].astype(np.uint8)
    P = vals[: (n_bytes // 8) * 8].reshape(-1, 8).copy()
    P = np.concatenate([P, vals[rng.integers(0, n_bytes, (20, 8))]])
    T = vals[rng.integers(0, n_bytes, 20000)].astype(np.uint8)
    for k in range(0, 20000 - 8, 997):  # plant occurrences
        T[k:k + 8] = P[k % len(P)]
    ix = mpm.build_ac(P)
    inf = ix.info()
    assert inf["n_classes"] == len(set(P.flatten().tolist()))
    table, classes = ix.export_ac()
    assert table.shape[1] == inf["n_classes"] + 1
    uoff, ids = ix.export_unique()
    got = expand(simulate_dfa(table, classes, 8, inf["d_unique"], T), uoff, ids)
    pos, idv = oracle.Win(P).scan(T)
    assert len(pos) > 0
    assert got == list(zip(pos.tolist(), idv.tolist()))


def test_count_guards():
    """Counts the kernels could not hold are refused on the host: a wave's
    32-bit prefix (64 lanes x lane_bytes x copies of one pattern) and a text's
    36-bit count (starting positions x copies)."""
    P = np.zeros((70000, 4), np.uint8)  # one string, 70,000 ids
    ix = mpm.build_ac(P)
    assert ix.info()["max_dup"] == 70000
    tot = C.c_uint64()

    def scan(n, lane_bytes):
        v = mpm.variant(lane_bytes=lane_bytes, block_threads=256)
        ws = mpm.workspace_bytes(ix, n, v)
        return mpm._L.mpm_scan_sync(ix.handle, C.c_void_p(4096), n, None, 0, C.c_void_p(4096),
                                    ws, C.c_void_p(8), C.byref(v), None, C.byref(tot))
    # 64 * 1024 * 70,000 >= 2^32: a wave's prefix would overflow
    assert scan(1 << 20, 1024) == mpm.MPM_EUNSUPPORTED
    assert b"32-bit" in mpm._L.mpm_last_error()
    # (2^20 - 3) * 70,000 >= 2^36: the text's count would overflow
    assert scan(1 << 20, 16) == mpm.MPM_ETOOBIG
    # within both bounds the request goes on (and stops at the missing upload)
    assert scan(1 << 19, 16) == mpm.MPM_ESTATE


def test_ac_state_count_matches_oracle_trie():
    rng = np.random.default_rng(3)
    P = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, (300, 8))]
    ix = mpm.build_ac(P)
    assert ix.info()["n_states"] == oracle.AC(P).nstates
    assert ix.info()["state_bytes"] == 2


def test_unique_csr():
    P = np.frombuffer(b"CCAAGGAACC", np.uint8).reshape(5, 2)   # CC AA GG AA CC
    ix = mpm.build_ac(P)
    uoff, ids = ix.export_unique()
    # strings with one id first, then repeated ones, each in string order:
    # GG:{2} AA:{1,3} CC:{0,4}
    assert uoff.tolist() == [0, 1, 3, 5]
    assert ids.tolist() == [2, 1, 3, 0, 4]
    assert ix.info()["max_dup"] == 2
    # groups by id count, each in string order: GG:{3}, then CC:{1,5} TT:{2,7},
    # then AA:{0,4,6}
    P = np.frombuffer(b"AACCTTGGAACCAATT", np.uint8).reshape(8, 2)
    for build in (mpm.build_ac, mpm.build_wm):
        uoff, ids = build(P).export_unique()
        assert uoff.tolist() == [0, 1, 3, 5, 8]
        assert ids.tolist() == [3, 1, 5, 2, 7, 0, 4, 6]


def wm_hash2(block, sh):
    h = 0
    for k, c in enumerate(block):
        h |= ((c >> sh) & 3) << (2 * k)
    return h


@pytest.mark.parametrize("B", [0, 1, 2, 3, 5, 8])
def test_wm_shift_table_definition(B):
    rng = np.random.default_rng(B + 10)
    m = 12
    P = np.frombuffer(b"ACGTN", np.uint8)[rng.integers(0, 5, (60, m))]
    ix = mpm.build_wm(P, B=B)
    inf = ix.info()
    B = inf["wm_block"]
    sh = inf["wm_code_shift"]
    table = ix.export_wm_shift()
    assert table.size == 4 ** B
    best = {}
    for p in P:
        for q in range(B, m + 1):
            h = wm_hash2(bytes(p[q - B:q]), sh)
            best[h] = min(best.get(h, m - B + 1), m - q)
    for h in range(4 ** B):
        assert table[h] == best.get(h, m - B + 1)
    assert inf["wm_zero_shift"] == int((table == 0).sum())


def test_wm_code_shift_separates_dna():
    P = np.frombuffer(b"ACGTACGTACGTGGCC", np.uint8).reshape(2, 8)
    inf = mpm.build_wm(P).info()
    codes = {(c >> inf["wm_code_shift"]) & 3 for c in b"ACGT"}
    assert len(codes) == 4


def test_wm_auto_block_prefers_long_blocks_for_sparse_sets():
    rng = np.random.default_rng(0)
    P = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, (1000, 16))]
    inf = mpm.build_wm(P).info()
    assert inf["wm_block"] >= 6
    assert inf["wm_mean_shift"] > 5


def test_placement_resolution():
    """Tables larger than LDS: whole-LDS placement is refused, the hot part in
    LDS (or all of it global) is accepted, automatic placement picks one of
    them, and the two-chain variant has no hot placement. Host-only."""
    rng = np.random.default_rng(21)
    P = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, (3000, 20))]
    for build in (mpm.build_ac, mpm.build_wm):
        ix = build(P)
        assert ix.info()["table_bytes"] > 160 * 1024
        with pytest.raises(mpm.MpmError) as e:
            mpm.workspace_bytes(ix, 1 << 20, mpm.variant(64, 256, mpm.PLACE_LDS))
        assert e.value.status == mpm.MPM_EUNSUPPORTED
        for pl in (mpm.PLACE_AUTO, mpm.PLACE_GLOBAL, mpm.PLACE_HOT):
            assert mpm.workspace_bytes(ix, 1 << 20, mpm.variant(64, 256, pl)) > 0
    ix = mpm.build_ac(P)
    with pytest.raises(mpm.MpmError) as e:
        mpm.workspace_bytes(ix, 1 << 20, mpm.variant(64, 256, mpm.PLACE_HOT, 0, mpm.VARIANT_ILP2))
    assert e.value.status == mpm.MPM_EUNSUPPORTED
    with pytest.raises(mpm.MpmError) as e:
        mpm.workspace_bytes(ix, 1 << 20, mpm.variant(64, 256, 4))
    assert e.value.status == mpm.MPM_EINVAL


def test_supply_walk_variant_resolution():
    """The goto + supply-link walk needs an index that kept the goto function;
    it has one chain per lane and no hot placement; unknown flags are
    refused. Host-only."""
    rng = np.random.default_rng(23)
    P = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, (50, 8))]
    sup = mpm.VARIANT_SUPPLY
    plain, withgo = mpm.build_ac(P), mpm.build_ac(P, goto=True)
    assert withgo.info()["device_bytes"] > plain.info()["device_bytes"]
    assert withgo.info()["table_bytes"] == plain.info()["table_bytes"]
    with pytest.raises(mpm.MpmError) as e:
        mpm.workspace_bytes(plain, 1 << 20, mpm.variant(64, 256, mpm.PLACE_AUTO, 0, sup))
    assert e.value.status == mpm.MPM_EUNSUPPORTED
    for pl in (mpm.PLACE_AUTO, mpm.PLACE_LDS, mpm.PLACE_GLOBAL):
        assert mpm.workspace_bytes(withgo, 1 << 20, mpm.variant(64, 256, pl, 0, sup)) > 0
    for pl, fl in ((mpm.PLACE_HOT, sup), (mpm.PLACE_AUTO, sup | mpm.VARIANT_ILP2)):
        with pytest.raises(mpm.MpmError) as e:
            mpm.workspace_bytes(withgo, 1 << 20, mpm.variant(64, 256, pl, 0, fl))
        assert e.value.status == mpm.MPM_EUNSUPPORTED
    with pytest.raises(mpm.MpmError) as e:
        mpm.workspace_bytes(withgo, 1 << 20, mpm.variant(64, 256, 0, 0, 8))
    assert e.value.status == mpm.MPM_EINVAL


def test_text_access_variant_resolution():
    """The ladder's text-access variants: Aho-Corasick with 16-bit entries
    and one pattern length, one at a time, one chain per lane, tables in LDS
    or global memory; the staged text must fit in LDS beside the tables.
    Host-only."""
    rng = np.random.default_rng(29)
    P = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, (60, 8))]
    ac, wm = mpm.build_ac(P), mpm.build_wm(P)
    tb, tl = mpm.VARIANT_TEXT_BYTES, mpm.VARIANT_TEXT_LDS
    for fl in (tb, tl):
        for pl in (mpm.PLACE_AUTO, mpm.PLACE_LDS, mpm.PLACE_GLOBAL):
            assert mpm.workspace_bytes(ac, 1 << 20, mpm.variant(64, 256, pl, 0, fl)) > 0
    bad = [(ac, mpm.PLACE_AUTO, tb | tl), (ac, mpm.PLACE_HOT, tb), (ac, mpm.PLACE_AUTO, tl | mpm.VARIANT_ILP2),
           (wm, mpm.PLACE_AUTO, tb), (mpm.build_ac_var([b"ACG", b"ACGTT"]), mpm.PLACE_AUTO, tl),
           (ac, mpm.PLACE_AUTO, tl | mpm.VARIANT_SUPPLY)]
    for ix, pl, fl in bad:
        with pytest.raises(mpm.MpmError) as e:
            mpm.workspace_bytes(ix, 1 << 20, mpm.variant(64, 256, pl, 0, fl))
        assert e.value.status == mpm.MPM_EUNSUPPORTED, (pl, fl)
    # 4096-byte lanes of 1024 threads: 4 MiB of text cannot be staged
    with pytest.raises(mpm.MpmError) as e:
        mpm.workspace_bytes(ac, 1 << 24, mpm.variant(4096, 1024, mpm.PLACE_GLOBAL, 0, tl))
    assert e.value.status == mpm.MPM_EUNSUPPORTED
