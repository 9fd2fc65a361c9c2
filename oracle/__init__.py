"""CPU oracle for exact multiple pattern matching (Python side).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg. The product library never imports, links or
calls anything here, and nothing here imports the product package.

``oracle.c`` holds the four C implementations (brute force over the
definition of Section 1, sorted-window lookup, Aho-Corasick per Algorithms 1-3,
Wu-Manber per Algorithms 4-5). This module compiles it with gcc, loads it with
ctypes and adds numpy conveniences. ``mlp.py`` holds the FP64 reference of the
variant-selector network.

Pattern sets are a ``uint8 [d, m]`` array (equal lengths, as in the paper) or
a list of byte strings, which may differ in length.

All scans return ``(pos, id)`` as two uint32 arrays in ascending (pos, id)
order. Range scans cover start positions ``[lo, hi)``; ``parallel_scan`` splits
a text into contiguous ranges (the paper's split, Section 4.4) and concatenates
the per-range results in range order.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

u8p = C.POINTER(C.c_uint8)
u32p = C.POINTER(C.c_uint32)
i32p = C.POINTER(C.c_int32)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (plain gcc, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            u64, u32, vp = C.c_uint64, C.c_uint32, C.c_void_p
            u64p = C.POINTER(C.c_uint64)
            L.orc_bf.restype = u64
            L.orc_bf.argtypes = [u8p, u64, u8p, u32, u32, u64, u64, u32p, u32p, u64]
            L.orc_bf_v.restype = u64
            L.orc_bf_v.argtypes = [u8p, u64, u8p, u64p, u32, u64, u64, u32p, u32p, u64]
            L.orc_win_build.restype = vp
            L.orc_win_build.argtypes = [u8p, u32, u32]
            L.orc_win_build_v.restype = vp
            L.orc_win_build_v.argtypes = [u8p, u64p, u32]
            L.orc_ac_build_v.restype = vp
            L.orc_ac_build_v.argtypes = [u8p, u64p, u32]
            L.orc_wm_build_v.restype = vp
            L.orc_wm_build_v.argtypes = [u8p, u64p, u32, u32, u32, u32]
            L.orc_ac_nout_all.restype = u32
            L.orc_ac_nout_all.argtypes = [vp, u64]
            L.orc_ac_out_all.restype = u32
            L.orc_ac_out_all.argtypes = [vp, u64, u32]
            L.orc_win_free.argtypes = [vp]
            L.orc_win_scan.restype = u64
            L.orc_win_scan.argtypes = [vp, u8p, u64, u64, u64, u32p, u32p, u64]
            L.orc_ac_build.restype = vp
            L.orc_ac_build.argtypes = [u8p, u32, u32]
            L.orc_ac_free.argtypes = [vp]
            L.orc_ac_nstates.restype = u64
            L.orc_ac_nstates.argtypes = [vp]
            L.orc_ac_goto.restype = C.c_int32
            L.orc_ac_goto.argtypes = [vp, u64, u32]
            L.orc_ac_supply.restype = C.c_int32
            L.orc_ac_supply.argtypes = [vp, u64]
            L.orc_ac_depth.restype = u32
            L.orc_ac_depth.argtypes = [vp, u64]
            L.orc_ac_nout.restype = u32
            L.orc_ac_nout.argtypes = [vp, u64]
            L.orc_ac_out.restype = u32
            L.orc_ac_out.argtypes = [vp, u64, u32]
            L.orc_ac_scan.restype = u64
            L.orc_ac_scan.argtypes = [vp, u8p, u64, u64, u64, u32p, u32p, u64]
            L.orc_ac_trace.argtypes = [vp, u8p, u64, u64, i32p]
            L.orc_wm_table_size.restype = u64
            L.orc_wm_table_size.argtypes = [u32, u32]
            L.orc_wm_build.restype = vp
            L.orc_wm_build.argtypes = [u8p, u32, u32, u32, u32, u32]
            L.orc_wm_free.argtypes = [vp]
            L.orc_wm_tsize.restype = u64
            L.orc_wm_tsize.argtypes = [vp]
            L.orc_wm_shift.restype = u32
            L.orc_wm_shift.argtypes = [vp, u64]
            L.orc_wm_nhash.restype = u32
            L.orc_wm_nhash.argtypes = [vp, u64]
            L.orc_wm_hash_entry.restype = u32
            L.orc_wm_hash_entry.argtypes = [vp, u64, u32]
            L.orc_wm_prefix.restype = u64
            L.orc_wm_prefix.argtypes = [vp, u32]
            L.orc_wm_scan.restype = u64
            L.orc_wm_scan.argtypes = [vp, u8p, u64, u64, u64, u32p, u32p, u64]
            _lib = L
    return _lib


def _u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray)):
        a = np.frombuffer(bytes(a), dtype=np.uint8)
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a


def _ptr(a: np.ndarray, t=u8p):
    return a.ctypes.data_as(t)


class PatternSet:
    """d patterns as one byte array and offsets: pattern r is
    bytes[off[r]:off[r + 1]]. m is the common length, or None when lengths
    differ."""

    def __init__(self, P):
        if isinstance(P, PatternSet):
            self.__dict__.update(P.__dict__)
            return
        if isinstance(P, (list, tuple)):
            pats = [bytes(p) for p in P]
            assert all(len(p) > 0 for p in pats), "patterns must be non-empty"
            self.bytes = np.frombuffer(b"".join(pats) or b"\0", np.uint8)
            self.lengths = np.array([len(p) for p in pats], np.uint64)
        else:
            A = np.ascontiguousarray(P, dtype=np.uint8)
            assert A.ndim == 2
            self.bytes = A.reshape(-1) if A.size else np.zeros(1, np.uint8)
            self.lengths = np.full(A.shape[0], A.shape[1], np.uint64)
        self.d = len(self.lengths)
        self.off = np.zeros(self.d + 1, np.uint64)
        self.off[1:] = np.cumsum(self.lengths)
        lens = set(self.lengths.tolist())
        self.m = int(next(iter(lens))) if len(lens) == 1 else None
        self.shortest = int(self.lengths.min()) if self.d else 0
        self.longest = int(self.lengths.max()) if self.d else 0

    def pattern(self, r: int) -> bytes:
        return self.bytes[int(self.off[r]):int(self.off[r + 1])].tobytes()

    def args(self):
        return _ptr(self.bytes), self.off.ctypes.data_as(C.POINTER(C.c_uint64)), self.d


def _run(fn, cap_guess: int):
    """Call fn(pos, id, cap) -> count, growing the buffers once if needed."""
    cap = max(16, int(cap_guess))
    pos = np.empty(cap, np.uint32)
    ids = np.empty(cap, np.uint32)
    cnt = fn(pos, ids, cap)
    if cnt > cap:
        pos = np.empty(cnt, np.uint32)
        ids = np.empty(cnt, np.uint32)
        cnt2 = fn(pos, ids, cnt)
        assert cnt2 == cnt
    return pos[:cnt].copy(), ids[:cnt].copy()


def _cap_guess(lo, hi, n):
    span = max(0, min(hi, n) - lo)
    return span // 64 + 1024


def bf(text, P, lo: int = 0, hi: int | None = None):
    """Brute force over the definition (Section 1). Small inputs only."""
    L = lib()
    T = _u8(text)
    ps = PatternSet(P)
    n = len(T)
    hi = n if hi is None else hi
    Tp = T if n else np.zeros(1, np.uint8)
    return _run(lambda p, i, c: L.orc_bf_v(_ptr(Tp), n, *ps.args(), lo, hi,
                                           _ptr(p, u32p), _ptr(i, u32p), c),
                _cap_guess(lo, hi, n))


class _Handle:
    _free = None

    def __init__(self, h, keep):
        self.h = h
        self._keep = keep

    def close(self):
        if self.h:
            type(self)._free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Win(_Handle):
    """Sorted-window lookup: the definition at scale."""

    def __init__(self, P):
        L = lib()
        ps = PatternSet(P)
        self.ps, self.d, self.m = ps, ps.d, ps.m
        type(self)._free = L.orc_win_free
        super().__init__(L.orc_win_build_v(*ps.args()), ps)

    def scan(self, text, lo: int = 0, hi: int | None = None):
        L = lib()
        T = _u8(text)
        n = len(T)
        hi = n if hi is None else hi
        Tp = T if n else np.zeros(1, np.uint8)
        return _run(lambda p, i, c: L.orc_win_scan(self.h, _ptr(Tp), n, lo, hi,
                                                   _ptr(p, u32p), _ptr(i, u32p), c),
                    _cap_guess(lo, hi, n))


class AC(_Handle):
    """Aho-Corasick per Algorithms 1-3 (goto over 256 byte values)."""

    def __init__(self, P):
        L = lib()
        ps = PatternSet(P)
        self.ps, self.d, self.m = ps, ps.d, ps.m
        type(self)._free = L.orc_ac_free
        super().__init__(L.orc_ac_build_v(*ps.args()), ps)

    @property
    def nstates(self) -> int:
        return int(lib().orc_ac_nstates(self.h))

    def goto(self, q: int, c) -> int:
        return int(lib().orc_ac_goto(self.h, q, c if isinstance(c, int) else ord(c)))

    def supply(self, q: int) -> int:
        return int(lib().orc_ac_supply(self.h, q))

    def depth(self, q: int) -> int:
        return int(lib().orc_ac_depth(self.h, q))

    def output(self, q: int) -> list[int]:
        """Patterns whose own path ends at state q (Algorithm 1)."""
        L = lib()
        return [int(L.orc_ac_out(self.h, q, k)) for k in range(L.orc_ac_nout(self.h, q))]

    def output_all(self, q: int) -> list[int]:
        """The merged output set of q: every pattern that is a suffix of the
        state's label (its own patterns and those of its supply chain)."""
        L = lib()
        return [int(L.orc_ac_out_all(self.h, q, k)) for k in range(L.orc_ac_nout_all(self.h, q))]

    def trace(self, text, lo: int = 0, hi: int | None = None) -> np.ndarray:
        T = _u8(text)
        hi = len(T) if hi is None else hi
        out = np.empty(max(0, hi - lo), np.int32)
        if hi > lo:
            lib().orc_ac_trace(self.h, _ptr(T), lo, hi, _ptr(out, i32p))
        return out

    def scan(self, text, lo: int = 0, hi: int | None = None):
        L = lib()
        T = _u8(text)
        n = len(T)
        hi = n if hi is None else hi
        Tp = T if n else np.zeros(1, np.uint8)
        return _run(lambda p, i, c: L.orc_ac_scan(self.h, _ptr(Tp), n, lo, hi,
                                                  _ptr(p, u32p), _ptr(i, u32p), c),
                    _cap_guess(lo, hi, n))


class WM(_Handle):
    """Wu-Manber per Algorithms 4-5 (shift-and-add hash over byte values)."""

    def __init__(self, P, B: int = 3, Bp: int = 2, bitshift: int = 2):
        L = lib()
        ps = PatternSet(P)
        self.ps, self.d, self.m = ps, ps.d, ps.m
        self.B, self.Bp, self.bitshift = B, Bp, bitshift
        h = L.orc_wm_build_v(*ps.args(), B, Bp, bitshift)
        if not h:
            raise ValueError(f"Wu-Manber needs every pattern at least B and B' long "
                             f"(shortest {ps.shortest}, B={B}, B'={Bp})")
        type(self)._free = L.orc_wm_free
        super().__init__(h, ps)

    @property
    def tsize(self) -> int:
        return int(lib().orc_wm_tsize(self.h))

    def shift_table(self) -> np.ndarray:
        L = lib()
        return np.array([L.orc_wm_shift(self.h, t) for t in range(self.tsize)], np.int64)

    def hash_list(self, t: int) -> list[int]:
        L = lib()
        return [int(L.orc_wm_hash_entry(self.h, t, k)) for k in range(L.orc_wm_nhash(self.h, t))]

    def prefix(self, r: int) -> int:
        return int(lib().orc_wm_prefix(self.h, r))

    def scan(self, text, lo: int = 0, hi: int | None = None):
        L = lib()
        T = _u8(text)
        n = len(T)
        hi = n if hi is None else hi
        Tp = T if n else np.zeros(1, np.uint8)
        return _run(lambda p, i, c: L.orc_wm_scan(self.h, _ptr(Tp), n, lo, hi,
                                                  _ptr(p, u32p), _ptr(i, u32p), c),
                    _cap_guess(lo, hi, n))


def parallel_scan(obj, text, lo: int = 0, hi: int | None = None, workers: int | None = None,
                  parts: int | None = None):
    """Scan [lo, hi) as contiguous ranges on a thread pool (ctypes drops the
    GIL) and concatenate in range order. Each range reads up to (longest
    pattern length - 1) characters past its end, as in the paper's split
    (Section 4.4)."""
    T = _u8(text)
    n = len(T)
    hi = n if hi is None else min(hi, n)
    workers = workers or min(16, os.cpu_count() or 1)
    parts = parts or workers * 4
    if hi <= lo:
        return np.empty(0, np.uint32), np.empty(0, np.uint32)
    bounds = np.linspace(lo, hi, parts + 1).astype(np.int64)
    with ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(lambda k: obj.scan(T, int(bounds[k]), int(bounds[k + 1])), range(parts)))
    return (np.concatenate([r[0] for r in res]), np.concatenate([r[1] for r in res]))


def ids_per_position_ok(pos: np.ndarray, ids: np.ndarray) -> bool:
    """True if the pairs are in strictly ascending (pos, id) order."""
    if len(pos) < 2:
        return True
    key = (pos.astype(np.uint64) << np.uint64(32)) | ids.astype(np.uint64)
    return bool(np.all(key[1:] > key[:-1]))
