"""Exact multiple pattern matching on MI355X: Python binding of libmpm.so.

The binding only marshals arguments: every step of a scan runs in the HIP
kernels behind the C-ABI (``include/mpm.h``). PyTorch supplies device memory
(index images, workspaces, outputs) and the current stream. There is no CPU
fallback: importing this package fails when ``libmpm.so`` is missing, and
scans need a GPU.

    import paper_1407_2889_amd as mpm
    ix = mpm.build_ac(patterns_uint8_d_by_m)         # or mpm.build_wm(...)
    ix.upload()                                       # device image on cuda
    pairs = mpm.scan(ix, text_cuda_uint8)             # int32 [M, 2]: (pos, id)
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1407_2889_amd.build` "
        "(there is no CPU fallback)")

# torch first: it ships its own HIP runtime under the same soname as the one
# libmpm.so was linked against. Loaded in this order, libmpm binds to torch's
# copy; loaded the other way round, the process holds two HIP runtimes and the
# one libmpm uses finds no device.
import torch  # noqa: E402,F401

_L = C.CDLL(LIB_PATH)

NOALLOC_SCRATCH_BYTES = 1 << 20  # MPM_NOALLOC_SCRATCH_BYTES
MPM_OK, MPM_EINVAL, MPM_EOVERFLOW, MPM_ENOMEM, MPM_EHIP, MPM_ETOOBIG, MPM_EUNSUPPORTED, MPM_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
ALGO_AC, ALGO_WM = 1, 2
PLACE_AUTO, PLACE_LDS, PLACE_GLOBAL, PLACE_HOT = 0, 1, 2, 3

_STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "EOVERFLOW", -3: "ENOMEM", -4: "EHIP",
                 -5: "ETOOBIG", -6: "EUNSUPPORTED", -7: "ESTATE"}


class MpmError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _L.mpm_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Opts(C.Structure):
    _fields_ = [("wm_block", C.c_uint32), ("ac_goto", C.c_uint32), ("reserved", C.c_uint32 * 6)]


VARIANT_NO_SWAR = 1
VARIANT_ILP2 = 2
VARIANT_SUPPLY = 4
VARIANT_DENSE = 8
VARIANT_TEXT_BYTES = 16
VARIANT_TEXT_LDS = 32


class Variant(C.Structure):
    _fields_ = [("lane_bytes", C.c_uint32), ("block_threads", C.c_uint32),
                ("placement", C.c_uint32), ("grid", C.c_uint32), ("flags", C.c_uint32)]

    def __repr__(self):
        return (f"Variant(lane_bytes={self.lane_bytes}, block_threads={self.block_threads}, "
                f"placement={self.placement}, grid={self.grid}, flags={self.flags})")

    def key(self):
        return (self.lane_bytes, self.block_threads, self.placement, self.grid, self.flags)


class Info(C.Structure):
    _fields_ = [("algo", C.c_uint32), ("m", C.c_uint32), ("d", C.c_uint32),
                ("d_unique", C.c_uint32), ("max_dup", C.c_uint32), ("n_classes", C.c_uint32),
                ("n_states", C.c_uint64), ("state_bytes", C.c_uint32), ("wm_block", C.c_uint32),
                ("wm_code_shift", C.c_uint32), ("wm_zero_shift", C.c_uint32),
                ("wm_mean_shift", C.c_double), ("table_bytes", C.c_uint64),
                ("device_bytes", C.c_uint64), ("m_max", C.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Request(C.Structure):
    _fields_ = [("idx", C.c_void_p), ("d_text", C.c_void_p), ("n", C.c_uint64),
                ("d_out", C.c_void_p), ("capacity", C.c_uint64), ("d_total", C.c_void_p),
                ("variant", Variant), ("cost_hint", C.c_float), ("d_cost", C.c_void_p)]


_vp, _u32, _u64 = C.c_void_p, C.c_uint32, C.c_uint64
_pvp = C.POINTER(C.c_void_p)


def _sig(name, res, args):
    f = getattr(_L, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("mpm_last_error", C.c_char_p, [])
_sig("mpm_version", C.c_char_p, [])
_sig("mpm_build_ac", C.c_int32, [_vp, _u32, _u32, C.POINTER(Opts), _pvp])
_sig("mpm_build_ac_var", C.c_int32, [_vp, _vp, _u32, C.POINTER(Opts), _pvp])
_sig("mpm_build_wm_var", C.c_int32, [_vp, _vp, _u32, C.POINTER(Opts), _pvp])
_sig("mpm_build_wm", C.c_int32, [_vp, _u32, _u32, C.POINTER(Opts), _pvp])
_sig("mpm_free", None, [_vp])
_sig("mpm_device_bytes", _u64, [_vp])
_sig("mpm_upload", C.c_int32, [_vp, _vp, _u64, _vp])
_sig("mpm_index_info", C.c_int32, [_vp, C.POINTER(Info)])
_sig("mpm_workspace_bytes", C.c_int32, [_vp, _u64, C.POINTER(Variant), C.POINTER(_u64)])
_sig("mpm_scan", C.c_int32, [_vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp, C.POINTER(Variant), _vp])
_sig("mpm_scan_sync", C.c_int32, [_vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp, C.POINTER(Variant),
                                  _vp, C.POINTER(_u64)])
_sig("mpm_batch_plan", C.c_int32, [C.POINTER(Request), _u32, _pvp])
_sig("mpm_batch_device_bytes", _u64, [_vp])
_sig("mpm_batch_upload", C.c_int32, [_vp, _vp, _u64, _vp])
_sig("mpm_batch_run", C.c_int32, [_vp, _vp])
_sig("mpm_batch_capture", C.c_int32, [_vp, _vp])
_sig("mpm_batch_replay", C.c_int32, [_vp, _vp])
_sig("mpm_batch_groups", _u32, [_vp])
_sig("mpm_batch_free", None, [_vp])
_sig("mpm_batch_launch_key", C.c_int32, [_vp, C.POINTER(Variant), C.POINTER(_u32)])
_sig("mpm_export_ac", C.c_int32, [_vp, _vp, _vp])
_sig("mpm_export_wm_shift", C.c_int32, [_vp, _vp])
_sig("mpm_export_unique", C.c_int32, [_vp, _vp, _vp])
_sig("mpm_read_probe", C.c_int32, [_vp, _u64, _vp, _vp])
_sig("mpm_read_probe_lanes", C.c_int32, [_vp, _u64, _u32, _vp, _vp])
_sig("mpm_count_ids", C.c_int32, [_vp, _u64, _u32, _vp, _vp])
_sig("mpm_scan_host", C.c_int32, [_vp, _vp, _u64, _vp, _u64, _u64, _vp, _u64, _vp, _u64, _vp,
                                  C.POINTER(Variant), _vp, C.POINTER(_u64)])
_sig("mpm_scan_noalloc", C.c_int32, [_vp, _vp, _u64, _vp, _u64, _vp, C.POINTER(Variant), _vp])
_sig("mpm_tune_time", C.c_int32, [_vp, _vp, _u64, _u32, C.POINTER(Variant), _vp, _u64, _vp, _vp,
                                  _u64, _u32, _vp, C.POINTER(C.c_float)])
_sig("mpm_tune_work_bytes", _u64, [_vp, _u64, _u32, C.POINTER(Variant)])
_sig("mpm_mlp_act_floats", _u64, [_u32])
_sig("mpm_mlp_forward", C.c_int32, [_vp, _vp, _u32, _vp, _vp, _vp])
_sig("mpm_mlp_loss_grad", C.c_int32, [_vp, _vp, _vp, _u32, _vp, _vp, _vp])
_sig("mpm_mlp_backward", C.c_int32, [_vp, _vp, _vp, _vp, _u32, _vp, _vp, _vp])
_sig("mpm_mlp_adam", C.c_int32, [_vp, _vp, _vp, _vp, _u32, _u32, C.c_float, C.c_float, C.c_float,
                                 C.c_float, _vp])

# Every symbol include/mpm.h declares (checked by the CPU tests).
EXPORTS = [
    "mpm_build_ac", "mpm_build_wm", "mpm_free", "mpm_device_bytes", "mpm_upload",
    "mpm_index_info", "mpm_workspace_bytes", "mpm_scan", "mpm_scan_sync", "mpm_batch_plan",
    "mpm_batch_device_bytes", "mpm_batch_upload", "mpm_batch_run", "mpm_batch_capture",
    "mpm_batch_replay", "mpm_batch_groups", "mpm_batch_free", "mpm_export_ac",
    "mpm_export_wm_shift", "mpm_export_unique", "mpm_last_error", "mpm_version", "mpm_read_probe",
    "mpm_tune_time", "mpm_tune_work_bytes", "mpm_mlp_act_floats", "mpm_mlp_forward",
    "mpm_mlp_loss_grad", "mpm_mlp_backward", "mpm_mlp_adam", "mpm_count_ids",
    "mpm_scan_host", "mpm_scan_noalloc", "mpm_batch_launch_key", "mpm_build_ac_var",
    "mpm_build_wm_var", "mpm_read_probe_lanes",
]


def _check(st: int, where: str):
    if st != MPM_OK:
        raise MpmError(st, where)


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def variant(lane_bytes=0, block_threads=0, placement=PLACE_AUTO, grid=0, flags=0) -> Variant:
    return Variant(lane_bytes, block_threads, placement, grid, flags)


def _patterns_np(patterns) -> np.ndarray:
    if isinstance(patterns, (list, tuple)):
        m = len(patterns[0]) if patterns else 0
        patterns = np.frombuffer(b"".join(bytes(p) for p in patterns), np.uint8).reshape(-1, m)
    if hasattr(patterns, "detach"):
        patterns = patterns.detach().cpu().numpy()
    P = np.ascontiguousarray(patterns, dtype=np.uint8)
    if P.ndim != 2:
        raise ValueError("patterns must be a 2-D array [d, m]")
    return P


class Index:
    """A built index (host tables) plus, once uploaded, its device image."""

    def __init__(self, handle: int, algo: int):
        self._h = C.c_void_p(handle)
        self.algo = algo
        self._dev = None  # torch buffer holding the device image

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        inf = Info()
        _check(_L.mpm_index_info(self._h, C.byref(inf)), "mpm_index_info")
        return inf.as_dict()

    @property
    def m(self) -> int:
        return self.info()["m"]

    @property
    def uploaded(self) -> bool:
        return self._dev is not None

    def upload(self, device="cuda", stream=None):
        torch = _torch()
        nbytes = int(_L.mpm_device_bytes(self._h))
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        with torch.cuda.device(buf.device):
            _check(_L.mpm_upload(self._h, C.c_void_p(buf.data_ptr()), buf.numel(),
                                 _stream_handle(stream)), "mpm_upload")
        self._dev = buf
        return self

    def export_ac(self):
        inf = self.info()
        S, cp = inf["n_states"], inf["n_classes"] + 1
        table = np.empty(S * cp, np.uint32)
        classes = np.empty(max(1, inf["n_classes"]), np.uint8)
        _check(_L.mpm_export_ac(self._h, table.ctypes.data, classes.ctypes.data), "mpm_export_ac")
        return table.reshape(S, cp), classes[:inf["n_classes"]]

    def export_wm_shift(self):
        inf = self.info()
        sh = np.empty(4 ** inf["wm_block"], np.uint8)
        _check(_L.mpm_export_wm_shift(self._h, sh.ctypes.data), "mpm_export_wm_shift")
        return sh

    def export_unique(self):
        inf = self.info()
        uoff = np.empty(inf["d_unique"] + 1, np.uint32)
        _check(_L.mpm_export_unique(self._h, uoff.ctypes.data, None), "mpm_export_unique")
        ids = np.empty(max(1, int(uoff[-1])), np.uint32)
        _check(_L.mpm_export_unique(self._h, None, ids.ctypes.data), "mpm_export_unique")
        return uoff, ids[:int(uoff[-1])]

    def close(self):
        if self._h:
            _L.mpm_free(self._h)
            self._h = C.c_void_p(0)
        self._dev = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_ac(patterns, upload: bool = False, goto: bool = False) -> Index:
    """Aho-Corasick index (dense DFA). Host-only unless upload=True. goto=True
    also keeps the goto function and supply links for VARIANT_SUPPLY scans."""
    P = _patterns_np(patterns)
    h = C.c_void_p()
    Pp = P if P.size else np.zeros(1, np.uint8)
    o = Opts()
    o.ac_goto = 1 if goto else 0
    _check(_L.mpm_build_ac(Pp.ctypes.data, P.shape[0], P.shape[1], C.byref(o), C.byref(h)),
           "mpm_build_ac")
    ix = Index(h.value, ALGO_AC)
    return ix.upload() if upload else ix


def build_wm(patterns, B: int = 0, upload: bool = False) -> Index:
    """Wu-Manber index (SHIFT/HASH/PREFIX). B = 0 lets the builder choose."""
    P = _patterns_np(patterns)
    h = C.c_void_p()
    o = Opts()
    o.wm_block = B
    Pp = P if P.size else np.zeros(1, np.uint8)
    _check(_L.mpm_build_wm(Pp.ctypes.data, P.shape[0], P.shape[1], C.byref(o), C.byref(h)),
           "mpm_build_wm")
    ix = Index(h.value, ALGO_WM)
    return ix.upload() if upload else ix


def _var_patterns(patterns):
    """Patterns of any lengths (a list of byte strings or uint8 arrays) as
    one byte array and d + 1 offsets."""
    pats = [bytes(np.asarray(p, np.uint8).tobytes()) if not isinstance(p, (bytes, bytearray))
            else bytes(p) for p in patterns]
    if not pats:
        raise MpmError(MPM_EINVAL, "no patterns")
    off = np.zeros(len(pats) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in pats])
    data = np.frombuffer(b"".join(pats) or b"\0", np.uint8).copy()
    return data, off


def build_ac_var(patterns, upload: bool = False) -> Index:
    """Aho-Corasick index over patterns of different lengths (the automaton of
    the reversed strings; equal lengths give build_ac's index)."""
    data, off = _var_patterns(patterns)
    h = C.c_void_p()
    _check(_L.mpm_build_ac_var(data.ctypes.data, off.ctypes.data, len(off) - 1, None, C.byref(h)),
           "mpm_build_ac_var")
    ix = Index(h.value, ALGO_AC)
    return ix.upload() if upload else ix


def build_wm_var(patterns, B: int = 0, upload: bool = False) -> Index:
    """Wu-Manber index over patterns of different lengths (window: the
    shortest length; equal lengths give build_wm's index)."""
    data, off = _var_patterns(patterns)
    h = C.c_void_p()
    o = Opts()
    o.wm_block = B
    _check(_L.mpm_build_wm_var(data.ctypes.data, off.ctypes.data, len(off) - 1, C.byref(o),
                               C.byref(h)), "mpm_build_wm_var")
    ix = Index(h.value, ALGO_WM)
    return ix.upload() if upload else ix


def workspace_bytes(ix: Index, n: int, var: Variant | None = None) -> int:
    out = C.c_uint64()
    _check(_L.mpm_workspace_bytes(ix.handle, n, C.byref(var) if var else None, C.byref(out)),
           "mpm_workspace_bytes")
    return int(out.value)


def launch_key(ix: Index, var: Variant | None = None) -> int:
    """Key of the batched launch a request with this index and variant joins
    (equal keys share a launch). Host-only."""
    out = _u32()
    _check(_L.mpm_batch_launch_key(ix.handle, C.byref(var) if var else None, C.byref(out)),
           "mpm_batch_launch_key")
    return int(out.value)


def new_workspace(ix: Index, n: int, var: Variant | None = None, device="cuda"):
    """Zero-filled workspace for scans of up to n bytes (reusable)."""
    torch = _torch()
    nb = workspace_bytes(ix, n, var)
    return torch.zeros((nb + 7) // 8, dtype=torch.int64, device=device)


class Scanner:
    """Reusable buffers for repeated scans of one index (workspace, total,
    output); scans are enqueued on the current stream without host waits."""

    def __init__(self, ix: Index, n_max: int, capacity: int, var: Variant | None = None,
                 device="cuda"):
        torch = _torch()
        if not ix.uploaded:
            ix.upload(device)
        self.ix = ix
        self.var = var
        self.ws = new_workspace(ix, n_max, var, device)
        self.total = torch.zeros(1, dtype=torch.int64, device=device)
        self.capacity = int(capacity)
        self.out = torch.empty((max(1, self.capacity), 2), dtype=torch.int32, device=device)

    def scan_async(self, text, n: int | None = None, stream=None):
        n = text.numel() if n is None else n
        _check(_L.mpm_scan(self.ix.handle, C.c_void_p(text.data_ptr()), n,
                           C.c_void_p(self.out.data_ptr()), self.capacity,
                           C.c_void_p(self.ws.data_ptr()), self.ws.numel() * 8,
                           C.c_void_p(self.total.data_ptr()),
                           C.byref(self.var) if self.var else None, _stream_handle(stream)),
               "mpm_scan")

    def scan(self, text, stream=None):
        """Synchronous scan; returns int32 [M, 2] (a view of the output buffer)."""
        tot = C.c_uint64()
        st = _L.mpm_scan_sync(self.ix.handle, C.c_void_p(text.data_ptr()), text.numel(),
                              C.c_void_p(self.out.data_ptr()), self.capacity,
                              C.c_void_p(self.ws.data_ptr()), self.ws.numel() * 8,
                              C.c_void_p(self.total.data_ptr()),
                              C.byref(self.var) if self.var else None, _stream_handle(stream),
                              C.byref(tot))
        if st == MPM_EOVERFLOW:
            raise MpmError(st, "mpm_scan_sync")
        _check(st, "mpm_scan_sync")
        return self.out[: tot.value]


def scan(ix: Index, text, capacity: int | None = None, var: Variant | None = None,
         stream=None):
    """Scan a uint8 CUDA tensor; returns int32 [M, 2] of (pos, id) in
    ascending order. Grows the output once if the first capacity was short."""
    torch = _torch()
    if not ix.uploaded:
        ix.upload(text.device)
    n = text.numel()
    cap = capacity if capacity is not None else n // 32 + 4096
    ws = new_workspace(ix, n, var, text.device)
    total = torch.zeros(1, dtype=torch.int64, device=text.device)
    for _ in range(2):
        out = torch.empty((max(1, cap), 2), dtype=torch.int32, device=text.device)
        tot = C.c_uint64()
        st = _L.mpm_scan_sync(ix.handle, C.c_void_p(text.data_ptr()), n,
                              C.c_void_p(out.data_ptr()), cap, C.c_void_p(ws.data_ptr()),
                              ws.numel() * 8, C.c_void_p(total.data_ptr()),
                              C.byref(var) if var else None, _stream_handle(stream), C.byref(tot))
        if st == MPM_EOVERFLOW and capacity is None:
            cap = int(tot.value)
            continue
        _check(st, "mpm_scan_sync")
        return out[: tot.value]
    raise MpmError(MPM_EOVERFLOW, "scan")


def scan_host(ix: Index, text, chunk: int = 64 << 20, capacity: int | None = None,
              var: Variant | None = None, stream=None):
    """Scan a text held in host memory (a uint8 CPU tensor, pinned for
    overlap, or a numpy array, copied into pinned memory first), `chunk`
    starting positions per device copy. Returns int32 [M, 2] (pos, id) on
    the current device; grows the output once if the first capacity was
    short."""
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device())
    if isinstance(text, np.ndarray):
        t = torch.empty(len(text), dtype=torch.uint8, pin_memory=True)
        t.numpy()[:] = text
        text = t
    assert text.dtype == torch.uint8 and text.device.type == "cpu" and text.is_contiguous()
    if not ix.uploaded:
        ix.upload(dev)
    n = text.numel()
    ns = max(0, n - ix.m + 1)
    c = max(1, min(chunk, ns))
    nch = (ns + c - 1) // c if ns else 1
    stage = torch.empty((2 if nch > 1 else 1) * (c + ix.m - 1), dtype=torch.uint8, device=dev)
    ws = new_workspace(ix, c + ix.m - 1, var, dev)
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    cap = capacity if capacity is not None else n // 32 + 4096
    for _ in range(2):
        out = torch.empty((max(1, cap), 2), dtype=torch.int32, device=dev)
        tot = C.c_uint64()
        st = _L.mpm_scan_host(ix.handle, C.c_void_p(text.data_ptr() if n else 0), n,
                              C.c_void_p(stage.data_ptr()), stage.numel(), c,
                              C.c_void_p(out.data_ptr()), cap, C.c_void_p(ws.data_ptr()),
                              ws.numel() * 8, C.c_void_p(total.data_ptr()),
                              C.byref(var) if var else None, _stream_handle(stream), C.byref(tot))
        if st == MPM_EOVERFLOW and capacity is None:
            cap = int(tot.value)
            continue
        _check(st, "mpm_scan_host")
        return out[: tot.value]
    raise MpmError(MPM_EOVERFLOW, "scan_host")


def count_ids(pairs, d: int, out=None, stream=None):
    """Per-pattern counts of an int32 [M, 2] (pos, id) device list: int32 [d]
    tensor (values are uint32 counts) with out[r] = number of pairs of id r."""
    torch = _torch()
    if out is None:
        out = torch.empty(d, dtype=torch.int32, device=pairs.device)
    assert out.numel() >= d and out.dtype == torch.int32 and out.is_contiguous()
    assert pairs.dtype == torch.int32 and pairs.is_contiguous() and (pairs.numel() == 0 or pairs.shape[1] == 2)
    M = pairs.shape[0] if pairs.numel() else 0
    _check(_L.mpm_count_ids(C.c_void_p(pairs.data_ptr() if M else 0), M, d,
                            C.c_void_p(out.data_ptr()), _stream_handle(stream)), "mpm_count_ids")
    return out[:d]


def read_probe(buf, sink, stream=None):
    """Stream-read a 16-byte aligned CUDA tensor once (HBM ceiling probe)."""
    _check(_L.mpm_read_probe(C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                             C.c_void_p(sink.data_ptr()), _stream_handle(stream)), "mpm_read_probe")


def read_probe_lanes(buf, lane_bytes: int, sink, stream=None):
    """Read a 128-byte aligned CUDA tensor in the scans' lane pattern (each
    of 1024 lanes per workgroup reads its own lane_bytes range by lines)."""
    _check(_L.mpm_read_probe_lanes(C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                                   lane_bytes, C.c_void_p(sink.data_ptr()), _stream_handle(stream)),
           "mpm_read_probe_lanes")


def pairs_numpy(t) -> tuple[np.ndarray, np.ndarray]:
    """(pos, id) as uint32 numpy arrays from an int32 [M, 2] device tensor."""
    a = t.cpu().numpy().view(np.uint32)
    return a[:, 0].copy(), a[:, 1].copy()


from . import batch  # noqa: E402,F401  (batched launches)
