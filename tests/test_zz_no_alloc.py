"""The scan entry point that allocates nothing (mpm_scan_noalloc): its
workspace is the library's static per-device scratch. Its lists and totals
must equal those of mpm_scan on a caller workspace, call after call on the
same scratch (the second call with a smaller text), and requests that need
more scratch than it holds are refused before anything is enqueued."""

import ctypes as C
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mpm():
    import paper_1407_2889_amd as m
    return m


def noalloc(mpm, ix, text, n, out, cap, total, var):
    return mpm._L.mpm_scan_noalloc(ix.handle, C.c_void_p(text.data_ptr()), n,
                                   C.c_void_p(out.data_ptr()), cap,
                                   C.c_void_p(total.data_ptr()),
                                   C.byref(var) if var is not None else None,
                                   mpm._stream_handle())


def test_noalloc_refuses_oversized_requests_on_the_host(mpm):
    """A request with more chunks than the static scratch has status words
    fails with ENOMEM before the scratch is touched (no GPU needed)."""
    P = np.frombuffer(b"ACGTACGT", np.uint8).reshape(1, 8)
    ix = mpm.build_ac(P)
    v = mpm.variant(lane_bytes=16, block_threads=256)
    n = 600 << 20  # 600 MiB / 4 KiB chunks = 153,600 status words > (1 MiB - 64) / 8
    assert mpm.workspace_bytes(ix, n, v) > mpm.NOALLOC_SCRATCH_BYTES
    st = mpm._L.mpm_scan_noalloc(ix.handle, C.c_void_p(4096), n, None, 0, C.c_void_p(8),
                                 C.byref(v), None)
    assert st == mpm.MPM_ENOMEM
    assert b"static scratch" in mpm._L.mpm_last_error()


@pytest.mark.gpu
@pytest.mark.parametrize("algo", ["ac", "wm"])
def test_noalloc_equals_workspace_scan_twice(mpm, algo):
    assert torch.cuda.is_available()
    text, ps = synth.workload_est256(n=24 << 20)
    dev = torch.from_numpy(text).cuda()
    ix = (mpm.build_ac if algo == "ac" else mpm.build_wm)(ps.patterns, upload=True)
    for var in (None, mpm.variant(lane_bytes=1024, block_threads=1024),
                mpm.variant(lane_bytes=64, block_threads=256, placement=mpm.PLACE_GLOBAL)):
        # two calls in a row on the same scratch, the second on a smaller text
        for n in (len(text), 3_000_017):
            say(f"[noalloc] {algo} n={n} variant={var}")
            want = mpm.scan(ix, dev[:n], var=var)
            cap = int(want.shape[0]) + 8
            out = torch.full((cap, 2), -1, dtype=torch.int32, device="cuda")
            total = torch.full((1,), -1, dtype=torch.int64, device="cuda")
            st = noalloc(mpm, ix, dev, n, out, cap, total, var)
            assert st == mpm.MPM_OK, mpm._L.mpm_last_error()
            torch.cuda.synchronize()
            assert int(total.item()) == want.shape[0]
            assert torch.equal(out[: want.shape[0]], want)
            assert bool((out[want.shape[0]:] == -1).all())
    # a counting call (capacity 0) and an overflowing one keep the sorted prefix
    want = mpm.scan(ix, dev, var=None)
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.full((5, 2), -1, dtype=torch.int32, device="cuda")
    assert noalloc(mpm, ix, dev, len(text), out, 0, total, None) == mpm.MPM_OK
    torch.cuda.synchronize()
    assert int(total.item()) == want.shape[0]
    assert bool((out == -1).all())
    assert noalloc(mpm, ix, dev, len(text), out, 5, total, None) == mpm.MPM_OK
    torch.cuda.synchronize()
    assert int(total.item()) == want.shape[0]
    assert torch.equal(out, want[:5])
