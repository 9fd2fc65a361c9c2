"""Host-side checks of the benchmark script (no GPU): the one-GPU rule, the
committed HBM counter record it reads, and the digest that retires the
record when kernel sources change."""

import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_record_matches_current_kernels():
    """While the committed FETCH/WRITE record applies to the kernels as they
    are, its calibrated bytes are at least the scan's algorithmic bytes (the
    text is read once) and within twice them; after a kernel change the
    benchmark reports no traffic until the counters are taken again."""
    p = os.path.join(ROOT, "profiles", "scan_est256_hbm_counters.md")
    rec = next(json.loads(l[len("counters: "):]) for l in open(p) if l.startswith("counters: "))
    if rec["digest"] != bench.kernel_digest():
        assert bench.recorded_traffic("est256", "ac") is None
        pytest.skip("kernel sources changed since the counters were taken")
    n = 268435456
    for algo in ("ac", "wm"):
        t = bench.recorded_traffic("est256", algo)
        assert t is not None and n <= t <= 2 * n, (algo, t)


def test_digest_changes_with_sources(tmp_path, monkeypatch):
    """A change to any source of the single-text scan kernels hashes
    differently (the record then no longer applies); other sources do not
    enter the digest."""
    import shutil
    d0 = bench.kernel_digest()
    src = os.path.join(os.path.dirname(bench.__file__), "paper_1407_2889_amd", "csrc")
    csrc = tmp_path / "paper_1407_2889_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.SCAN_SOURCES:
        shutil.copy(os.path.join(src, f), csrc / f)
    monkeypatch.setattr(bench, "__file__", str(tmp_path / "bench.py"))
    assert bench.kernel_digest() == d0
    (csrc / "unrelated.hip").write_text("// another kernel\n")
    assert bench.kernel_digest() == d0
    with open(csrc / "mpm_scan_impl.h", "a") as f:
        f.write("// changed\n")
    assert bench.kernel_digest() != d0
