"""Build libmpm.so for gfx950 with hipcc (in-tree, next to this file).

    python paper_1407_2889_amd/build.py        # run by path: the package's
                                               # __init__ needs the library
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libmpm.so")
SOURCES = [  # longest compiles first (parallel build)
    "mpm_scan_var.hip", "mpm_scan_ladder.hip", "mpm_scan_ac16_hot.hip", "mpm_scan_ac16_glb.hip", "mpm_scan_ac16_lds.hip",
    "mpm_scan_ac_supply.hip", "mpm_scan_batch_other.hip", "mpm_scan_ac32_glb.hip",
    "mpm_scan_batch_ac16_hot.hip", "mpm_scan_batch_ac16_glb.hip", "mpm_scan_batch_ac16_lds.hip",
    "mpm_scan_wm.hip", "mpm_host.cpp", "mpm_scan.hip", "mpm_mlp.hip", "mpm_count.hip",
    "mpm_stream.hip", "mpm_noalloc.hip", "mpm_mixed.cpp", "mpm_probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    # no packed-FP32 instructions in any kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE,
]


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _headers() -> list[str]:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    return hs + [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]


def build(verbose: bool = False, extra: list[str] | None = None, jobs: int = 8,
          incremental: bool = False) -> str:
    """Compile every source (in parallel, one object per source) and link
    libmpm.so. Recompiles everything unless `incremental`, which keeps the
    objects in _build/ at the repository root and recompiles a source only
    when it, or any header, is newer than its object."""
    import concurrent.futures as cf
    import tempfile
    compile_flags = [f for f in FLAGS if f != "-shared"]
    keep = os.path.join(os.path.dirname(HERE), "_build") if incremental else None
    with tempfile.TemporaryDirectory(prefix="mpm_build_") as td:
        odir = keep or td
        os.makedirs(odir, exist_ok=True)
        newest_h = max((os.path.getmtime(h) for h in _headers()), default=0.0)
        objs = []
        cmds = []
        for src in sources():
            obj = os.path.join(odir, os.path.basename(src) + ".o")
            objs.append(obj)
            if keep and os.path.exists(obj) and os.path.getmtime(obj) > max(
                    os.path.getmtime(src), newest_h):
                continue
            cmds.append([HIPCC, *compile_flags, *(extra or []), "-c", src, "-o", obj])
        if cmds:
            with cf.ThreadPoolExecutor(max(1, min(jobs, len(cmds)))) as ex:
                for cmd in cmds:
                    if verbose:
                        print(" ".join(cmd), flush=True)
                list(ex.map(subprocess.check_call, cmds))
        tmp = LIB + f".tmp{os.getpid()}"
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    args = sys.argv[1:]
    inc = "--incremental" in args
    build(verbose=True, extra=[a for a in args if a != "--incremental"], incremental=inc)
    print(LIB)
