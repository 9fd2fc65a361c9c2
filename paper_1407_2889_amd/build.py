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
SOURCES = ["mpm_host.cpp", "mpm_scan.hip", "mpm_scan_ac16_lds.hip", "mpm_scan_ac16_glb.hip",
           "mpm_scan_ac16_hot.hip", "mpm_scan_ac32_glb.hip", "mpm_scan_wm.hip",
           "mpm_scan_batch_ac16_lds.hip", "mpm_scan_batch_ac16_glb.hip",
           "mpm_scan_batch_ac16_hot.hip", "mpm_scan_batch_other.hip", "mpm_mlp.hip",
           "mpm_count.hip", "mpm_stream.hip",
           "mpm_scan_ac_supply.hip"]
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


def build(verbose: bool = False, extra: list[str] | None = None, jobs: int = 8) -> str:
    """Compile every source (in parallel, one object per source) and link
    libmpm.so. Always recompiles."""
    import concurrent.futures as cf
    import tempfile
    compile_flags = [f for f in FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="mpm_build_") as td:
        objs = []
        cmds = []
        for src in sources():
            obj = os.path.join(td, os.path.basename(src) + ".o")
            objs.append(obj)
            cmds.append([HIPCC, *compile_flags, *(extra or []), "-c", src, "-o", obj])
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
    build(verbose=True, extra=sys.argv[1:])
    print(LIB)
