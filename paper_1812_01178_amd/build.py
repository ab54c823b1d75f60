"""Build libtri.so (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_1812_01178_amd.build`` or ``build()`` from Python.
Always recompiles (the build check must exercise the compiler).  Every
source compiles to its own object (in parallel), then one link makes the
shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libtri.so")
SOURCES = ["tri_api.hip", "tri_kernels.hip", "tri_contig_reg.hip", "tri_refine.hip", "tri_contig_refine.hip",
           "tri_general_refine.hip", "tri_copy.hip", "tri_fft.hip", "tri_ns.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # no packed FP32 instructions anywhere in the device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
    ]


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(8, n, int(os.environ.get("MAX_JOBS", "8"))))


def build(verbose: bool = False) -> str:
    with tempfile.TemporaryDirectory(prefix="libtri_build_") as tmpdir:
        objs = []
        cmds = []
        for src in sources():
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            objs.append(obj)
            cmds.append([HIPCC] + flags() + ["-c", src, "-o", obj])

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)

        with ThreadPoolExecutor(_jobs()) as pool:
            list(pool.map(run, cmds))
        tmp = LIB + ".tmp"
        link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp]
        run(link)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
