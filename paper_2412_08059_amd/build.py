"""Build the gfx950 HIP library ``libmpcg.so`` in-tree with hipcc.

    python paper_2412_08059_amd/build.py     (run as a script: importing the
                                             package would load the library)

Device code is compiled for gfx950 only, with packed-FP32 instructions turned
off.  The host-side kNN file is compiled with -ffp-contract=off so that its
floating-point sequence is exactly the one written in the source.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(REPO, "include")
LIB = os.path.join(HERE, "libmpcg.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIP_SOURCES = ["kernels_cg.hip", "kernels_sell.hip", "kernels_bfs.hip", "kernels_jacobi.hip", "kernels_batch.hip",
               "batch_engine.hip", "capi.hip"]
HOST_SOURCES = ["knn.cpp", "tune.cpp"]


def _hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout)
        raise RuntimeError(f"build step failed: {cmd[0]} ... {cmd[-1]}")
    return r.stdout


def build(verbose: bool = False) -> str:
    """Compile every source and link libmpcg.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    hipcc = _hipcc()
    common = ["-O3", "-fPIC", "-std=c++17", "-pthread", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall"]
    dev = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    cmds, objs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmds.append([hipcc, *common, *dev, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmds.append(["g++", "-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", f"-I{INCLUDE}", f"-I{CSRC}",
                     "-Wall", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # one compiler process per source, a few at a time
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
        list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
