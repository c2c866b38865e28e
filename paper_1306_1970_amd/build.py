"""Build libflr.so (HIP, gfx950) in-tree with hipcc.

Every call compiles; the result lands next to this file so that it travels
with the source tree.  Flags: -O3 for gfx950 only, packed-FP32 instruction
selection disabled, position-independent shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libflr.so")
SOURCES = ["flr_kernels.hip", "flr_engine.hip", "flr_grid.hip", "flr_gemm.hip", "flr_dense.hip", "flr_server.hip"]
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include")]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False, jobs: int = 4) -> str:
    objs = []
    procs = []
    for src in sources():
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0), verbose)
    while procs:
        _wait(procs.pop(0), verbose)
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SO)
    for o in objs:
        os.remove(o)
    return SO


def _wait(item, verbose):
    proc, src = item
    out, _ = proc.communicate()
    text = out.decode(errors="replace")
    # the host pass does not know the packed-fp32 feature; that warning is harmless
    lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and "is not a recognized feature" not in l]
    if proc.returncode != 0:
        sys.stderr.write("\n".join(lines) + "\n")
        raise RuntimeError("hipcc failed on " + src)
    if verbose and lines:
        print("\n".join(lines))


if __name__ == "__main__":
    print(build(verbose=True))
