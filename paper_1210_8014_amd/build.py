"""Build libamr.so (HIP kernels for gfx950 + host builder) in-tree with hipcc.

python -m paper_1210_8014_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libamr.so")
# the VALU issue-rate probe (a measurement aid, not part of the library)
PROBE_SRC = "probe.hip"
PROBE_LIB = os.path.join(HERE, "libamrprobe.so")
SOURCES = ["render.hip", "batch.hip", "lod.hip", "post.hip", "stream.hip", "tree.cpp"]
HEADERS = ["traverse.h", "internal.h", os.path.join("..", "..", "include", "amr.h")]

HIP_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-ffp-contract=off",                      # no fused products: exact-order arithmetic
    "-fno-gpu-flush-denormals-to-zero",       # keep fp32 denormals (max stays bit-exact)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    for f in SOURCES + HEADERS:
        if os.path.getmtime(os.path.join(CSRC, f)) > t:
            return True
    return False


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every source for gfx950 and link libamr.so in the package dir."""
    if not force and not _stale():
        return LIB
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc"] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-pthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    tmp = PROBE_LIB + ".tmp"
    cmd = ["hipcc"] + HIP_FLAGS + ["-shared", os.path.join(CSRC, PROBE_SRC), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose="-v" in sys.argv)
    print(LIB)
