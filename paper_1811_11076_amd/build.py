"""Compiles the HIP library (libtsknn.so) for gfx950, in-tree.

Flags:
  -ffp-contract=off   no implicit a*b+c fusion: every fp32 rounding is where
                      the source puts it (the DP must match the fp32 mirror
                      arithmetic bit for bit);
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      no packed-fp32 VALU instructions.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtsknn.so")
ARCH = os.environ.get("TSK_ARCH", "gfx950")

SOURCES = ["tsknn.hip"]
DEPS = ["device.hpp", "kernels.hpp"]


def lib_path() -> str:
    return LIB


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES] + (extra or [])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
