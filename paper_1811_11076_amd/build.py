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

SOURCES = ["tsknn.hip", "k_band.hip", "k_tube.hip", "k_wave.hip", "k_bound.hip", "k_lbu.hip", "mlp.hip", "subseq.hip"]


def lib_path() -> str:
    return LIB


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


def _flags() -> list[str]:
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
            "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    """Compiles every source to an object in parallel, then links the .so."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    tag = "%d" % os.getpid()

    def compile_one(src):
        obj = os.path.join(objdir, src.replace(".hip", "") + "." + tag + ".o")
        cmd = [hipcc()] + _flags() + (extra or []) + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp" + tag
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
