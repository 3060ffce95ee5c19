"""Build libhefk.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.environ.get("HEFK_LIBRARY") or os.path.join(PKG, "libhefk.so")
SOURCES = ["hefk_kernels.hip", "hefk_grad.hip", "hefk_energy.cpp"]
ARCH = os.environ.get("HEFK_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            # fuse multiply-adds only inside one source expression: the fused / unfused
            # choice then does not depend on the inlining context, so a propagation resumed
            # from stored walkers is bitwise the same as an uninterrupted one
            "-ffp-contract=on",
            # packed FP32 arithmetic stays off (v_pk_* forms are avoided on this target)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", HERE] + os.environ.get("HEFK_DEFINES", "").split()


def build(verbose: bool = False) -> str:
    """Compile every source to an object, then link the shared library."""
    bdir = os.path.join(HERE, "_build" + os.environ.get("HEFK_BUILD_TAG", ""))
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + flags() + ["-c", os.path.join(HERE, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-x", "c++",
                   "-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if not os.environ.get("HEFK_LIBRARY"):
        build_rates(verbose)
    return LIB


RATES = os.path.join(PKG, "valu_rates")


def build_rates(verbose: bool = False) -> str:
    """The issue-cost calibration program (valu_rates.hip): a standalone executable."""
    tmp = RATES + ".tmp"
    cmd = [hipcc()] + flags() + [os.path.join(HERE, "valu_rates.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, RATES)
    return RATES


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
