"""Builds libsynth.so (the C ABI and every HIP kernel) in-tree for gfx950.

Usage: python -m paper_2104_12922_amd.build [-v]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsynth.so")

SOURCES = ["api.cpp", "params.hip", "render.hip", "spectral.hip", "adjoint.hip", "gemm.hip",
           "mlp.hip", "dft.hip", "reduce.hip", "mmd.hip", "vcf.hip", "fm.hip"]

# Packed-FP32 instructions are disabled for all device code (plain float code
# is scheduled onto the non-packed VALU).  Machine LICM is disabled: it hoists
# the float64 constants of the once-per-voice exp2/log2/pow code out of every
# loop and keeps them live across the audio-rate loops, which doubles the
# render kernel's VGPR count (200 -> 112) and halves its occupancy.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-disable-machine-licm",
             "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libsynth.so)")


def build(verbose: bool = False) -> str:
    """Compile every source and link libsynth.so next to this file; returns its path."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"]
        cmd = [hipcc(), *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, *lang, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
