"""Builds the native libraries of the package in-tree.

* ``libhrms.so``       -- the gfx950 harmonic-sum library (HIP kernels + C ABI),
                          compiled with hipcc for gfx950 only;
* ``libhrms_synth.so`` -- the host input generator (gcc).

Floating-point flags: no multiply-add contraction (``-ffp-contract=off``), so
every FP32 sum is the sequence of additions the kernels write, and packed FP32
instructions are disabled for device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhrms.so")

HIP_SOURCES = ["hrms_kernels.hip", "hrms_abi.cpp", "hrms_noalloc.hip"]
HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build_hip(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp,
           *[os.path.join(CSRC, s) for s in HIP_SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def build_all(verbose: bool = False) -> None:
    from . import synth
    synth.build(force=True)
    build_hip(verbose=verbose)


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    from paper_1812_02647_amd import build as _b
    _b.build_all(verbose=True)
