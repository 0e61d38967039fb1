"""Build libsmcx.so in-tree with hipcc for gfx950.

Usage: python -m paper_2503_12591_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsmcx.so")

SOURCES = ["smcx_kernels.hip", "smcx_api.cpp"]

# -ffp-contract=off: every binary64 multiply and add of dE is rounded on its
# own, in the order written, so that trajectories are reproducible bit for bit.
# -packed-fp32-ops: packed FP32 instructions are kept out of the generated code.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    cmd = (["hipcc"] + FLAGS + ["-I", INCLUDE, "-I", CSRC, "-o", LIB + ".tmp"] +
           [os.path.join(CSRC, s) for s in SOURCES])
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libsmcx.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
