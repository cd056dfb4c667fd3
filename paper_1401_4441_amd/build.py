"""Build ``liblc.so`` (the HIP library behind include/lc.h) for gfx950.

    python -m paper_1401_4441_amd.build

The library is built in-tree next to this file.  Flags:
  --offload-arch=gfx950        MI355X only
  -ffp-contract=off            the canonical pair sequence rounds after every
                               operation (no FMA contraction)
  -Xclang -target-feature -Xclang -packed-fp32-ops
                               no packed FP32 instructions
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblc.so")

SOURCES = [os.path.join(CSRC, "lc.hip"), os.path.join(CSRC, "lc_sched.cpp")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *(extra or []), *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
