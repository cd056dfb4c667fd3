"""Compile the C oracle into ``oracle/liblc_oracle.so`` with gcc.

Test infrastructure only.  -ffp-contract=off keeps every floating-point
operation separately rounded (no fused multiply-add), which the oracle's
canonical FP32 pair sequence relies on.  -fopenmp: the loop-exchange
sweep (the benchmark's parallel CPU reference) runs with OpenMP.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lc_oracle.c")
LIB = os.path.join(HERE, "liblc_oracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
          "-fPIC", "-shared", "-Wall", "-Wextra", "-fopenmp"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
