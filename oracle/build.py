"""Compile the CPU oracle (plain C) into oracle/liboracle.so with gcc.

Flags: -O2 -ffp-contract=off so that no multiply-add is fused unless the
source asks for it (fmaf in the float skeleton update); -fopenmp for the
loops over independent rows, planes and elements (same bits for any thread
count).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["oracle.c", "surrogate.c"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c11", "-Wall", "-Wextra",
           "-shared", "-fPIC", *srcs, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
