"""Builds the CPU oracle's shared library (test infrastructure only).

    python -m oracle.build

Compiles ``pfc_oracle.c`` with gcc, -O2, OpenMP, no fast-math and no FMA
contraction, into ``oracle/liboracle_pfc.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pfc_oracle.c")
LIB = os.path.join(HERE, "liboracle_pfc.so")


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
           "-Wall", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
