"""Compile the C oracle into oracle/_lb_oracle.so with the host compiler.

TEST INFRASTRUCTURE: building the checker is part of the project build, using
it is reserved for the tests, the smoke check and the CPU-baseline leg.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lb_oracle.c")
LIB = os.path.join(HERE, "_lb_oracle.so")

# Plain IEEE binary64: no contraction into FMA, no fast-math, scalar code.
# OpenMP only runs the column loops on several host threads (all-core
# baseline); the thread count is 1 unless the caller sets it.
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp"]


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
    sys.exit(0)
