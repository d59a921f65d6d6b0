"""Compile the oracle's C stepper into oracle/_lbe_oracle.so (gcc, OpenMP).

TEST INFRASTRUCTURE: building the checker is not using it; only tests, the smoke
check and the benchmark's CPU-baseline leg load the result.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbe_oracle.c")
OUT = os.path.join(HERE, "_lbe_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99", "-Wall", "-Wextra", SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


def ensure_built() -> str:
    if not os.path.exists(OUT) or os.path.getmtime(OUT) < os.path.getmtime(SRC):
        build()
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
