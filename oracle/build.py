"""Compile the oracle's C stencil into oracle/libhisq_oracle.so with gcc.

Test infrastructure: the library built here is loaded only by the tests, the
smoke check and the CPU-baseline leg of the benchmark.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hisq_stencil.c")
LIB = os.path.join(HERE, "libhisq_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fcx-limited-range", "-fopenmp", "-fPIC",
           "-shared", "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
