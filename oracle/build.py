"""Builds the CPU oracle (test infrastructure) with gcc.

The oracle is compiled without floating-point contraction or fast-math so
that every binary32 operation is one IEEE round-to-nearest-even operation,
as its schedules require.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "coxo.c")
LIB = os.path.join(HERE, "libcoxo.so")

CFLAGS = ["-std=gnu11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-fno-strict-aliasing", "-Wall", "-Wno-unused-function",
          "-pthread"]


def build(verbose=False):
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
