"""Builds the SIMD-collapsed CPU executor three ways with gcc.

libcoxs_avx512.so (AVX-512 F/BW/DQ/VL/CD), libcoxs_avx2.so (AVX2 + FMA)
and libcoxs_scalar.so (lane loops, no auto-vectorisation: the build
without SIMD).  All without floating-point contraction or fast-math, so
every binary32 operation is one IEEE round-to-nearest-even operation and
fused multiply-adds appear only where the schedules name them.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "coxs.c")
COMMON = ["-std=gnu11", "-O3", "-fPIC", "-shared", "-pthread", "-ffp-contract=off", "-fno-fast-math",
          "-fno-strict-aliasing", "-Wall", "-Wno-unused-function"]
VARIANTS = {
    "avx512": ["-DCOXS_ISA=512", "-mavx512f", "-mavx512bw", "-mavx512dq", "-mavx512vl", "-mavx512cd", "-mfma",
               "-mpopcnt", "-mbmi2"],
    "avx2": ["-DCOXS_ISA=256", "-mavx2", "-mfma", "-mpopcnt", "-mbmi2", "-mno-avx256-split-unaligned-load",
             "-mno-avx256-split-unaligned-store"],
    "scalar": ["-DCOXS_ISA=0", "-fno-tree-vectorize", "-fno-tree-slp-vectorize"],
}


def lib_path(isa):
    return os.path.join(HERE, f"libcoxs_{isa}.so")


def build(verbose=False):
    out = []
    for isa, flags in VARIANTS.items():
        dst = lib_path(isa)
        cmd = ["gcc", *COMMON, *flags, SRC, "-o", dst + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(dst + ".tmp", dst)
        out.append(dst)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
