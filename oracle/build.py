"""Build the CPU oracle (test infrastructure) with gcc.

Plain C11, no fast-math and no FP contraction, so FP32 results follow the
stated operation order exactly; ``fmaf`` is the C library's correctly rounded
fused multiply-add.  OpenMP shares the per-cell kernel evaluation out over
rows (every cell is computed on its own, so the results do not depend on the
thread count); OMP_NUM_THREADS sets the count.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libhdoracle.so")


def build(verbose=False):
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-Wall", "-Wno-unused-value", "-o", LIB, os.path.join(HERE, "hdoracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
