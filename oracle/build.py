"""Compile the CPU oracle (test infrastructure only) into oracle/liboracle.so.

Plain gcc, no vendor BLAS, IEEE operations without contraction or
reassociation so that the oracle's arithmetic is exactly what its source says
(optimisation and vector instructions then change speed, never a result bit).
x86-64-v3 (AVX2) rather than -march=native: the library is built here and
loaded on other hosts, which must be able to run it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dsu_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
