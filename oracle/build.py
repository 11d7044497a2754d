"""Build the CPU oracle library (plain g++, OpenMP).  Test infrastructure."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

# x86-64-v3 (AVX2/FMA) rather than -march=native: the library is built here
# and loaded on other hosts too.  -fcx-limited-range: plain complex product
# and quotient formulas (no NaN-recovery slow path).
FLAGS = ["-O3", "-march=x86-64-v3", "-fcx-limited-range", "-fopenmp", "-std=c++17",
         "-fPIC", "-shared"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["g++", *FLAGS, SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
