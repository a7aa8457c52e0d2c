"""Build the CPU oracle (test infrastructure only) into oracle/libffo.so.

Run as ``python oracle/build.py`` or call :func:`build`.  The flags keep IEEE
semantics: no fast-math, no contraction of a*b+c into fused multiply-adds
except where the source writes std::fma.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libffo.so")
SRCS = [os.path.join(HERE, "ffo.cpp"), os.path.join(HERE, "ffo_expr.cpp")]

FLAGS = ["-std=c++17", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
         "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["g++", *FLAGS, *SRCS, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
