"""Build step for the CPU oracle (test infrastructure only).

Compiles ``vto.c`` into ``liboracle.so`` next to this file with plain gcc:
IEEE binary64, no fused multiply-add contraction, no fast-math, OpenMP.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

FLAGS = ["-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp",
         "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
         "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose=False):
    """Compile the oracle; returns the path of the shared library."""
    src = os.path.join(HERE, "vto.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", *FLAGS, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
