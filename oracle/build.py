"""Build the CPU oracle shared library (test infrastructure only).

    python oracle/build.py

Compiles zeus_oracle.c with gcc into oracle/libzeus_oracle.so.  No fused
multiply-add (-ffp-contract=off), no fast-math; OpenMP over starts.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libzeus_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "zeus_oracle.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu99", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
