"""Compile the CPU oracle (plain C, FP64, OpenMP) into oracle/liblbm81_oracle.so.

Test infrastructure only: the oracle is the checker of the GPU library, never
part of it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm81_oracle.c")
LIB = os.path.join(HERE, "liblbm81_oracle.so")


def build(verbose: bool = False) -> str:
    # -O2 without fast-math keeps IEEE semantics; the default x86-64 target has
    # no FMA, so gcc does not contract multiply-adds.
    cmd = ["gcc", "-std=c99", "-O2", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
