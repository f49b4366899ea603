"""Compile the C oracle into oracle/libyyo.so (test infrastructure only).

gcc, -O2, no FMA contraction and no fast-math, so that the oracle rounds
each operation as written; OpenMP only distributes independent lines and
points.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libyyo.so")


def build(verbose=False):
    src = os.path.join(HERE, "yyo.c")
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
