"""Build the FP64 oracle's shared library (test infrastructure only).

Plain C11 with OpenMP over agents; IEEE arithmetic (no fast-math), so every
result follows the order written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libgmapp_oracle.so")
SOURCES = [os.path.join(HERE, "gmapp_oracle.c"), os.path.join(HERE, "gmapp_oracle_grad.c"),
           os.path.join(HERE, "gmapp_oracle_pose.c")]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB + ".tmp"] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
