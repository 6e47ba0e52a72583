"""Build the oracle's shared library (test infrastructure only).

Compiles ``rlb_oracle.cpp`` with g++ at -O2 with floating-point contraction off
(the oracle evaluates every formula in the written order, IEEE FP64,
round-to-nearest-even) into ``liboracle_rlb.so`` next to this file.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rlb_oracle.cpp")
LIB = os.path.join(HERE, "liboracle_rlb.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
        "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC,
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
