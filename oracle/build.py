"""Build the CPU oracle shared library (test infrastructure).

    python oracle/build.py

Compiles pn_oracle.cpp with g++ in plain IEEE double (no fast-math, no FMA
contraction) into oracle/liboracle.so.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pn_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-fno-fast-math", "-ffp-contract=off",
           "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
