"""Builds the oracle's shared library (test infrastructure: see labs_oracle.c).

Plain gcc, -O2, no vectorisation flags beyond the defaults: the oracle is meant to be read,
not tuned.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "labs_oracle.c")
LIB = os.path.join(HERE, "liblabs_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", SRC, "-o", LIB]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
