"""Build the oracle's shared library with gcc (plain C99, FP64, no fast-math).

    python oracle/build_oracle.py

-ffp-contract=off keeps every multiply and add separately rounded as the
source is written; OpenMP is used only by the optional threaded site loop.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "elbm_oracle.c")
LIB = os.path.join(HERE, "liboracle_elbm.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
