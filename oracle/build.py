"""Compile the C oracle into ``oracle/liboracle.so`` (test infrastructure only)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

CMD = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
       "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB,
       os.path.join(HERE, "oracle.c"), "-lm"]


def build(verbose: bool = False) -> str:
    if verbose:
        print(" ".join(CMD), flush=True)
    subprocess.run(CMD, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
