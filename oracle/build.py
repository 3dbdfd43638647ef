"""Compile the CPU oracle into oracle/libea_oracle.so with gcc.

The oracle is test infrastructure: only the tests, the smoke check and the
benchmark's CPU-baseline leg load the library this produces.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libea_oracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "ea_oracle.c")
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
