"""Builds the FP64 oracle's shared library (plain C, gcc, no GPU code).

TEST INFRASTRUCTURE ONLY: the library built here is loaded by the tests, the
package smoke check and the benchmark's CPU-baseline leg, never by the GPU path.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gsr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    # plain IEEE double arithmetic: no fast-math, no FMA contraction, and no
    # -march=native (the library also runs on other hosts' CPUs)
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wextra", "-Wno-unused-parameter", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
