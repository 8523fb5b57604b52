"""Compile the CPU oracle into oracle/liboracle.so.

Test infrastructure: the oracle is built (not used) by the package build step,
and loaded only by the tests, the smoke check and the benchmark's CPU-baseline
leg.  Plain gcc, FP64, no floating-point contraction, no -march=native (the
library may run on a different host CPU than the one that built it).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=c11", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
        "-fPIC", "-shared", "-Wall", "-Wextra",
        "-o", LIB + ".tmp", os.path.join(HERE, "lbm_oracle.c"), "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
