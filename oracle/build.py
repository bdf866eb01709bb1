"""Compile the C oracle into ``oracle/liboracle_sff.so`` (gcc, -O2, OpenMP).

Test infrastructure: the oracle is built beside the GPU library so that the
checker exists wherever the tests run; nothing in the product path loads it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sff_oracle.c")
LIB = os.path.join(HERE, "liboracle_sff.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    # -ffp-contract=off: the FP32 cost sums are rounded operation by operation
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
