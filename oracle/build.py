"""Build the FT-GCR CPU oracle (test infrastructure only).

The oracle is plain C compiled by gcc with no fast-math and no FP contraction,
so every operation is the IEEE-754 binary64 operation written in the source;
OpenMP splits only loops whose results do not depend on the thread count.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ftgcr_oracle.c")
LIB = os.path.join(HERE, "libftgcr_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-fopenmp",
           "-Wall", "-Wextra", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
