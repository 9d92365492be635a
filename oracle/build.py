"""Compile the FP64 CPU oracle (plain C, gcc) into oracle/liboracle.so.

Test infrastructure: the product library never links or loads the result.
Built with -O2 and -ffp-contract=off (no fused multiply-add, no fast-math) so
the oracle's arithmetic is plain IEEE double in the order the source states,
and with -fopenmp for its parallel particle and node loops (their scatters sum
private per-thread grids in thread order; see the C source).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-Wall", "-Wextra",
           "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
