"""Builds the CPU oracle (test infrastructure) with gcc: oracle/liboracle.so (serial plain
loops and the reference inspector) and oracle/liboracle_omp.so (the same value loops over host
cores with OpenMP, the benchmark's many-core CPU baseline).

IEEE binary64 without contraction: -O2 -ffp-contract=off.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ddf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
SRC_OMP = os.path.join(HERE, "ddf_oracle_omp.c")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11", "-fPIC", "-shared",
           "-Wall", "-Wextra", SRC_OMP, "-o", LIB_OMP + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_OMP + ".tmp", LIB_OMP)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
