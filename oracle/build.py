"""Build step for the CPU oracle libraries (test infrastructure only).

Compiles esdg_oracle.c with gcc into liboracle.so beside this file:
plain -O3 with OpenMP, no fast-math, no -march=native (the library travels
to hosts with other CPUs).  opcount.cpp (the oracle's pointwise physics
compiled over a counting scalar) becomes libopcount.so.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "esdg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
OPC_SRC = os.path.join(HERE, "opcount.cpp")
OPC_LIB = os.path.join(HERE, "libopcount.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-Wall", "-Wextra", "-o", OPC_LIB + ".tmp", OPC_SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OPC_LIB + ".tmp", OPC_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
