"""Compile the CPU oracle (test infrastructure) into oracle/liboracle_vbdr.so.

Plain gcc, no HIP headers, no code shared with the HIP library.  FP
contraction is off so that the FP64 estimator rounds each operation once.
No -march=native: the library is built here and also loaded on other hosts.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vbdr_oracle.c")
LIB = os.path.join(HERE, "liboracle_vbdr.so")


def build_oracle(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))
