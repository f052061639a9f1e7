"""Compile the float64 CPU oracle (plain C + OpenMP) into oracle/libsst_oracle.so.

Test infrastructure only: the oracle is what the GPU library is checked
against, never part of the product path.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sst_oracle.c")
SRCS = [SRC, os.path.join(HERE, "sst_oracle_abi.c")]
LIB = os.path.join(HERE, "libsst_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra"] + SRCS + ["-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
