"""Compile the FP64 CPU oracle (plain C, gcc, OpenMP over subsystems).

Test infrastructure: the oracle is the checker of the GPU library and is
built beside it, never linked into it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "btd_oracle.c")
LIB = os.path.join(HERE, "libbtd_oracle.so")


def build(verbose: bool = False) -> str:
    """Compile oracle/btd_oracle.c into oracle/libbtd_oracle.so and return its path.

    -O2 without -ffast-math (no reassociation) and without -march=native, so
    the same shared object runs on any x86-64 host.
    """
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
