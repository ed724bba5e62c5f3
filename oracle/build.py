"""Build the CPU oracle library (test infrastructure only).

Compiles oracle/vref.c into oracle/libvref.so with plain gcc flags: -O2, no
floating-point contraction (every sum rounded once, as written), OpenMP for the
optional block-parallel loop.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libvref.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "vref.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
