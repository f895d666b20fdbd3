"""Build the oracle's shared library (test infrastructure only).

gcc, FP64, -O2 -ffp-contract=off (no fused multiply-add contraction, no
fast-math), OpenMP for the ring / m loops.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "fnl_oracle.c")]


def build(verbose=False):
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-std=c11", "-Wall", "-shared", "-fPIC", "-o", LIB + ".tmp"] + SRC + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built():
    """Return the library path, building it only if it is missing or older
    than its source."""
    if not os.path.exists(LIB) or any(os.path.getmtime(s) > os.path.getmtime(LIB) for s in SRC):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
