"""Build the FP64 CPU oracle (test infrastructure only) into oracle/libgamer_oracle.so.

Plain gcc, -O2 with floating-point contraction off and no fast-math, OpenMP
over independent groups.  Run as a script or call ``build()``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gamer_oracle.c")
SRCS = [SRC, os.path.join(HERE, "gamer_rtvd.c"), os.path.join(HERE, "gamer_ctu.c")]
LIB = os.path.join(HERE, "libgamer_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, *SRCS, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
