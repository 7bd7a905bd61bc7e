"""Build the FP64 CPU oracle shared library (test infrastructure only).

Compiled with gcc, -O2, -ffp-contract=off and no fast-math, so that every
floating-point operation is rounded as written in the C source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "arlbm_oracle.c")
LIB = os.path.join(HERE, "libarlbm_oracle.so")


def build(verbose: bool = False) -> str:
    """Compile the oracle; always recompiles.  Returns the library path."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
