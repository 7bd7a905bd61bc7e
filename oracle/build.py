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
# the same source with OpenMP over rows (all-core timing; same bits)
LIB_OMP = os.path.join(HERE, "libarlbm_oracle_omp.so")


def build(verbose: bool = False) -> str:
    """Compile both builds of the oracle; always recompiles.  Returns the
    path of the single-threaded library."""
    common = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
              "-fPIC", "-shared", "-Wall", "-Wextra"]
    for out, extra in ((LIB, ["-Wno-unknown-pragmas"]), (LIB_OMP, ["-fopenmp"])):
        tmp = out + ".tmp"
        cmd = common + extra + ["-o", tmp, SRC, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
