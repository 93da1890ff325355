"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle_su2.so.

Plain gcc with OpenMP; no HIP, no code shared with the GPU library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "su2_oracle.c")
LIB = os.path.join(HERE, "liboracle_su2.so")


def build(verbose: bool = False) -> str:
    """Compile the oracle shared library and return its path."""
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
        "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    """Build only when the library is missing or older than its source."""
    if (not os.path.exists(LIB)
            or os.path.getmtime(LIB) < os.path.getmtime(SRC)
            or os.path.getmtime(LIB) < os.path.getmtime(os.path.join(HERE, "su2_oracle.h"))):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
