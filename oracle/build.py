"""Build the FP64 oracle shared library (test infrastructure).

gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp: IEEE double, no FMA
contraction, so every sum and product rounds exactly as written.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle_mevp.so")
SRC = os.path.join(HERE, "mevp_oracle.c")


FLAGS = ["-std=c99", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
         "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False, src: str = SRC, lib: str = LIB, extra=()) -> str:
    """Compile ``src`` (default: the oracle) to ``lib`` with the oracle's flags."""
    cmd = ["gcc"] + FLAGS + list(extra) + ["-I", HERE, "-o", lib + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
