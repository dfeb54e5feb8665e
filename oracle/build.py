"""Build the CPU oracle shared library (test infrastructure only).

g++ -O2 with OpenMP, no fast-math and no floating-point contraction, so the
FP64 arithmetic and the fp32 decision arithmetic are exactly what the source
says.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_rng.cpp", "orc_geom.cpp", "orc_render.cpp", "orc_svgf.cpp", "orc_svgf_adjoint.cpp", "orc_encode.cpp"]
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
