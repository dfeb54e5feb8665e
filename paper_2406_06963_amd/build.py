"""Builds libdhr.so (the HIP library behind include/dhr.h) for gfx950, in-tree.

hipcc cross-compiles without a GPU.  Packed-FP32 instructions are disabled
(``-packed-fp32-ops``) and floating-point contraction honours the source
pragmas, which the filter uses where a decision must be reproducible.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdhr.so")
SOURCES = ["api.cpp", "bvh_build.cpp", "trace.hip", "svgf.hip", "svgf_bwd.hip", "encode.hip", "bvh_device.hip", "raster.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


def flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-result",
            "-ffp-contract=fast-honor-pragmas", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(HERE, "..", "include")]


# Per-source additions.  trace.hip (the BVH walks): the control-flow
# structurizer leaves regions whose branches are all wave-uniform as they
# are.  The walk's decisions are ballots and scalar loads; structurised,
# each of them was carried as a 64-bit lane mask through flag blocks and
# re-tested, a third of the walk's scalar instructions.
SOURCE_FLAGS = {"trace.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]}


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object in parallel, then link the library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc()] + flags() + SOURCE_FLAGS.get(src, []) + lang + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append(src)
        if out.strip() and (verbose or p.returncode != 0):
            # the host pass warns that it does not know the packed-fp32 feature; keep the rest
            lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l]
            if lines:
                print("\n".join(lines), file=sys.stderr)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
