"""Build the gfx950 shared library libbura.so in-tree with hipcc.

Usage: python -m paper_1612_04846_amd.build   (or call build()).
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbura.so")
HIP_SOURCES = ["bura_kernels.hip", "bura_engine.cpp", "bura_server.cpp"]
HOST_SOURCES = ["bura_remez.cpp", "bura_sinc.cpp"]   # plain C++ (Remez in __float128; quadrature), built by g++

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd[:2]))


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for s in HOST_SOURCES:
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        _run(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c", os.path.join(CSRC, s), "-o", obj], verbose)
        objs.append(obj)
    srcs = [os.path.join(CSRC, s) for s in HIP_SOURCES]
    tmp = LIB + ".tmp"
    _run([HIPCC] + FLAGS + ["-o", tmp, "-x", "hip"] + srcs + ["-x", "none"] + objs + ["-lquadmath"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
