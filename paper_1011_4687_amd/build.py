"""Compile the gfx950 library ``libenvpot.so`` in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with packed FP32 instructions
disabled (-packed-fp32-ops): the kernels are written as scalar FP32/FP64 code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libenvpot.so")

SOURCES = ["kernels.hip", "pairlist.cpp", "layout.cpp", "api.cpp", "batch.cpp", "surrogate.hip", "surrogate.cpp",
           "probe.hip", "cells.hip", "cells.cpp", "field.hip", "field.cpp",
           "server.cpp", "update.hip", "update.cpp", "sortpts.hip"]

HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def generate() -> None:
    """Regenerate hermite_gen.h (gen_hermite.py) and field_gen.h (gen_field.py)."""
    for gen, header in (("gen_hermite.py", "hermite_gen.h"), ("gen_field.py", "field_gen.h")):
        out = subprocess.run([sys.executable, os.path.join(CSRC, gen)],
                             check=True, capture_output=True, text=True).stdout
        path = os.path.join(CSRC, header)
        old = open(path).read() if os.path.exists(path) else None
        if old != out:
            with open(path, "w") as f:
                f.write(out)


def build(verbose: bool = False, extra=None) -> str:
    generate()
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIP_FLAGS + ["-shared", "-I", INCLUDE, "-I", CSRC]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    cmd += list(extra or []) + ["-o", tmp, "-lpthread", "-lrt"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
