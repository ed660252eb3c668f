"""Compile the gfx950 library ``libenvpot.so`` in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with packed FP32 instructions
disabled (-packed-fp32-ops): the kernels are written as scalar FP32/FP64 code.
Sources are compiled to objects in parallel (one hipcc per source) and then
linked; every call compiles every source again.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libenvpot.so")

SOURCES = ["kernels.hip", "pairlist.cpp", "layout.cpp", "api.cpp", "batch.cpp", "surrogate.hip", "surrogate.cpp",
           "probe.hip", "cells.hip", "cells.cpp", "field.hip", "field.cpp",
           "server.cpp", "update.hip", "update.cpp", "sortpts.hip", "hosteval.cpp", "noalloc.hip", "devbuild.hip"]

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


def _jobs() -> int:
    for k in ("MAX_JOBS", "CMAKE_BUILD_PARALLEL_LEVEL"):
        v = os.environ.get(k)
        if v and v.isdigit() and int(v) > 0:
            return min(int(v), 16)
    return min(os.cpu_count() or 1, 16)


def build(verbose: bool = False, extra=None) -> str:
    generate()
    extra = list(extra or [])
    with tempfile.TemporaryDirectory(prefix="envpot_build_") as tmpd:
        def compile_one(src):
            obj = os.path.join(tmpd, src.replace(".", "_") + ".o")
            cmd = [hipcc()] + HIP_FLAGS + ["-c", "-I", INCLUDE, "-I", CSRC, os.path.join(CSRC, src)] + extra
            cmd += ["-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            return src, obj, r

        with ThreadPoolExecutor(max_workers=_jobs()) as ex:
            results = list(ex.map(compile_one, SOURCES))
        failed = [(s, r) for s, _, r in results if r.returncode != 0]
        for s, _, r in results:
            # hipcc's host pass warns about the device-only feature flag; keep the rest
            msg = "\n".join(ln for ln in (r.stdout + r.stderr).splitlines()
                            if "packed-fp32-ops" not in ln)
            if msg.strip() and (verbose or r.returncode != 0):
                print(f"--- {s}\n{msg}", file=sys.stderr, flush=True)
        if failed:
            raise subprocess.CalledProcessError(failed[0][1].returncode, f"hipcc {failed[0][0]}")
        tmp = LIB + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for _, o, _ in results]
        cmd += ["-o", tmp, "-lpthread", "-lrt"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
