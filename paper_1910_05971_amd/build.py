"""Compile the native parts in-tree.

* ``_lib/libfastsv.so``      -- HIP kernels + C ABI for gfx950 (hipcc)
* ``_lib/libfastsv_gen.so``  -- seeded graph generators (gcc, OpenMP)

Run ``python -m paper_1910_05971_amd.build`` or ``__graft_entry__.build()``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
INCLUDE = os.path.join(ROOT, "include")

HIP_LIB = os.path.join(LIBDIR, "libfastsv.so")
GEN_LIB = os.path.join(LIBDIR, "libfastsv_gen.so")

HIP_SOURCES = ["fastsv.hip", "server.hip"]

# Packed-FP32 instructions are switched off for all device code; the solver
# itself is integer-only, the flag keeps any float helper scalar.
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _atomic_out(path):
    return path + ".tmp"


def build_gen():
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = _atomic_out(GEN_LIB)
    _run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-std=c11",
          os.path.join(CSRC, "graphgen.c"), "-o", tmp, "-lm"])
    os.replace(tmp, GEN_LIB)


def build_hip():
    os.makedirs(LIBDIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = _atomic_out(HIP_LIB)
    _run([hipcc, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, *[os.path.join(CSRC, s) for s in HIP_SOURCES],
          "-o", tmp])
    os.replace(tmp, HIP_LIB)


def build_all():
    build_gen()
    if all(os.path.exists(os.path.join(CSRC, s)) for s in HIP_SOURCES):
        build_hip()


if __name__ == "__main__":
    what = sys.argv[1:] or ["all"]
    for w in what:
        {"gen": build_gen, "hip": build_hip, "all": build_all}[w]()
