"""Build libwfsthip.so (gfx950) in-tree.

The HIP translation unit (kernels + C ABI) is compiled with hipcc for gfx950;
the host layout builder is plain C++.  Packed-FP32 instruction selection is
switched off and FP32 denormals are kept (no flush), so that every Viterbi
candidate is one IEEE binary32 round-to-nearest-even addition.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libwfsthip.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("WFST_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-flush-denormals-to-zero", "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), file=sys.stderr, flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    os.makedirs(BUILD, exist_ok=True)
    lay_o = os.path.join(BUILD, "layout.o")
    att_o = os.path.join(BUILD, "att.o")
    api_o = os.path.join(BUILD, "wfst_api.o")
    _run(["g++", "-O3", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wextra", "-I", INCLUDE,
          "-c", os.path.join(CSRC, "layout.cpp"), "-o", lay_o], verbose)
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-I", INCLUDE,
          "-c", os.path.join(CSRC, "att.cpp"), "-o", att_o], verbose)
    _run([hipcc, *HIP_FLAGS, "-I", INCLUDE, "-c", os.path.join(CSRC, "wfst_api.hip"), "-o", api_o], verbose)
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, api_o, lay_o, att_o, "-pthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
