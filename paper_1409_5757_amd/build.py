"""Build the gfx950 shared library ``libefft.so`` in place with hipcc.

Run as ``python -m paper_1409_5757_amd.build``; ``__graft_entry__.build()``
calls :func:`build_library`.  The library is compiled for gfx950 only.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libefft.so")
SOURCES = ["efft_api.hip", "efft_kernels.hip", "efft_real.hip", "efft_bluestein.hip", "efft_mixed.hip",
           "efft_stream.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code: the compiler
# still vectorises, but never emits the packed forms.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build_library(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs,
           "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build_library(verbose="-v" in sys.argv)
    print(LIB)
