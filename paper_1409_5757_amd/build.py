"""Build the gfx950 shared library ``libefft.so`` in place with hipcc.

Run as ``python -m paper_1409_5757_amd.build``; ``__graft_entry__.build()``
calls :func:`build_library`.  The library is compiled for gfx950 only.  Each
source is compiled to an object of its own (in parallel), then the objects
are linked; ``extra_flags`` adds compiler flags (e.g. ``-D`` settings of the
tuning macros in ``csrc/efft_internal.hpp``), ``out`` another output path.
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
LIB = os.path.join(PKG, "libefft.so")
SOURCES = ["efft_api.hip", "efft_kernels.hip", "efft_stage_f64_lo.hip", "efft_stage_f64_hi.hip",
           "efft_stage_f32_lo.hip", "efft_stage_f32_hi.hip", "efft_real.hip", "efft_bluestein.hip", "efft_mixed.hip",
           "efft_stream.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code: the compiler
# still vectorises, but never emits the packed forms.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build_library(verbose: bool = False, extra_flags=(), out: str | None = None, csrc: str = CSRC) -> str:
    out = out or LIB
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    with tempfile.TemporaryDirectory(prefix="efft_build_") as tmp:
        def compile_one(src: str) -> str:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            cmd = [HIPCC, *FLAGS, *extra_flags, *inc, "-c", os.path.join(csrc, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            return obj

        jobs = max(1, min(len(SOURCES), len(os.sched_getaffinity(0)), 16))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        cmd = [HIPCC, *FLAGS, "-shared", *objs, "-o", out + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build_library(verbose="-v" in sys.argv)
    print(LIB)
