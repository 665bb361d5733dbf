"""The CPU oracle and the library's host side under AddressSanitizer and
UndefinedBehaviorSanitizer (no GPU needed).

* ``tests/sanitize/oracle_driver.c`` drives every oracle entry point (every
  power-of-two size to 2^16 in both directions, the single-precision entry,
  the chunked direct sum at lengths that are and are not powers of two, bins
  outside [0, N), rejected sizes and slices), built with gcc and both
  sanitizers, leak checking on.
* ``tests/sanitize/planner_driver.cpp`` drives the library's host code: the
  planner's dry run (``efft_schedule``) for every q <= 36, element type,
  placement and digit-buffer size, plan creation with valid and invalid
  arguments (valid ones fail cleanly at the first device allocation on a
  host without a GPU), chosen decompositions, every exec entry point with
  NULL and foreign handles, and the bandwidth reference's argument checks.
  Every library source is compiled with the sanitizers on its host side only
  (device code is not instrumented), and linked into the driver.

A sanitizer report or a wrong status fails the test."""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all"]

pytestmark = pytest.mark.slow


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed ({r.returncode}):\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_driver")
        _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "efft_oracle.c"),
              os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe, "-lm"])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
        r = _run([exe], env=env)
        assert "oracle driver ok" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_library_host_code_under_sanitizers():
    csrc = os.path.join(ROOT, "paper_1409_5757_amd", "csrc")
    sources = sorted(f for f in os.listdir(csrc) if f.endswith(".hip"))
    with tempfile.TemporaryDirectory() as tmp:
        flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                 "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument", *SAN,
                 "-I", os.path.join(ROOT, "include"), "-I", csrc]

        def compile_one(src):
            obj = os.path.join(tmp, src + ".o")
            _run([HIPCC, *flags, "-c", os.path.join(csrc, src), "-o", obj])
            return obj

        with ThreadPoolExecutor(max_workers=max(1, min(8, len(os.sched_getaffinity(0))))) as ex:
            objs = list(ex.map(compile_one, sources))
        drv = os.path.join(tmp, "driver.o")
        _run([HIPCC, *flags, "-c", os.path.join(ROOT, "tests", "sanitize", "planner_driver.cpp"), "-o", drv])
        exe = os.path.join(tmp, "planner_driver")
        _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
              "-fsanitize=undefined", *objs, drv, "-o", exe])
        # leak checking stays off here: the HIP runtime keeps process-lifetime
        # allocations of its own; the library's device-memory ownership is
        # checked on the GPU (plan create/destroy leaves device memory as it was)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
        r = _run([exe], env=env)
        assert "planner driver ok" in r.stdout
