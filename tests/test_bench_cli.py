"""bench.py's command line on the host: runs on more than one GPU are refused
with a message, unknown workloads are rejected, and the workload table names
the configurations the benchmark measures (no GPU is touched)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_unknown_workload_is_rejected():
    r = _run("--workload", "c9")
    assert r.returncode == 2
    assert "invalid choice" in r.stderr


def test_workload_table():
    w = bench.OTHER_WORKLOADS
    assert sorted(w) == ["c1", "c2f32", "c3", "c4", "c5"]
    # (description, log2 N, dtype, in place, batch)
    assert (w["c1"][1], w["c1"][2], w["c1"][3], w["c1"][4]) == (20, "complex128", False, 1)
    assert (w["c3"][1], w["c3"][2], w["c3"][3], w["c3"][4]) == (32, "complex64", False, 1)
    assert (w["c4"][1], w["c4"][2], w["c4"][3], w["c4"][4]) == (34, "complex64", True, 1)
    assert (w["c5"][1], w["c5"][2], w["c5"][3], w["c5"][4]) == (24, "complex64", False, 64)
    assert (w["c2f32"][1], w["c2f32"][2], w["c2f32"][3], w["c2f32"][4]) == (30, "complex64", True, 1)


def test_roofline_fields():
    r = bench.roofline([2.0, 4.0, 1.0], 8e9)
    assert r["kernel_pass"] == 1 and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert abs(r["achieved"] - 2000.0) < 1e-9 and abs(r["frac"] - 0.25) < 1e-12
