"""bench.py's command line on the host: runs on more than one GPU are refused
with a message, unknown workloads are rejected, the workload table names the
configurations the benchmark measures, and the counted HBM traffic is
reported only for the kernel sources it was counted on (no GPU is touched)."""
import json
import os
import shutil
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


KERNEL_SOURCES = ("efft_kernels.hip", "efft_stage.hpp", "efft_device.hpp", "efft_internal.hpp", "efft_api.hip")


def test_traffic_is_reported_only_for_the_sources_it_was_counted_on(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1409_5757_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in KERNEL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_1409_5757_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = {"w": {"source_hash": bench.kernel_source_hash(), "passes": {"0": {"hbm_bytes": 123}}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_record("w", 0) == 123
    assert bench.traffic_record("w", 1) is None
    assert bench.traffic_record("other", 0) is None
    # any edit of a kernel source (a comment too) retires the record
    with open(csrc / "efft_stage.hpp", "a") as fh:
        fh.write("// edited\n")
    assert bench.traffic_record("w", 0) is None


def test_committed_traffic_records_cover_the_headline_kernel():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    for key in ("c128_inplace_fwd_q30", "c64_inplace_fwd_q30", "c64_oop_fwd_q32", "c64_inplace_fwd_inv_q34"):
        assert key in rec and rec[key]["passes"], key
        for p in rec[key]["passes"].values():
            assert p["hbm_bytes"] > 0
    # the headline's dominant pass moves its algorithmic bytes (2 N 16 B), to
    # within the counters' calibration
    assert rec["c128_inplace_fwd_q30"]["passes"]["0"]["hbm_bytes"] >= 0.99 * 2 * (1 << 30) * 16
