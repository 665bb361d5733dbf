#!/usr/bin/env python3
"""Throughput of one enormous in-memory 1D complex FFT on one MI355X.

Workload (default): forward in-place transform of N = 2^30 complex128 points
(16 GiB), inputs i.i.d. uniform [-1, 1) per component from a seed, already
resident in HBM.  A step is one whole transform (every pass of the plan).
Reports GFLOP/s = 5 N log2 N / t (the nominal complex-FFT count; the paper's
Eq. "eqflops" is the real-input half of it), per-pass HBM bandwidth from HIP
events recorded on the launch stream inside the timed region, the same
transform in complex64 for the FP32 speedup and its error against the FP64
path, the paper's own real-input FP32 transform at the same N, the other
workloads (2^20 complex128 out of place, 2^32 complex64 out of place, 2^34
complex64 forward + inverse in place, 64 x 2^24 complex64 through autograd)
under "other_workloads", a device-copy ceiling, and the FP64 CPU oracle timed
on a bounded sample on the host cores.

    python bench.py [--steps K] [--warmup W] [--log2n Q] [--no-fp32] [--no-real] [--no-cpu] [--no-others]
    python bench.py --workload c1|c3|c4|c5    # the other workloads, one line each:
        c1 2^20 complex128 out of place; c3 2^32 complex64 out of place;
        c4 2^34 complex64 in place, forward + inverse; c5 64 x 2^24 complex64
        forward + loss + adjoint backward through autograd; c2f32 the default
        transform in complex64 alone
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
METRIC = "1D C2C FFT GFLOP/s (5N·log2N/t) + HBM GB/s % peak, FP64 vs FP32"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("efft_kernels.hip", "efft_stage.hpp", "efft_device.hpp", "efft_internal.hpp", "efft_api.hip"):
        with open(os.path.join(ROOT, "paper_1409_5757_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(workload_key: str, pass_index: int):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    entry = rec.get(workload_key, {})
    if entry.get("source_hash") != kernel_source_hash():
        return None
    p = entry.get("passes", {}).get(str(pass_index))
    return None if p is None else p.get("hbm_bytes")


def time_transform(plan, x, steps: int, warmup: int, scratch=None, out=None):
    """Warm up, then time exactly `steps` transforms (in place, or into `out`
    for out-of-place plans); per-pass event times."""
    import torch
    out = x if out is None else out
    for _ in range(warmup):
        if plan.inplace:
            plan.execute(x, scratch=scratch)
        else:
            plan.execute(x, out=out)
    torch.cuda.synchronize()
    npass = plan.passes if scratch is None else plan.scratch_passes
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(npass + 1)] for _ in range(steps)]
    for row in evs:  # materialise every hipEvent before the timed region
        for e in row:
            e.record()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for row in evs:
        plan.execute_events(x, out, [e.cuda_event for e in row], scratch=scratch)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_pass = [sum(row[i].elapsed_time(row[i + 1]) for row in evs) / steps for i in range(npass)]
    event_step = sum(row[0].elapsed_time(row[-1]) for row in evs) / steps
    return wall / steps * 1e3, event_step, per_pass


def copy_ceiling(nbytes: int) -> tuple[float, float]:
    """Device-to-device copy bandwidth (read + write) in GB/s: the library's
    streaming copy (the STREAM-style reference, 16-byte non-temporal accesses
    like the transform's passes; the better of a copy into a second array and
    an in-place rewrite) and torch's copy kernel (which is also the
    calibration of the HBM byte counters: known bytes per launch)."""
    import ctypes
    import torch
    from paper_1409_5757_amd import _lib
    lib = _lib.load()
    n = nbytes // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def lib_copy(dst):
        _lib.check(lib.efft_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                                        n * 8, s), "efft_stream_copy")

    out = []
    for copy in (lambda: lib_copy(b), lambda: lib_copy(a), lambda: b.copy_(a)):
        copy()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            copy()
        e1.record()
        torch.cuda.synchronize()
        out.append(2 * n * 8 / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9)
    if not torch.equal(a, b):
        raise RuntimeError("copy check failed")
    del a, b
    torch.cuda.empty_cache()
    return max(out[0], out[1]), out[2]


def calibration_copy() -> None:
    """One elementwise torch kernel over 2^26 doubles (torch.neg: 512 MiB read
    + 512 MiB written, contiguous): the kernel of known traffic whose
    FETCH_SIZE / WRITE_SIZE readings scale the counters of the transform's
    passes."""
    import torch
    a = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b
    torch.cuda.empty_cache()


def cpu_baseline(budget_s: float = 12.0):
    """The FP64 oracle (radix-2, OpenMP) on 2^24-point transforms, repeated
    until the budget is used; GFLOP/s by the same 5 N log2 N count."""
    import numpy as np
    import oracle
    from paper_1409_5757_amd import inputs
    q = 24
    n = 1 << q
    x = inputs.generate("uniform", 0, n)
    lib = oracle.load()
    reps, t_total = 0, 0.0
    while t_total < budget_s and reps < 50:
        t0 = time.perf_counter()
        oracle.fft(x, -1, lib=lib)
        t_total += time.perf_counter() - t0
        reps += 1
    per = t_total / reps
    out = {"value": round(5 * n * q / per / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.threads(lib),
           "kind": "oracle",
           "sample": f"{reps} forward transforms of N=2^{q} complex128 (uniform [-1,1)), "
                     f"{per:.2f} s each; same 5N log2N count"}
    # the same oracle on one thread at 2^20 and 2^24 (OpenMP thread count set
    # through the runtime the oracle library uses)
    try:
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return out
    gomp.omp_set_num_threads(1)
    single = []
    for q1, reps1 in ((20, 3), (24, 1)):
        x1 = x[:1 << q1].copy()
        t0 = time.perf_counter()
        for _ in range(reps1):
            oracle.fft(x1, -1, lib=lib)
        per1 = (time.perf_counter() - t0) / reps1
        single.append({"value": round(5 * (1 << q1) * q1 / per1 / 1e9, 3), "unit": "GFLOP/s",
                       "sample": f"{reps1} transform(s) of N=2^{q1}, {per1 * 1e3:.1f} ms each"})
    gomp.omp_set_num_threads(out["cores"])
    out["single_thread"] = single
    return out


# The other workloads: name -> (description, log2 N, dtype name, in place, batch)
OTHER_WORKLOADS = {
    "c1": ("forward out-of-place 1D C2C FFT, N=2^20 complex128 (16 MiB), uniform [-1,1) inputs in HBM",
           20, "complex128", False, 1),
    "c3": ("forward out-of-place 1D C2C FFT, N=2^32 complex64 (32 GiB in, 32 GiB out), "
           "standard normal inputs in HBM", 32, "complex64", False, 1),
    "c4": ("forward then inverse in-place 1D C2C FFT, N=2^34 complex64 (128 GiB), uniform [-1,1) "
           "inputs in HBM; a step is both transforms", 34, "complex64", True, 1),
    "c5": ("64 signals of N=2^24 complex64 (8 GiB): y = FFT(x) through autograd, loss = sum |w*y - t|^2, "
           "backward through the hand-written adjoint; a step is forward + loss + backward",
           24, "complex64", False, 64),
    # the FP32 companion of the default workload on its own (what the HBM
    # byte counters of its passes are taken on)
    "c2f32": ("forward in-place 1D C2C FFT, N=2^30 complex64 (8 GiB), uniform [-1,1) inputs in HBM",
              30, "complex64", True, 1),
}


def roofline(per_pass, bytes_pass):
    dom = max(range(len(per_pass)), key=lambda i: per_pass[i])
    achieved = bytes_pass / (per_pass[dom] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": None, "kernel_pass": dom}


# records of profiles/traffic.json taken on the other workloads' passes
TRAFFIC_KEYS = {"c2f32": "c64_inplace_fwd_q30", "c3": "c64_oop_fwd_q32", "c4": "c64_inplace_fwd_inv_q34"}


def run_other(args) -> int:
    """One JSON line for workload c1, c2f32, c3, c4 or c5 (same keys as the
    default line)."""
    result = measure_other(args.workload, args.steps, args.warmup)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)
    return 0


def measure_other(workload: str, steps: int, warmup: int) -> dict:
    """Measure workload c1, c2f32, c3, c4 or c5 (per-pass times from the
    library's events on the launch stream); the arrays are freed on return."""
    import types
    import torch
    from paper_1409_5757_amd import _lib, api, inputs

    args = types.SimpleNamespace(workload=workload, steps=steps, warmup=warmup)
    _lib.load()
    label, q, dtn, inplace, batch = OTHER_WORKLOADS[args.workload]
    dt = getattr(torch, dtn)
    eb = 16 if dt == torch.complex128 else 8
    n = 1 << q
    dev = torch.device("cuda", 0)
    bytes_pass = 2 * batch * n * eb
    x = torch.empty((batch, n) if batch > 1 else (n,), dtype=dt, device=dev)
    if args.workload == "c3":
        inputs.fill_normal_torch(x, seed=0)
    elif batch == 1:
        inputs.fill_uniform_torch(x, seed=0)
    flops = 5 * batch * n * q
    extra = {}
    if args.workload == "c2f32":
        plan = api.Plan(n, dt, -1, True, device=dev)
        ms_step, _, per_pass = time_transform(plan, x, args.steps, args.warmup)
        plan.close()
    elif args.workload in ("c1", "c3"):
        plan = api.Plan(n, dt, -1, False, device=dev)
        y = torch.empty_like(x)
        ms_step, _, per_pass = time_transform(plan, x, args.steps, args.warmup, out=y)
        if args.workload == "c1":
            # launch-bound: the same transform captured once in a HIP graph
            # and replayed (no host launch cost per kernel)
            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream(dev)
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                with torch.cuda.graph(g, stream=s):
                    plan.execute(x, out=y)
            torch.cuda.current_stream().wait_stream(s)
            g.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                g.replay()
            torch.cuda.synchronize()
            gms = (time.perf_counter() - t0) / args.steps * 1e3
            extra = {"graph_replay": {"ms_per_step": round(gms, 4),
                                      "value": round(flops / (gms * 1e-3) / 1e9, 2), "unit": "GFLOP/s"}}
        plan.close()
    elif args.workload == "c4":
        # forward, then the inverse (backward direction scaled by 2^-q, exact)
        # (each step restores the data, so repeated steps stay in range)
        pf = api.Plan(n, dt, -1, True, device=dev)
        pi = api.Plan(n, dt, +1, True, scale=2.0 ** -q, device=dev)
        for _ in range(args.warmup):
            pf.execute(x)
            pi.execute(x)
        torch.cuda.synchronize()
        ev = [[[torch.cuda.Event(enable_timing=True) for _ in range(p.passes + 1)] for p in (pf, pi)]
              for _ in range(args.steps)]
        for row in ev:
            for e in row[0] + row[1]:
                e.record()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for row in ev:
            pf.execute_events(x, x, [e.cuda_event for e in row[0]])
            pi.execute_events(x, x, [e.cuda_event for e in row[1]])
        torch.cuda.synchronize()
        ms_step, flops = (time.perf_counter() - t0) / args.steps * 1e3, 2 * flops
        per_pass = [sum(r[d][i].elapsed_time(r[d][i + 1]) for r in ev) / args.steps
                    for d, p in enumerate((pf, pi)) for i in range(p.passes)]
        extra = {"forward_ms": round(sum(r[0][0].elapsed_time(r[0][-1]) for r in ev) / args.steps, 3),
                 "inverse_ms": round(sum(r[1][0].elapsed_time(r[1][-1]) for r in ev) / args.steps, 3)}
        pf.close()
        pi.close()
    else:
        yt = torch.empty_like(x)
        w = torch.empty(batch, n, dtype=torch.float32, device=dev)
        for b in range(batch):
            inputs.fill_normal_torch(x[b], seed=1000 + b)
            inputs.fill_normal_torch(yt[b], seed=2000 + b)
            inputs.fill_weights_torch(w[b], seed=3000 + b)
        x.requires_grad_(True)

        def step():
            x.grad = None
            f = api.fft(x)
            torch.view_as_real(w * f - yt).pow(2).sum().backward()

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms_step, flops = (time.perf_counter() - t0) / args.steps * 1e3, 2 * flops
        # per-pass times of the batched forward plan the step uses
        pf = api.get_plan(n, dt, -1, False, 1.0, dev, batch)
        xd = x.detach()
        _, _, per_pass = time_transform(pf, xd, args.steps, 1, out=torch.empty_like(xd))
        fft_ms = sum(per_pass)
        extra = {"transforms_per_step": 2, "forward_plan_ms_per_pass": [round(t, 4) for t in per_pass],
                 # the transforms alone (the rest of a step is the loss and its
                 # gradient, computed by torch): one batched transform's time
                 # and its rate by the same 5 N log2 N count
                 "fft_ms_per_direction": round(fft_ms, 4),
                 "fft_GFLOPs": round(5 * batch * n * q / (fft_ms * 1e-3) / 1e9, 2)}
    result = {
        "metric": METRIC, "value": round(flops / (ms_step * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if eb == 16 else "f32", "data": "synthetic",
        "config": {"workload": label, "log2n": q, "batch": batch, "inplace": inplace,
                   "digits_log2": _lib.schedule(n, 2 if eb == 16 else 1, inplace)[0]},
        "roofline": roofline(per_pass, bytes_pass),
        "passes_detail": [{"pass": i, "ms": round(t, 4), "GBps": round(bytes_pass / (t * 1e-3) / 1e9, 1)}
                          for i, t in enumerate(per_pass)],
        **extra,
    }
    if workload in TRAFFIC_KEYS:
        result["roofline"]["traffic"] = traffic_record(TRAFFIC_KEYS[workload], result["roofline"]["kernel_pass"])
    del x
    torch.cuda.empty_cache()
    return result


# The other workloads measured by the default run, with their step counts
# (steps, warmup), so that one run of bench.py reports every workload.  The
# 2^20 transform takes about 40 us, so it runs 200 steps: the fixed cost of
# starting and synchronising the timed loop is then a small part of a step.
COMPANIONS = {"c1": (200, 20), "c3": (5, 1), "c4": (2, 1), "c5": (3, 1)}


def companion(r: dict) -> dict:
    """The part of a workload's line that the default line carries."""
    keep = ("value", "unit", "ms_per_step", "steps", "warmup", "dtype", "graph_replay", "forward_ms",
            "inverse_ms", "fft_ms_per_direction", "fft_GFLOPs")
    out = {"workload": r["config"]["workload"], "digits_log2": r["config"]["digits_log2"]}
    out.update({k: r[k] for k in keep if k in r})
    rf = r["roofline"]
    out["dominant_pass"] = {"pass": rf["kernel_pass"], "GBps": rf["achieved"], "frac_of_hbm_peak": rf["frac"]}
    out["ms_per_pass"] = [p["ms"] for p in r["passes_detail"]]
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=30)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-real", action="store_true")
    ap.add_argument("--no-anylen", action="store_true")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the other workloads (c1, c3, c4, c5) that the default run also measures")
    ap.add_argument("--workload", choices=sorted(OTHER_WORKLOADS) + ["c2"], default="c2",
                    help="c2 (default): the in-place 2^30 complex128 transform with its companions; "
                         "c1, c3, c4, c5, c2f32: the other workloads, one JSON line each")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run one elementwise torch kernel over 512 MiB (the kernel of known "
                         "traffic that scales the HBM byte counters) before the workload")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one transform on one GPU; runs on more than one GPU are not "
              "part of this benchmark (use --gpus 1)", file=sys.stderr)
        return 2
    if args.calibrate:
        calibration_copy()
    if args.workload != "c2":
        return run_other(args)

    import torch
    from paper_1409_5757_amd import _lib, api, inputs

    _lib.load()  # fails loudly if the library is missing
    q = args.log2n
    n = 1 << q
    dev = torch.device("cuda", 0)
    x = torch.empty(n, dtype=torch.complex128, device=dev)
    inputs.fill_uniform_torch(x, seed=0)
    plan = api.Plan(n, torch.complex128, -1, True, device=dev)
    digits, passes = _lib.schedule(n, 2, True)
    ms_step, ms_events, per_pass = time_transform(plan, x, args.steps, args.warmup)
    gflops = 5 * n * q / (ms_step * 1e-3) / 1e9
    bytes_pass = 2 * n * 16
    dom = max(range(len(per_pass)), key=lambda i: per_pass[i])
    achieved = bytes_pass / (per_pass[dom] * 1e-3) / 1e9
    workload_key = f"c128_inplace_fwd_q{q}"
    traffic = traffic_record(workload_key, dom)
    passes_out = [{"pass": i, "ms": round(t, 4), "GBps": round(bytes_pass / (t * 1e-3) / 1e9, 1)}
                  for i, t in enumerate(per_pass)]

    result = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"forward in-place 1D C2C FFT, N=2^{q} complex128 "
                               f"({n * 16 / 2**30:.0f} GiB), uniform [-1,1) inputs in HBM",
                   "log2n": q, "inplace": True, "digits_log2": digits, "passes": passes},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
                     "traffic": traffic, "kernel_pass": dom},
        "hbm_GBps_whole_transform": round(passes * bytes_pass / (ms_events * 1e-3) / 1e9, 1),
        # the paper's memory metric (Section 5.3): device memory of the
        # transform = the array itself + the plan's tables
        "memory": {"array_bytes": n * 16, "plan_bytes": plan.device_bytes(),
                   "peak_allocated_bytes": int(torch.cuda.max_memory_allocated(dev))},
        "passes_detail": passes_out,
    }
    # the same plan with a scratch array of N elements (one pass fewer, 2x memory)
    scratch = plan.make_scratch()
    ms_s, ev_s, pp_s = time_transform(plan, x, args.steps, args.warmup, scratch=scratch)
    result["with_scratch"] = {
        "workload": f"same transform, in place with a caller-provided scratch array of N elements "
                    f"({n * 16 / 2**30:.0f} GiB)",
        "value": round(5 * n * q / (ms_s * 1e-3) / 1e9, 2), "unit": "GFLOP/s", "ms_per_step": round(ms_s, 4),
        "passes": plan.scratch_passes,
        "passes_detail": [{"pass": i, "ms": round(t, 4), "GBps": round(bytes_pass / (t * 1e-3) / 1e9, 1)}
                          for i, t in enumerate(pp_s)]}
    del x, scratch
    torch.cuda.empty_cache()

    if not args.no_fp32:
        x32 = torch.empty(n, dtype=torch.complex64, device=dev)
        inputs.fill_uniform_torch(x32, seed=0)
        p32 = api.Plan(n, torch.complex64, -1, True, device=dev)
        ms32, ev32, pp32 = time_transform(p32, x32, args.steps, args.warmup)
        # error of the FP32 path against the FP64 path on the same input
        inputs.fill_uniform_torch(x32, seed=1)
        x64 = x32.to(torch.complex128)
        p32.execute(x32)
        plan.execute(x64)
        torch.cuda.synchronize()
        diff = (x32.to(torch.complex128) - x64)
        rel = (torch.linalg.vector_norm(diff) / torch.linalg.vector_norm(x64)).item()
        mabs = diff.abs().max().item()
        del diff, x64
        result["fp32"] = {
            "workload": f"forward in-place N=2^{q} complex64", "value": round(5 * n * q / (ms32 * 1e-3) / 1e9, 2),
            "unit": "GFLOP/s", "ms_per_step": round(ms32, 4), "speedup_vs_fp64": round(ms_step / ms32, 3),
            "rel_l2_vs_fp64_path": rel, "max_abs_vs_fp64_path": mabs,
            "passes_detail": [{"pass": i, "ms": round(t, 4), "GBps": round(2 * n * 8 / (t * 1e-3) / 1e9, 1)}
                              for i, t in enumerate(pp32)]}
        del x32
        torch.cuda.empty_cache()

    if not args.no_real:
        # the paper's own workload: a real FP32 transform, GFLOP/s by its
        # real-data count 2.5 N log2 N (Eq. "eqflops")
        xr = torch.empty(n // 2, dtype=torch.complex64, device=dev)
        inputs.fill_uniform_torch(xr, seed=0, lo=-0.5, hi=0.5)
        xr = torch.view_as_real(xr).reshape(n)
        pr = api.RealPlan(n, torch.float32, -1, 1.0, device=dev)
        yr = torch.empty(n // 2 + 1, dtype=torch.complex64, device=dev)
        for _ in range(args.warmup):
            pr.execute(xr, yr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pr.execute(xr, yr)
        torch.cuda.synchronize()
        msr = (time.perf_counter() - t0) / args.steps * 1e3
        result["real_fp32"] = {"workload": f"forward real-to-complex N=2^{q} float32, out of place",
                               "value": round(2.5 * n * q / (msr * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
                               "count": "2.5 N log2 N", "ms_per_step": round(msr, 4),
                               "passes": pr.passes}
        del xr, yr
        pr.close()
        torch.cuda.empty_cache()

    if not args.no_anylen:
        # lengths that are not powers of two (the paper's N = M * 2^s class):
        # N = 3 * 2^(q-2) takes one radix-3 pass, the power-of-two passes of
        # the 2^(q-2)-point rows, the last written interleaved into the output;
        # N = 2^(q-2) + 1 (no small odd factor) takes the chirp path.  GFLOP/s
        # by the same nominal 5 N log2 N.
        for name, na, label in (("small_odd_factor", 3 << (q - 2),
                                 f"forward in-place N=3*2^{q - 2} complex128 (radix-3 pass, then the 2^{q - 2}-point rows, the last pass interleaving them)"),
                                ("any_length", (1 << (q - 2)) + 1,
                                 f"forward in-place N=2^{q - 2}+1 complex128 (chirp path)")):
            xa = torch.empty(na, dtype=torch.complex128, device=dev)
            inputs.fill_uniform_torch(xa, seed=0)
            pa = api.Plan(na, torch.complex128, -1, True, device=dev)
            msa, eva, ppa = time_transform(pa, xa, max(2, args.steps // 2), 1)
            result[name] = {"workload": label,
                            "value": round(5 * na * math.log2(na) / (msa * 1e-3) / 1e9, 2), "unit": "GFLOP/s",
                            "ms_per_step": round(msa, 4), "passes": pa.passes,
                            "ms_per_pass": [round(t, 4) for t in ppa]}
            del xa
            pa.close()
            torch.cuda.empty_cache()

    if not args.no_others:
        result["other_workloads"] = {name: companion(measure_other(name, st, wu))
                                     for name, (st, wu) in COMPANIONS.items()}

    stream_gbps, torch_gbps = copy_ceiling(min(8 << 30, n * 16))
    result["copy_ceiling_GBps"] = round(stream_gbps, 1)  # efft_stream_copy
    result["torch_copy_GBps"] = round(torch_gbps, 1)
    result["roofline"]["frac_of_copy_ceiling"] = round(achieved / stream_gbps, 4)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
