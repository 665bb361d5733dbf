"""Measured choice of a transform's decomposition and per-pass launch options.

The paper tunes EFFT by scanning its two parameters, the number of splits
and the number of workers, and keeping the fastest point for each size
(Section 5.2, Fig. "fig:heatmap").  The GPU counterparts are the digit
decomposition N = 2^d_0 ... 2^d_{m-1} (``efft_plan_digits``) and, for each
pass, the lines per workgroup, line sets, tile order and non-temporal hints
(``efft_set_pass_options``).  The launch options never change the
arithmetic (every setting gives bit-identical results); another
decomposition computes the same DFT with a different rounding pattern, within
the same error bound.

``tune(n, dtype, inplace)`` times candidate decompositions and, for each, the
launch options of every pass (one pass at a time, the others held), and
returns a wisdom entry; ``save``/``load`` keep entries in a JSON file keyed by
size, dtype, placement, batch, schedule and device; ``plan(...)`` builds a
plan from an entry.

    python -m paper_1409_5757_amd.tune --log2n 30 --dtype c128 --inplace --out wisdom.json
"""
from __future__ import annotations

import argparse
import ctypes
import itertools
import json
import os
import sys

import torch

from . import _lib, api, inputs
from ._lib import EFFT_FORWARD, EfftError

_DT = {"c64": torch.complex64, "c128": torch.complex128}
_DT_NAME = {v: k for k, v in _DT.items()}
_DT_CODE = {torch.complex64: _lib.EFFT_C64, torch.complex128: _lib.EFFT_C128}

LINE_CHOICES = (1, 2, 4, 8, 16, 32, 64, 128, 256)
HINT_CHOICES = ((0, 0), (0, 1), (1, 1))


def key(n: int, dtype: torch.dtype, inplace: bool, batch: int = 1, scratch: bool = False,
        device: torch.device | None = None) -> str:
    dev = torch.cuda.get_device_name(device or 0).replace("/", "_")
    return (f"{n}/{_DT_NAME[dtype]}/{'inplace' if inplace else 'oop'}/b{batch}/"
            f"{'scratch' if scratch else 'plain'}/{dev}")


def decompositions(q: int, inplace: bool, max_digits: int = 4, max_digit: int = 12) -> list[list[int]]:
    """Decompositions the strided kernels can run: digits in [4, max_digit]
    (at most 12; or one digit q <= 12), palindromic for in-place plans, at
    most max_digits."""
    if q <= 12:
        return [[q]]
    out = []
    for m in range(2, max_digits + 1):
        for d in itertools.product(range(4, min(max_digit, 12) + 1), repeat=m):
            if sum(d) == q and (not inplace or d == d[::-1]):
                out.append(list(d))
    # fewest passes first, then the most balanced (the planner's own preference)
    out.sort(key=lambda d: (len(d), max(d) - min(d), d))
    return out


def _options(plan: api.Plan, scratch: bool, i: int) -> list[int]:
    buf = (ctypes.c_int * 6)()
    _lib.check(plan.lib.efft_pass_options(plan.handle, int(scratch), i, buf), "efft_pass_options")
    return list(buf)


def _set_options(plan: api.Plan, scratch: bool, i: int, opts) -> bool:
    buf = (ctypes.c_int * 6)(*opts)
    return plan.lib.efft_set_pass_options(plan.handle, int(scratch), i, buf) == 0


def make_plan(n: int, dtype: torch.dtype, inplace: bool, digits=None, batch: int = 1,
              direction: int = EFFT_FORWARD, scale: float = 1.0, device=None) -> api.Plan:
    """A plan with the given decomposition (None: the planner's own)."""
    p = api.Plan.__new__(api.Plan)
    p.lib = _lib.load()
    p.n, p.batch, p.dtype = int(n), int(batch), dtype
    p.direction, p.inplace, p.scale = int(direction), bool(inplace), float(scale)
    p.device = torch.device("cuda", torch.cuda.current_device() if device is None
                            else torch.device(device).index or 0)
    with torch.cuda.device(p.device):
        if digits is None:
            h = p.lib.efft_plan_many(p.n, p.batch, _DT_CODE[dtype], p.direction, int(p.inplace), p.scale)
        else:
            arr = (ctypes.c_int * len(digits))(*digits)
            h = p.lib.efft_plan_digits(p.n, p.batch, _DT_CODE[dtype], p.direction, int(p.inplace),
                                       p.scale, arr, len(digits))
    if not h:
        raise EfftError(p.lib.efft_last_error(), "efft_plan_digits")
    p.handle = ctypes.c_void_p(h)
    p.passes = p.lib.efft_plan_passes(p.handle)
    p.scratch_passes = p.lib.efft_plan_passes_scratch(p.handle)
    p.scratch_bytes = int(p.lib.efft_scratch_bytes(p.handle))
    return p


def _time_passes(plan: api.Plan, x, scratch_buf, reps: int) -> list[float]:
    """Mean event time of each pass over `reps` transforms (after one warm-up)."""
    npass = plan.scratch_passes if scratch_buf is not None else plan.passes
    plan.execute(x, scratch=scratch_buf) if plan.inplace else plan.execute(x, out=_out(plan, x))
    torch.cuda.synchronize()
    rows = [[torch.cuda.Event(enable_timing=True) for _ in range(npass + 1)] for _ in range(reps)]
    for r in rows:
        for e in r:
            e.record()
    torch.cuda.synchronize()
    out = x if plan.inplace else _out(plan, x)
    for r in rows:
        plan.execute_events(x, out, [e.cuda_event for e in r], scratch=scratch_buf)
    torch.cuda.synchronize()
    return [sum(r[i].elapsed_time(r[i + 1]) for r in rows) / reps for i in range(npass)]


_OUT: dict = {}


def _out(plan, x):
    k = (x.shape, x.dtype, x.device)
    if k not in _OUT:
        _OUT.clear()
        _OUT[k] = torch.empty_like(x)
    return _OUT[k]


def tune_passes(plan: api.Plan, x, scratch_buf=None, reps: int = 3, log=None) -> tuple[list[list[int]], float]:
    """Choose every pass's launch options by its own time, one pass at a time
    (``log`` receives a line per pass)."""
    scratch = scratch_buf is not None
    npass = plan.scratch_passes if scratch else plan.passes
    chosen = []
    for i in range(npass):
        cur = _options(plan, scratch, i)
        best, best_t = cur, None
        if cur[0] == -1:
            cands = [[-1, 0, 0, 0, a, a] for a in (0, 1)]
        else:
            cands = [[cur[0], w, s, o, a, b] for w in LINE_CHOICES for s in (1, 2) for o in (0, 1, 2)
                     for a, b in HINT_CHOICES]
        for c in cands:
            if not _set_options(plan, scratch, i, c):
                continue
            t = _time_passes(plan, x, scratch_buf, reps)[i]
            if best_t is None or t < best_t:
                best, best_t = c, t
        _set_options(plan, scratch, i, best)
        chosen.append(best)
        if log:
            log(f"  pass {i}: options {cur} -> {best} ({best_t:.3f} ms)")
    total = sum(_time_passes(plan, x, scratch_buf, reps))
    return chosen, total


def tune(n: int, dtype: torch.dtype, inplace: bool, batch: int = 1, scratch: bool = False,
         reps: int = 3, max_digits: int = 4, search_digits: bool = True, log=None,
         max_candidates: int = 6) -> dict:
    """Measure and return a wisdom entry {"digits", "passes", "ms", "default_ms"}."""
    dev = torch.device("cuda", 0)
    x = torch.empty(batch * n, dtype=dtype, device=dev)
    inputs.fill_uniform_torch(x, seed=0)
    x = x.view(batch, n) if batch > 1 else x
    q = n.bit_length() - 1
    # timed plans scale by 2^-floor(q/2) so that repeated in-place transforms
    # of the same buffer keep its magnitude (the options do not depend on it)
    sc = 2.0 ** -(q // 2)
    base = make_plan(n, dtype, inplace, None, batch, scale=sc)
    sb = base.make_scratch() if scratch else None
    default_ms = sum(_time_passes(base, x, sb, reps))
    default_digits = _lib.schedule(n, _DT_CODE[dtype], inplace)[0]
    base.close()
    cands = decompositions(q, inplace, max_digits) if search_digits else [default_digits]
    if default_digits in cands:  # the planner's choice first
        cands.remove(default_digits)
    cands = [default_digits] + cands[:max(0, max_candidates - 1)]
    best = None
    for d in cands:
        try:
            p = make_plan(n, dtype, inplace, d, batch, scale=sc)
        except EfftError:
            continue
        sb = p.make_scratch() if scratch else None
        if scratch and sb is None:
            p.close()
            continue
        opts, ms = tune_passes(p, x, sb, reps, log)
        if log:
            log(f"digits {d}: {ms:.3f} ms")
        if best is None or ms < best["ms"]:
            best = {"digits": d, "passes": opts, "ms": round(ms, 4)}
        p.close()
        del sb
        torch.cuda.empty_cache()
    best["default_ms"] = round(default_ms, 4)
    return best


def load(path: str) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def save(path: str, wisdom: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(wisdom, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def plan(n: int, dtype: torch.dtype, inplace: bool, entry: dict, batch: int = 1, scratch: bool = False,
         direction: int = EFFT_FORWARD, scale: float = 1.0) -> api.Plan:
    """A plan with the decomposition and launch options of a wisdom entry."""
    p = make_plan(n, dtype, inplace, entry["digits"], batch, direction, scale)
    for i, opts in enumerate(entry["passes"]):
        if not _set_options(p, scratch, i, opts):
            p.close()
            raise ValueError(f"wisdom options {opts} not valid for pass {i}")
    return p


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--log2n", type=int, required=True)
    ap.add_argument("--dtype", choices=sorted(_DT), default="c128")
    ap.add_argument("--inplace", action="store_true")
    ap.add_argument("--scratch", action="store_true")
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--max-digits", type=int, default=4)
    ap.add_argument("--max-candidates", type=int, default=6)
    ap.add_argument("--out", default="wisdom.json")
    a = ap.parse_args(argv)
    n, dt = 1 << a.log2n, _DT[a.dtype]
    entry = tune(n, dt, a.inplace or a.scratch, a.batch, a.scratch, a.reps, a.max_digits,
                 log=lambda s: print(s, flush=True), max_candidates=a.max_candidates)
    w = load(a.out)
    w[key(n, dt, a.inplace or a.scratch, a.batch, a.scratch)] = entry
    save(a.out, w)
    print(json.dumps(entry), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
