"""Tuning: launch options never change the arithmetic (bit-identical results
for every option the tuner tries, among them the narrowed tiles of small
grids at 2^20 and the one- and two-set tiles of 256-point complex64 lines at
2^25), tuned decompositions stay within the oracle tolerance, and wisdom
entries round-trip through a file."""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from paper_1409_5757_amd import api, tune
from tests.gpu_util import TOL, host_input, rel_l2

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("q,dtype,inplace", [(20, torch.complex128, True), (22, torch.complex64, False),
                                             (14, torch.complex128, False), (25, torch.complex64, False)])
def test_every_option_gives_identical_bits(q, dtype, inplace):
    n = 1 << q
    xh = host_input("uniform", 40 + q, n, dtype)
    ref_plan = api.Plan(n, dtype, -1, inplace, device=torch.device("cuda", 0))
    ref = ref_plan.execute(torch.from_numpy(xh).cuda())
    p = tune.make_plan(n, dtype, inplace)
    tried = 0
    for i in range(p.passes):
        cur = tune._options(p, False, i)
        cands = ([[-1, 0, 0, 0, a, a] for a in (0, 1)] if cur[0] == -1 else
                 [[cur[0], w, s, o, a, b] for w in tune.LINE_CHOICES for s in (1, 2) for o in (0, 1, 2)
                  for a, b in tune.HINT_CHOICES])
        for c in cands:
            if not tune._set_options(p, False, i, c):
                continue
            tried += 1
            got = p.execute(torch.from_numpy(xh).cuda())
            assert torch.equal(got, ref), (i, c)
        tune._set_options(p, False, i, cur)
    print(f"q={q}: {tried} option settings, all bit-identical", flush=True)
    assert tried >= p.passes


def test_tune_and_wisdom_round_trip():
    n, dtype = 1 << 20, torch.complex64
    entry = tune.tune(n, dtype, True, reps=1, max_digits=3)
    assert sum(entry["digits"]) == 20 and entry["ms"] > 0 and entry["default_ms"] > 0
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "wisdom.json")
        k = tune.key(n, dtype, True)
        tune.save(path, {k: entry})
        back = tune.load(path)[k]
    assert back == entry
    p = tune.plan(n, dtype, True, back)
    xh = host_input("normal", 5, n, dtype)
    x = torch.from_numpy(xh).cuda()
    p.execute(x)
    assert rel_l2(x.cpu().numpy(), oracle.fft(xh)) <= TOL[dtype]
    for i, opts in enumerate(back["passes"]):
        assert tune._options(p, False, i) == opts


FORCED = [  # (n, dtype, in place, digits): balanced, unbalanced, and strided lines of 2^11 and 2^12 points
    (1 << 20, torch.complex128, True, [5, 10, 5]), (1 << 20, torch.complex128, False, [4, 8, 8]),
    (1 << 24, torch.complex64, True, [6, 6, 6, 6]), (1 << 24, torch.complex64, False, [10, 4, 10]),
    (1 << 24, torch.complex64, False, [12, 6, 6]), (1 << 24, torch.complex128, True, [6, 12, 6]),
    (1 << 22, torch.complex64, True, [5, 12, 5]), (1 << 23, torch.complex128, False, [11, 12]),
    (1 << 24, torch.complex64, True, [12, 12]), (1 << 22, torch.complex128, True, [11, 11]),
    (1 << 26, torch.complex64, False, [10, 12, 4]), (1 << 25, torch.complex128, False, [4, 11, 10]),
]


@pytest.mark.parametrize("n,dtype,inplace,digits", FORCED,
                         ids=[f"2^{f[0].bit_length() - 1}-{'c128' if f[1] == torch.complex128 else 'c64'}-"
                              f"{'ip' if f[2] else 'oop'}-{'.'.join(map(str, f[3]))}" for f in FORCED])
def test_forced_decompositions_match_oracle(n, dtype, inplace, digits):
    p = tune.make_plan(n, dtype, inplace, digits)
    for direction, scratch in ((-1, False), (1, inplace)):
        if direction == 1:
            p.close()
            p = tune.make_plan(n, dtype, inplace, digits, direction=1)
        xh = host_input("uniform", 9 + direction, n, dtype)
        x = torch.from_numpy(xh).cuda()
        y = p.execute(x, scratch=p.make_scratch() if scratch else None) if inplace else p.execute(x)
        err = rel_l2(y.cpu().numpy(), oracle.fft(xh, direction))
        print(f"n=2^{n.bit_length() - 1} digits={digits} dir={direction:+d} scratch={scratch}: rel_l2={err:.2e}",
              flush=True)
        assert err <= TOL[dtype]
    p.close()
