"""The entry point that allocates nothing, efft_exec_noalloc, called through
the C ABI and compared with efft_exec_scratch (the same transform with a
caller-owned scratch array) on the same plans and inputs: bit-identical
outputs on two calls in a row, the second with a smaller input, both also
within the parity bar of the FP64 oracle.  Requests beyond the fixed array
and plans of the wrong kind are refused before anything is enqueued."""
import ctypes

import pytest
import torch

import oracle
from paper_1409_5757_amd import _lib, api, inputs
from tests.gpu_util import TOL, rel_l2

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
LIMIT = 64 << 20  # EFFT_NOALLOC_SCRATCH_BYTES in include/efft.h
EFFT_ERR_SIZE, EFFT_ERR_PLAN_KIND = -1, -6


def _noalloc(plan: api.Plan, x: torch.Tensor) -> int:
    s = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    return _lib.load().efft_exec_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), s)


def _signals(batch: int, n: int, dtype, seed: int) -> torch.Tensor:
    x = torch.empty(batch, n, dtype=dtype, device=DEV)
    for b in range(batch):
        inputs.fill_uniform_torch(x[b], seed=seed + b)
    return x


# (log2 N, dtype, direction, batch): the first fills the fixed array exactly,
# the second is smaller (and runs after it, on the array's old contents)
CASES = [(22, torch.complex128, -1, 1), (16, torch.complex64, 1, 3)]


def test_noalloc_matches_scratch_schedule_two_calls():
    for i, (q, dtype, direction, batch) in enumerate(CASES):
        n = 1 << q
        plan = api.Plan(n, dtype, direction, True, device=DEV, batch=batch)
        assert 0 < plan.scratch_bytes <= LIMIT
        x = _signals(batch, n, dtype, seed=500 + 10 * i)
        xh = x.cpu().numpy()
        a, b = x.clone(), x.clone()
        plan.execute(a, scratch=plan.make_scratch())
        assert _noalloc(plan, b) == 0
        torch.cuda.synchronize()
        assert torch.equal(a, b), f"call {i}: efft_exec_noalloc differs from efft_exec_scratch"
        got = b.cpu().numpy()
        for r in range(batch):
            err = rel_l2(got[r], oracle.fft(xh[r], direction))
            print(f"noalloc call {i}: 2^{q} {dtype} dir={direction:+d} signal {r}: rel_l2={err:.3e}", flush=True)
            assert err <= TOL[dtype]
        plan.close()


def test_noalloc_refuses_what_does_not_fit():
    big = api.Plan(1 << 22, torch.complex128, -1, True, device=DEV, batch=2)  # 128 MiB of scratch
    x = torch.zeros(2, 1 << 22, dtype=torch.complex128, device=DEV)
    assert big.scratch_bytes > LIMIT
    assert _noalloc(big, x) == EFFT_ERR_SIZE
    oop = api.Plan(1 << 10, torch.complex64, -1, False, device=DEV)
    y = torch.zeros(1 << 10, dtype=torch.complex64, device=DEV)
    assert _noalloc(oop, y) == EFFT_ERR_PLAN_KIND
    torch.cuda.synchronize()
    assert torch.count_nonzero(x).item() == 0  # nothing was enqueued
    big.close()
    oop.close()
