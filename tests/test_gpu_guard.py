"""Guard bands and device-memory ownership.

Every transform writes inside its output and nowhere else.  Each array sits
inside one allocation with 4 KiB of a canary value on each side; after the
transform the canaries must be untouched and the input of an out-of-place
plan unchanged.  Covered: the pass layouts (one contiguous-line pass, strided
lines, the strided-to-row first pass of out-of-place plans, the row-to-column
last pass of the scratch schedule, the digit-reversal swap), the real-input
pairing passes, the radix-M path and the chirp path, with batches of 3 (tile
counts that are not powers of two).  The results are checked against the
oracle too.

Plans own device memory only while they live: creating and destroying plans
(including plans that own large work arrays, and a plan whose creation fails
part-way through its allocations) leaves the device's free memory where it
was."""
import numpy as np
import pytest
import torch

import oracle
from paper_1409_5757_amd import api
from paper_1409_5757_amd._lib import EfftError
from tests.gpu_util import NP, TOL, host_input, rel_l2

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
GUARD = 4096  # bytes on each side
CANARY = complex(1234.5, -6789.25)


class Guarded:
    """`rows` x `n` elements of `dtype` inside one allocation, canaries around."""

    def __init__(self, rows: int, n: int, dtype):
        esz = torch.empty(0, dtype=dtype).element_size()
        self.g = GUARD // esz
        self.total = rows * n
        self.buf = torch.empty(self.g + self.total + self.g, dtype=dtype, device=DEV)
        self.buf[:self.g] = CANARY if dtype.is_complex else 1234.5
        self.buf[self.g + self.total:] = CANARY if dtype.is_complex else 1234.5
        self.view = self.buf[self.g:self.g + self.total].view(rows, n) if rows > 1 else self.buf[self.g:self.g + n]

    def intact(self) -> bool:
        torch.cuda.synchronize()
        c = CANARY if self.buf.dtype.is_complex else 1234.5
        head, tail = self.buf[:self.g], self.buf[self.g + self.total:]
        return bool((head == c).all()) and bool((tail == c).all())


def _oracle_rows(xh, direction):
    return np.stack([oracle.fft(r, direction) for r in xh])


C2C_CASES = [  # (log2 N, mode): one row pass; in place (columns, rows, swap); out of place; scratch
    (12, "inplace"), (16, "inplace"), (16, "oop"), (16, "scratch"), (20, "oop"), (20, "scratch"),
]


@pytest.mark.parametrize("q,mode", C2C_CASES)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_power_of_two_writes_only_its_output(q, mode, dtype):
    n, batch = 1 << q, 3
    direction = -1 if q % 2 else 1
    xh = np.stack([host_input("uniform", 700 + q + r, n, dtype) for r in range(batch)])
    p = api.Plan(n, dtype, direction, mode != "oop", device=DEV, batch=batch)
    x = Guarded(batch, n, dtype)
    x.view.copy_(torch.from_numpy(xh))
    if mode == "oop":
        y = Guarded(batch, n, dtype)
        p.execute(x.view, out=y.view)
        out = y
        assert torch.equal(x.view.cpu(), torch.from_numpy(xh)), "input written"
    elif mode == "scratch":
        s = Guarded(batch, n, dtype)
        p.execute(x.view, scratch=s.view)
        assert s.intact(), "scratch canaries overwritten"
        out = x
    else:
        p.execute(x.view)
        out = x
    assert x.intact() and out.intact(), "canaries overwritten"
    got = out.view.cpu().numpy()
    ref = _oracle_rows(xh, direction)
    for r in range(batch):
        assert rel_l2(got[r], ref[r]) <= TOL[dtype]
    p.close()


@pytest.mark.parametrize("rdt", [torch.float64, torch.float32])
def test_real_pairing_writes_only_its_output(rdt):
    n = 1 << 16
    cdt = torch.complex128 if rdt == torch.float64 else torch.complex64
    rng = np.random.default_rng(5)
    xr = rng.uniform(-1, 1, n).astype(np.float64 if rdt == torch.float64 else np.float32)
    fwd = api.RealPlan(n, rdt, api.EFFT_FORWARD, 1.0, DEV)
    x = Guarded(1, n, rdt)
    x.view.copy_(torch.from_numpy(xr))
    y = Guarded(1, n // 2 + 1, cdt)
    fwd.execute(x.view, y.view)
    assert x.intact() and y.intact()
    assert torch.equal(x.view.cpu(), torch.from_numpy(xr))
    ref = oracle.fft(xr.astype(np.complex128), -1)[:n // 2 + 1]
    assert rel_l2(y.view.cpu().numpy(), ref) <= TOL[cdt]
    bwd = api.RealPlan(n, rdt, api.EFFT_BACKWARD, 1.0 / n, DEV)
    z = Guarded(1, n, rdt)
    keep = y.view.clone()
    bwd.execute(y.view, z.view)
    assert y.intact() and z.intact()
    assert torch.equal(y.view, keep)
    assert rel_l2(z.view.cpu().numpy(), xr) <= TOL[cdt]
    fwd.close()
    bwd.close()


ANY_CASES = [  # lengths that are not powers of two: radix-M rows of several passes, rows of one pass, chirp
    (3 << 14, "inplace"), (3 << 14, "oop"), (5 << 10, "inplace"), (5 << 10, "oop"), (1000, "inplace"),
    ((1 << 14) + 1, "oop"),
]


@pytest.mark.parametrize("n,mode", ANY_CASES)
def test_other_lengths_write_only_their_output(n, mode):
    dtype, batch, direction = torch.complex128, 3, -1
    xh = np.stack([host_input("uniform", 800 + r, n, dtype) for r in range(batch)])
    p = api.Plan(n, dtype, direction, mode == "inplace", device=DEV, batch=batch)
    x = Guarded(batch, n, dtype)
    x.view.copy_(torch.from_numpy(xh))
    if mode == "oop":
        y = Guarded(batch, n, dtype)
        p.execute(x.view, out=y.view)
        assert torch.equal(x.view.cpu(), torch.from_numpy(xh)), "input written"
    else:
        y = x
        p.execute(x.view)
    assert x.intact() and y.intact(), "canaries overwritten"
    got = y.view.cpu().numpy()
    bins = np.unique(np.concatenate([[0, 1, n - 1, n // 2], np.random.default_rng(n).integers(0, n, 12)]))
    for r in range(batch):
        ref = oracle.dft_at(xh[r], bins, sign=direction)
        assert rel_l2(got[r][bins], ref) <= TOL[dtype]
    p.close()


def _free() -> int:
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info(DEV)[0]


def test_plans_leave_device_memory_as_they_found_it():
    # warm up: the library's code object (and its fixed scratch array) loads
    # on first use, which holds device memory for the life of the process
    w = api.Plan(1 << 10, torch.complex64, -1, True, device=DEV)
    w.execute(torch.zeros(1 << 10, dtype=torch.complex64, device=DEV))
    w.close()
    torch.cuda.empty_cache()
    free0 = _free()
    specs = [(1 << 20, torch.complex128, True), (3 << 20, torch.complex64, False),
             ((1 << 20) + 1, torch.complex128, True), ((1 << 20) + 1, torch.complex64, False),
             (1 << 24, torch.complex64, True)]
    for cycle in range(3):
        plans = [api.Plan(n, dt, -1, ip, device=DEV) for n, dt, ip in specs]
        plans.append(api.RealPlan(1 << 20, torch.float32, -1, 1.0, DEV))
        held = sum(p.device_bytes() for p in plans)
        used = free0 - _free()
        assert used >= held * 0.9, (cycle, used, held)  # the plans' arrays are really on the device
        for p in plans:
            p.close()
        # no less free memory than before (the runtime may also return memory of its own)
        assert free0 - _free() <= (2 << 20), (cycle, free0 - _free())
    # a plan whose creation fails part-way (the chirp path's arrays for
    # N = 2^33 - 1 complex128 need far more than the device has) frees what
    # it had allocated before returning the error
    with pytest.raises(EfftError):
        api.Plan((1 << 33) - 1, torch.complex128, -1, True, device=DEV)
    assert free0 - _free() <= (2 << 20), free0 - _free()
