"""Batched plans (efft_plan_many): every signal of a batch must come out
bit-identical to the same signal transformed by a one-signal plan (the
kernels do the same arithmetic per line; only the grid grows), and equal to
the FP64 oracle within the path's tolerance.  Sizes cover every pass layout:
one row pass (N <= 2^12), out-of-place column-to-row + column passes, the
in-place column / row / digit-reversal passes, and the scratch schedule's
row-to-column pass; batches of 3 and 5 exercise tile counts that are not
powers of two."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1409_5757_amd import _lib, api
from tests.gpu_util import TOL, host_input, rel_l2

pytestmark = pytest.mark.gpu

CASES = [  # (q, batch)
    (0, 3), (5, 4), (12, 3), (13, 5), (16, 3), (20, 2), (22, 3),
]


def _one_by_one(xh, q, dtype, direction, inplace, scratch):
    n = 1 << q
    p = api.Plan(n, dtype, direction, inplace, device=torch.device("cuda", 0))
    rows = []
    for r in range(xh.shape[0]):
        x = torch.from_numpy(xh[r].copy()).cuda()
        sc = p.make_scratch() if scratch else None
        y = p.execute(x, scratch=sc) if inplace else p.execute(x)
        rows.append(y)
    torch.cuda.synchronize()
    return torch.stack(rows)


@pytest.mark.parametrize("q,batch", CASES)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("mode", ["inplace", "oop", "scratch"])
def test_batch_matches_single_signal_bitwise(q, batch, dtype, mode):
    n = 1 << q
    inplace = mode != "oop"
    xh = np.stack([host_input("uniform", 900 + 10 * q + r, n, dtype) for r in range(batch)])
    direction = -1 if (q + batch) % 2 else 1
    p = api.Plan(n, dtype, direction, inplace, device=torch.device("cuda", 0), batch=batch)
    assert p.lib.efft_plan_batch(p.handle) == batch
    x = torch.from_numpy(xh).cuda()
    if mode == "scratch":
        sc = p.make_scratch()
        if q > 12:
            assert sc is not None and sc.numel() == batch * n
        got = p.execute(x, scratch=sc)
    elif inplace:
        got = p.execute(x)
    else:
        got = p.execute(x)
        assert torch.equal(x.cpu(), torch.from_numpy(xh))  # input preserved
    ref = _one_by_one(xh, q, dtype, direction, inplace, mode == "scratch")
    torch.cuda.synchronize()
    print(f"q={q} batch={batch} {dtype} {mode}", flush=True)
    assert torch.equal(got, ref)
    gh = got.cpu().numpy()
    for r in range(batch):
        assert rel_l2(gh[r], oracle.fft(xh[r], direction)) <= TOL[dtype]


def test_batched_api_path_and_large_batch():
    """api.fft over a (B, N) tensor runs one batched plan; B = 64 rows of 2^14."""
    x = torch.from_numpy(np.stack([host_input("normal", 77 + r, 1 << 14, torch.complex64)
                                   for r in range(64)])).cuda()
    y = api.fft(x)
    xh, yh = x.cpu().numpy(), y.cpu().numpy()
    for r in (0, 17, 63):
        assert rel_l2(yh[r], oracle.fft(xh[r])) <= TOL[torch.complex64]
    z = api.ifft(y)
    assert rel_l2(z.cpu().numpy(), xh) < 2e-6


def test_batched_error_paths():
    lib = _lib.load()
    dev = torch.device("cuda", 0)
    p = api.Plan(1 << 14, torch.complex128, -1, True, device=dev, batch=3)
    assert p.scratch_bytes == 3 * (1 << 14) * 16
    buf = torch.zeros(7 * (1 << 14), dtype=torch.complex128, device=dev)
    base = buf.data_ptr()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # scratch overlapping the batch's data (which spans 3 signals)
    assert lib.efft_exec_scratch(p.handle, ctypes.c_void_p(base), ctypes.c_void_p(base + 2 * (1 << 14) * 16), s) == -7
    oop = api.Plan(1 << 14, torch.complex128, -1, False, device=dev, batch=3)
    assert lib.efft_exec_oop(oop.handle, ctypes.c_void_p(base), ctypes.c_void_p(base + (1 << 14) * 16), s) == -7
    with pytest.raises(ValueError):
        p.execute(torch.zeros(2, 1 << 14, dtype=torch.complex128, device=dev))  # 2 rows, batch 3
    torch.cuda.synchronize()


def test_stream_copy():
    """The bandwidth reference copies exactly, on the caller's stream, for
    sizes that are and are not multiples of its 16 KiB block."""
    lib = _lib.load()
    dev = torch.device("cuda", 0)
    s = torch.cuda.Stream(dev)
    for nbytes in (16, 4096, 16384 + 48, (1 << 24) + 16 * 7):
        a = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device=dev)
        b = torch.zeros(nbytes + 64, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            rc = lib.efft_stream_copy(ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(a.data_ptr()), nbytes,
                                      ctypes.c_void_p(s.cuda_stream))
        assert rc == 0
        s.synchronize()
        assert torch.equal(b[:nbytes], a)
        assert int(b[nbytes:].sum()) == 0  # nothing written past the end
