"""Lengths that are not powers of two (the chirp path): every bin against the
oracle's direct sum of Eq. "eqf" up to N ~ 10^4, sampled bins against it at
larger N, closed-form tones, round trips, batches, prime lengths whose
M-point plans have narrowed strided passes, and argument handling.
Tolerances are the path's bars (FP64 rel-L2 <= 1e-12, FP32 <= 1e-5); for
sampled bins the error of each bin is taken relative to the RMS of the
spectrum, which equals ||x||_2 (Parseval)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1409_5757_amd import _lib, api
from tests.gpu_util import NP, TOL, host_input, oracle_bins_from_device, rel_l2, run_library, sample_bins

pytestmark = pytest.mark.gpu

DTYPES = [torch.complex128, torch.complex64]
FULL_SIZES = [3, 5, 6, 7, 9, 12, 15, 100, 243, 1000, 1536, 4097, 9973]


@pytest.mark.parametrize("dtype", DTYPES)
def test_every_bin_against_direct_sum(dtype):
    for i, n in enumerate(FULL_SIZES):
        x = host_input("uniform", 3000 + n, n, dtype)
        direction = -1 if i % 2 == 0 else 1
        inplace = i % 3 == 0
        got, after = run_library(x, dtype, direction, inplace)
        ref = oracle.dft(x, direction)
        err = rel_l2(got, ref)
        print(f"n={n} {dtype} dir={direction} inplace={inplace}: rel_l2={err:.2e}", flush=True)
        assert err <= TOL[dtype], (n, err)
        if after is not None:
            np.testing.assert_array_equal(after, x)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [3 * (1 << 20), 5 ** 10, 10 ** 7 + 1])
def test_sampled_bins_large(dtype, n):
    x = torch.from_numpy(host_input("normal", 17, n, dtype)).cuda()
    y = api.fft(x)
    bins = sample_bins(n, 24, seed=n % 1000)
    ref = oracle_bins_from_device(x, bins)
    scale = float(torch.linalg.vector_norm(x.to(torch.complex128)))
    err = float(np.max(np.abs(y[torch.from_numpy(bins).cuda()].cpu().numpy() - ref))) / scale
    print(f"n={n} {dtype}: max bin error / rms = {err:.2e}", flush=True)
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_tone_closed_form(dtype):
    """x_j = exp(2 pi i (f j mod N)/N + i phi) -> N e^{i phi} at f, 0 elsewhere."""
    n = 1_000_003  # prime
    f, phi = 123_457, 0.7
    j = np.arange(n, dtype=np.int64)
    x = np.exp(2j * np.pi * ((f * j) % n) / n + 1j * phi).astype(NP[dtype])
    got, _ = run_library(x, dtype, -1, False)
    tol = 1e-9 * n if dtype == torch.complex128 else 2e-4 * n
    assert abs(got[f] - n * np.exp(1j * phi)) < tol
    rest = got.copy()
    rest[f] = 0
    assert np.max(np.abs(rest)) < tol


@pytest.mark.parametrize("dtype", DTYPES)
def test_round_trip_and_batch(dtype):
    for n in (1000, 3 * (1 << 16) + 1):
        x = torch.from_numpy(np.stack([host_input("uniform", 50 + r, n, dtype) for r in range(3)])).cuda()
        y = api.fft(x)               # one batched plan of 3 signals
        z = api.ifft(y)
        assert rel_l2(z.cpu().numpy(), x.cpu().numpy()) < (1e-13 if dtype == torch.complex128 else 3e-6)
        # each row of the batch equals the same signal transformed alone (bit for bit)
        for r in range(3):
            alone = api.fft(x[r].contiguous())
            assert torch.equal(alone, y[r])
        # and the in-place plan gives the same bits as the out-of-place one
        w = x.clone()
        api.fft(w, inplace=True)
        assert torch.equal(w, y)
        torch.cuda.synchronize()


# Prime lengths whose M-point plans (M = 2^15 .. 2^20, two strided passes)
# have fewer tiles than the device has CUs: the planner narrows those passes,
# and the chirp plan's fused first pass (pre-multiply as it loads) and last
# pass (post-multiply as it stores) must still run with tiles that have a
# kernel for their own layout.
CHIRP_SMALL_M = [9973, 25013, 50021, 100003, 300007]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", CHIRP_SMALL_M)
def test_chirp_fused_passes_on_small_m_point_plans(dtype, n):
    for direction, inplace in ((-1, True), (1, False)):
        x = host_input("uniform", 4000 + n, n, dtype)
        got, after = run_library(x, dtype, direction, inplace)
        bins = sample_bins(n, 24, seed=n % 977)
        ref = oracle.dft_at(x, bins, sign=direction)
        err = rel_l2(got[bins], ref)
        print(f"n={n} {dtype} dir={direction} inplace={inplace}: rel_l2 over {len(bins)} bins = {err:.2e}",
              flush=True)
        assert err <= TOL[dtype], (n, direction, inplace, err)
        if after is not None:
            np.testing.assert_array_equal(after, x)


def test_plan_reports_memory_and_passes():
    p = api.Plan(1000, torch.complex128, -1, False, device=torch.device("cuda", 0))
    # chirp (FP64) + V + work of M = 2048 points, plus the two inner plans' tables
    assert p.device_bytes() >= 1000 * 16 + 2 * 2048 * 16
    assert p.passes >= 5 and p.scratch_bytes == 0


MIXED = [(m, s) for m in (3, 5, 7, 9, 11, 13, 15) for s in (0, 1, 4, 7, 10)]


@pytest.mark.parametrize("dtype", DTYPES)
def test_small_odd_factor_every_bin(dtype):
    """N = M * 2^s with M odd and <= 15 takes the radix-M pass + power-of-two
    rows + reorder: every bin against the direct sum."""
    for i, (m, s) in enumerate(MIXED):
        n = m << s
        if n < 3:
            continue
        x = host_input("normal", 7000 + n, n, dtype)
        direction = -1 if i % 2 == 0 else 1
        inplace = i % 3 == 1
        got, after = run_library(x, dtype, direction, inplace)
        err = rel_l2(got, oracle.dft(x, direction))
        assert err <= TOL[dtype], (m, s, err)
        if after is not None:
            np.testing.assert_array_equal(after, x)
    print(f"{len(MIXED)} sizes M * 2^s within {TOL[dtype]}", flush=True)


@pytest.mark.parametrize("dtype,n", [(torch.complex128, 3 << 26), (torch.complex64, 15 << 24),
                                     (torch.complex128, 7 << 20), (torch.complex64, 13 << 21)])
def test_small_odd_factor_sampled_large(dtype, n):
    x = torch.from_numpy(host_input("uniform", 23, n, dtype)).cuda()
    y = api.fft(x)
    bins = sample_bins(n, 24, seed=n % 997)
    ref = oracle_bins_from_device(x, bins)
    scale = float(torch.linalg.vector_norm(x.to(torch.complex128)))
    err = float(np.max(np.abs(y[torch.from_numpy(bins).cuda()].cpu().numpy() - ref))) / scale
    print(f"n={n} {dtype}: max bin error / rms = {err:.2e}", flush=True)
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_small_odd_factor_batch_and_placement_bitwise(dtype):
    for n in (3 << 12, 9 << 9, 15):
        x = torch.from_numpy(np.stack([host_input("uniform", 80 + r, n, dtype) for r in range(5)])).cuda()
        y = api.fft(x)
        for r in range(5):
            assert torch.equal(api.fft(x[r].contiguous()), y[r])
        w = x.clone()
        api.fft(w, inplace=True)
        assert torch.equal(w, y)
        z = api.ifft(y)
        assert rel_l2(z.cpu().numpy(), x.cpu().numpy()) < (1e-13 if dtype == torch.complex128 else 3e-6)


FUSED = [(3, 13), (5, 13), (7, 13), (3, 14)]


@pytest.mark.parametrize("dtype", DTYPES)
def test_small_odd_factor_fused_rows_every_bin(dtype):
    """Rows of two or more digits end with a pass that writes them interleaved
    straight into the output (no reorder pass): every bin against the direct
    sum, both directions, in place and out of place."""
    for i, (m, s) in enumerate(FUSED):
        n = m << s
        digits, _ = _lib.schedule(1 << s, 2 if dtype == torch.complex128 else 1, True)
        p = api.Plan(n, dtype, -1, False, device=torch.device("cuda", 0))
        assert len(digits) >= 2 and p.passes == 1 + len(digits), (m, s, digits, p.passes)
        p.close()
        x = host_input("uniform", 9000 + n, n, dtype)
        direction = -1 if i % 2 == 0 else 1
        inplace = i % 2 == 1
        got, after = run_library(x, dtype, direction, inplace)
        err = rel_l2(got, oracle.dft(x, direction))
        print(f"n={m}*2^{s} {dtype} dir={direction} inplace={inplace}: rel_l2={err:.2e}", flush=True)
        assert err <= TOL[dtype], (m, s, err)
        if after is not None:
            np.testing.assert_array_equal(after, x)


@pytest.mark.parametrize("dtype", DTYPES)
def test_small_odd_factor_fused_rows_batch_scale_placement(dtype):
    n = 5 << 13
    x = torch.from_numpy(np.stack([host_input("normal", 300 + r, n, dtype) for r in range(3)])).cuda()
    y = api.fft(x)
    for r in range(3):
        assert torch.equal(api.fft(x[r].contiguous()), y[r])
    w = x.clone()
    api.fft(w, inplace=True)
    assert torch.equal(w, y)
    # the inverse scales by 1/N (not a power of two) in the interleaving pass
    z = api.ifft(y)
    assert rel_l2(z.cpu().numpy(), x.cpu().numpy()) < (1e-13 if dtype == torch.complex128 else 3e-6)
    ref = oracle.dft(x[1].cpu().numpy(), +1) / n
    assert rel_l2(api.ifft(x[1].contiguous()).cpu().numpy(), ref) <= TOL[dtype]
