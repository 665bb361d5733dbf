"""GPU parity of the HIP path against the FP64 oracle, element by element, on
seeded inputs: every size 2^0 .. 2^16 in both precisions, both directions,
in place and out of place, then larger sizes that span many tiles and all
decomposition shapes (one pass, two passes + square swap, three passes with
a middle digit, four passes)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1409_5757_amd import _lib, api, inputs
from tests.gpu_util import NP, TOL, host_input, max_abs, rel_l2, run_library

pytestmark = pytest.mark.gpu

DTYPES = [torch.complex128, torch.complex64]


def _check(q, dtype, direction, inplace, family="uniform", seed=None):
    n = 1 << q
    seed = q * 10 + (1 if dtype == torch.complex64 else 0) if seed is None else seed
    x = host_input(family, seed, n, dtype)
    got, x_after = run_library(x, dtype, direction, inplace)
    ref = oracle.fft(x, direction)
    err = rel_l2(got, ref)
    print(f"q={q} {dtype} dir={direction} inplace={inplace}: rel_l2={err:.3e} "
          f"max_abs={max_abs(got, ref):.3e}", flush=True)
    assert err <= TOL[dtype], err
    if x_after is not None:  # out of place: input preserved
        np.testing.assert_array_equal(x_after, x)
    return got


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("inplace", [True, False])
@pytest.mark.parametrize("direction", [-1, 1])
def test_every_small_size(dtype, inplace, direction):
    for q in range(0, 17):
        _check(q, dtype, direction, inplace)


@pytest.mark.parametrize("q", [17, 18, 19, 20, 21, 22])
@pytest.mark.parametrize("dtype", DTYPES)
def test_medium_sizes(q, dtype):
    _check(q, dtype, -1, True)
    _check(q, dtype, -1, False)


@pytest.mark.parametrize("q", [23, 24])
def test_three_pass_sizes(q):
    _check(q, torch.complex128, -1, True)
    _check(q, torch.complex64, 1, False)


def test_one_pass_inplace_equals_out_of_place_bitwise():
    """For N <= 2^12 both plans run the same single pass: identical bits."""
    for dtype in DTYPES:
        for q in (0, 3, 7, 12):
            x = host_input("normal", 99 + q, 1 << q, dtype)
            a, _ = run_library(x, dtype, -1, True)
            b, _ = run_library(x, dtype, -1, False)
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("dtype", DTYPES)
def test_closed_form_tones_full_spectrum(dtype):
    """Sum of 8 integer-frequency unit tones: N e^{i phi} at each frequency and
    zero elsewhere, checked on every bin (inputs synthesised in FP64)."""
    for q, inplace in ((20, True), (22, False), (24, True)):
        n = 1 << q
        x = inputs.tones(5, n, dtype=NP[dtype])
        got, _ = run_library(x, dtype, -1, inplace)
        f, v = inputs.tone_spectrum_peaks(5, n)
        tol = 1e-8 * n if dtype == torch.complex128 else 3e-4 * n
        assert np.max(np.abs(got[f] - v)) < tol
        rest = got.copy()
        rest[f] = 0
        assert np.max(np.abs(rest)) < tol


@pytest.mark.parametrize("dtype", DTYPES)
def test_impulse_and_constant(dtype):
    for q in (5, 13, 20):
        n = 1 << q
        k = np.arange(n)
        for n0 in (0, 1, n - 1, n // 3):
            x = np.zeros(n, dtype=NP[dtype])
            x[n0] = 1
            got, _ = run_library(x, dtype, -1, q % 2 == 0)
            ref = np.exp(-2j * np.pi * ((k * n0) % n) / n)
            assert max_abs(got, ref) < (1e-13 if dtype == torch.complex128 else 2e-6)
        x = np.full(n, 1.0 + 0.0j, dtype=NP[dtype])
        got, _ = run_library(x, dtype, 1, False)
        ref = np.zeros(n)
        ref[0] = n
        assert max_abs(got, ref) < (1e-10 * n if dtype == torch.complex128 else 1e-5 * n)


@pytest.mark.parametrize("dtype", DTYPES)
def test_round_trip_ifft(dtype):
    for q in (1, 10, 16, 21):
        n = 1 << q
        x = torch.from_numpy(host_input("uniform", q, n, dtype)).cuda()
        y = api.ifft(api.fft(x))
        err = rel_l2(y.cpu().numpy(), x.cpu().numpy())
        assert err < (1e-14 if dtype == torch.complex128 else 2e-6), err
        z = x.clone()
        api.fft(z, inplace=True)
        api.ifft(z, inplace=True)
        assert rel_l2(z.cpu().numpy(), x.cpu().numpy()) < (1e-14 if dtype == torch.complex128 else 2e-6)


def test_batched_rows():
    x = torch.from_numpy(inputs.generate("normal", 3, 8 * 4096).reshape(8, 4096)).cuda()
    y = api.fft(x).cpu().numpy()
    xh = x.cpu().numpy()
    for r in range(8):
        assert rel_l2(y[r], oracle.fft(xh[r])) < 1e-12


def test_hermitian_symmetry_for_real_input():
    n = 1 << 18
    x = inputs.generate("uniform", 8, n)
    x.imag = 0
    got, _ = run_library(x, torch.complex128, -1, True)
    k = np.arange(n)
    assert np.max(np.abs(got[(-k) % n] - np.conj(got))) < 1e-9
    assert abs(got[0].imag) < 1e-9 and abs(got[n // 2].imag) < 1e-9


def test_error_paths_on_device():
    lib = _lib.load()
    dev = torch.device("cuda", 0)
    ip = api.Plan(1024, torch.complex128, -1, True, device=dev)
    oop = api.Plan(1024, torch.complex128, -1, False, device=dev)
    buf = torch.zeros(2050, dtype=torch.complex128, device=dev)
    base = buf.data_ptr()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.efft_exec(ip.handle, ctypes.c_void_p(base + 8), s) == -5          # misaligned
    assert lib.efft_exec(oop.handle, ctypes.c_void_p(base), s) == -6             # wrong kind
    assert lib.efft_exec_oop(ip.handle, ctypes.c_void_p(base), ctypes.c_void_p(base + 16384 + 16), s) == -6
    assert lib.efft_exec_oop(oop.handle, ctypes.c_void_p(base), ctypes.c_void_p(base + 16 * 512), s) == -7
    assert lib.efft_exec_oop(oop.handle, ctypes.c_void_p(base), ctypes.c_void_p(base), s) == -7
    assert lib.efft_exec_oop(oop.handle, None, ctypes.c_void_p(base), s) == -4
    assert lib.efft_plan_passes(ip.handle) == 1 and ip.device_bytes() > 0
    h = ip.handle
    assert lib.efft_destroy(h) == 0
    assert lib.efft_destroy(h) == -10       # double destroy is reported, not a crash
    assert lib.efft_exec(h, ctypes.c_void_p(base), s) == -10
    ip.handle = None
    torch.cuda.synchronize()


def test_plan_events_cover_every_pass():
    dev = torch.device("cuda", 0)
    p = api.Plan(1 << 20, torch.complex128, -1, True, device=dev)
    x = torch.from_numpy(inputs.generate("uniform", 1, 1 << 20)).to(dev)
    ref = oracle.fft(x.cpu().numpy())
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(p.passes + 1)]
    for e in evs:
        e.record()  # materialise the underlying hipEvent
    torch.cuda.synchronize()
    p.execute_events(x, x, [e.cuda_event for e in evs])
    torch.cuda.synchronize()
    times = [evs[i].elapsed_time(evs[i + 1]) for i in range(p.passes)]
    assert all(t > 0 for t in times)
    assert rel_l2(x.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("dtype", DTYPES)
def test_scratch_schedule_matches_in_place_bitwise(dtype):
    """With a scratch array the in-place plan drops its digit-reversal pass; the
    sub-FFT arithmetic is the same, so the result must be bit-identical to the
    scratch-free schedule (and both match the oracle)."""
    for q in (1, 12, 13, 14, 15, 17, 20, 22, 24):
        n = 1 << q
        for direction in (-1, 1):
            xh = host_input("uniform", 500 + q, n, dtype)
            plan = api.get_plan(n, dtype, direction, True, 1.0, torch.device("cuda", 0))
            a = torch.from_numpy(xh).cuda()
            b = a.clone()
            plan.execute(a)
            scratch = plan.make_scratch()
            if q >= 13:
                assert scratch is not None and plan.scratch_passes == plan.passes - 1
            plan.execute(b, scratch=scratch)
            torch.cuda.synchronize()
            assert torch.equal(a, b), (q, direction)
            err = rel_l2(b.cpu().numpy(), oracle.fft(xh, direction))
            assert err <= TOL[dtype], (q, err)


def test_scratch_error_paths():
    lib = _lib.load()
    dev = torch.device("cuda", 0)
    n = 1 << 14
    ip = api.Plan(n, torch.complex128, -1, True, device=dev)
    oop = api.Plan(n, torch.complex128, -1, False, device=dev)
    assert ip.scratch_bytes == n * 16 and oop.scratch_bytes == 0
    buf = torch.zeros(3 * n, dtype=torch.complex128, device=dev)
    base = buf.data_ptr()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    data, scr = ctypes.c_void_p(base), ctypes.c_void_p(base + n * 16)
    assert lib.efft_exec_scratch(oop.handle, data, scr, s) == -6                        # wrong kind
    assert lib.efft_exec_scratch(ip.handle, data, ctypes.c_void_p(base + 8 * n), s) == -7  # overlap
    assert lib.efft_exec_scratch(ip.handle, data, ctypes.c_void_p(base + n * 16 + 8), s) == -5  # align
    assert lib.efft_exec_scratch(ip.handle, data, None, s) == -4
    torch.cuda.synchronize()
