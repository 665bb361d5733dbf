"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (in-place N = 2^30 complex128 is the headline), on outputs the
CPU oracle can compute one by one (direct Eq. "eqf" at sampled bins, the input
streamed from the device), on closed forms that hold at any size (sparse tone
spectrum, Parseval), and on round trips over the whole array.

Input recipes: re, im i.i.d. U[-1, 1) (counter-based generator; the device
fill is bit-identical to the host one), i.i.d. N(0, 1), or a sum of 8
integer-frequency unit tones with random phases."""
import numpy as np
import pytest
import torch

from paper_1409_5757_amd import api, inputs
from tests.gpu_util import (NP, TOL, device_rel_l2, max_abs, oracle_bins_from_device, rel_l2,
                            sample_bins, tone_spectrum_errors)

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DEV = torch.device("cuda", 0)


def _parseval(spec: torch.Tensor, x_sumsq: float, n: int) -> float:
    s = 0.0
    for i in range(0, spec.shape[0], 1 << 26):
        c = spec[i:i + (1 << 26)].to(torch.complex128)
        s += float(torch.sum(c.real ** 2 + c.imag ** 2))
    return s / (n * x_sumsq) - 1.0


def _sumsq(x: torch.Tensor) -> float:
    s = 0.0
    for i in range(0, x.shape[0], 1 << 26):
        c = x[i:i + (1 << 26)].to(torch.complex128)
        s += float(torch.sum(c.real ** 2 + c.imag ** 2))
    return s


def test_device_generator_matches_host_bitwise():
    x = torch.empty(1 << 20, dtype=torch.complex128, device=DEV)
    inputs.fill_uniform_torch(x, seed=0, offset=(1 << 30) - (1 << 20))
    np.testing.assert_array_equal(x.cpu().numpy(),
                                  inputs.generate("uniform", 0, 1 << 20, offset=(1 << 30) - (1 << 20)))


def test_c1_2p20_complex128_out_of_place_full_spectrum():
    """N = 2^20 complex128 out of place: every bin against the FP64 radix-2
    oracle for seeds 0-4, input preserved, and the inverse round trip."""
    import oracle
    n = 1 << 20
    for seed in range(5):
        xh = inputs.generate("uniform", seed, n)
        x = torch.from_numpy(xh).to(DEV)
        y = api.fft(x)
        ref = oracle.fft(xh)
        yh = y.cpu().numpy()
        err = rel_l2(yh, ref)
        print(f"C1 seed={seed}: rel_l2={err:.3e} max_abs={max_abs(yh, ref):.3e}", flush=True)
        assert err <= TOL[torch.complex128]
        np.testing.assert_array_equal(x.cpu().numpy(), xh)
        assert rel_l2(api.ifft(y).cpu().numpy(), xh) < 1e-15 * 20


def test_c2_2p30_complex128_in_place_sampled_and_round_trip():
    """N = 2^30 complex128 in place (the benchmark's plan): sampled bins against
    the oracle, Parseval, then the inverse in place back to the input."""
    n = 1 << 30
    x = torch.empty(n, dtype=torch.complex128, device=DEV)
    inputs.fill_uniform_torch(x, seed=0)
    bins = sample_bins(n, 12, seed=30)
    ref = oracle_bins_from_device(x, bins)  # dense every-bin check: test_gpu_dense.py
    sumsq = _sumsq(x)
    plan = api.get_plan(n, torch.complex128, -1, True, 1.0, DEV)
    plan.execute(x)
    torch.cuda.synchronize()
    got = x[torch.from_numpy(bins).to(DEV)].cpu().numpy()
    err = rel_l2(got, ref)
    pe = _parseval(x, sumsq, n)
    print(f"C2 sampled {len(bins)} bins: rel_l2={err:.3e} max_abs={max_abs(got, ref):.3e} "
          f"parseval={pe:.2e}", flush=True)
    assert err <= TOL[torch.complex128]
    assert abs(pe) < 1e-12
    api.ifft(x, inplace=True)
    x0 = torch.empty_like(x)
    inputs.fill_uniform_torch(x0, seed=0)
    rt = device_rel_l2(x, x0)
    print(f"C2 round trip rel_l2={rt:.3e}", flush=True)
    assert rt < 1e-14


def test_c2_2p30_complex128_scratch_schedule_bitwise():
    """The scratch schedule of the benchmark plan gives the same bits as the
    scratch-free schedule, whose parity the previous test establishes."""
    n = 1 << 30
    torch.cuda.empty_cache()
    a = torch.empty(n, dtype=torch.complex128, device=DEV)
    inputs.fill_uniform_torch(a, seed=0)
    b = a.clone()
    plan = api.get_plan(n, torch.complex128, -1, True, 1.0, DEV)
    plan.execute(a)
    scratch = plan.make_scratch()
    plan.execute(b, scratch=scratch)
    torch.cuda.synchronize()
    assert plan.scratch_passes == 3 and plan.passes == 4
    same = all(torch.equal(a[i:i + (1 << 26)], b[i:i + (1 << 26)]) for i in range(0, n, 1 << 26))
    assert same


def test_c2_2p30_complex128_tones_full_spectrum():
    """The 8-tone variant: exact peaks N e^{i phi} and zero elsewhere, checked
    on all 2^30 bins on the device."""
    n = 1 << 30
    x = torch.empty(n, dtype=torch.complex128, device=DEV)
    inputs.fill_tones_torch(x, seed=1)
    api.get_plan(n, torch.complex128, -1, True, 1.0, DEV).execute(x)
    torch.cuda.synchronize()
    rel, mabs, perr = tone_spectrum_errors(x, 1, n)
    print(f"C2 tones, every bin: rel_l2={rel:.3e} max_abs/N={mabs:.3e} peak err/N={perr:.3e}", flush=True)
    assert rel <= TOL[torch.complex128]
    assert mabs < 1e-12


@pytest.mark.timeout(600)
def test_c3_2p32_complex64_out_of_place_vs_fp64_oracle():
    """N = 2^32 complex64, normal inputs, out of place: error against the FP64
    oracle at 64 sampled bins (relative L2 and max abs), Parseval, input kept."""
    n = 1 << 32
    torch.cuda.empty_cache()
    x = torch.empty(n, dtype=torch.complex64, device=DEV)
    inputs.fill_normal_torch(x, seed=3)
    bins = sample_bins(n, 60, seed=32)
    ref = oracle_bins_from_device(x, bins)
    sumsq = _sumsq(x)
    probe = x[:4096].clone()
    y = torch.empty_like(x)
    api.get_plan(n, torch.complex64, -1, False, 1.0, DEV).execute(x, out=y)
    torch.cuda.synchronize()
    got = y[torch.from_numpy(bins).to(DEV)].cpu().numpy()
    err = rel_l2(got, ref)
    pe = _parseval(y, sumsq, n)
    print(f"C3 sampled {len(bins)} bins: rel_l2={err:.3e} max_abs={max_abs(got, ref):.3e} "
          f"max|F|={np.abs(ref).max():.3e} parseval={pe:.2e}", flush=True)
    assert err <= TOL[torch.complex64]
    assert abs(pe) < 1e-5
    assert torch.equal(x[:4096], probe)


@pytest.mark.timeout(600)
def test_c4_2p34_complex64_in_place_forward_and_inverse():
    """N = 2^34 complex64 (128 GiB) in place, forward then inverse: 16 sampled
    bins against the FP64 oracle and the round trip over the whole array."""
    n = 1 << 34
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info(DEV)
    if free < n * 8 + (8 << 30):
        pytest.skip(f"needs {n * 8 / 2**30 + 8:.0f} GiB free on the device, have {free / 2**30:.0f}")
    x = torch.empty(n, dtype=torch.complex64, device=DEV)
    inputs.fill_uniform_torch(x, seed=4)
    bins = sample_bins(n, 12, seed=34)
    ref = oracle_bins_from_device(x, bins, chunk=1 << 26)
    api.get_plan(n, torch.complex64, -1, True, 1.0, DEV).execute(x)
    torch.cuda.synchronize()
    got = x[torch.from_numpy(bins).to(DEV)].cpu().numpy()
    err = rel_l2(got, ref)
    print(f"C4 forward sampled {len(bins)} bins: rel_l2={err:.3e} max_abs={max_abs(got, ref):.3e}",
          flush=True)
    assert err <= TOL[torch.complex64]
    api.ifft(x, inplace=True)
    torch.cuda.synchronize()
    # compare with the regenerated input chunk by chunk
    chunk = 1 << 28
    buf = torch.empty(chunk, dtype=torch.complex64, device=DEV)
    num = den = 0.0
    for s in range(0, n, chunk):
        inputs.fill_uniform_torch(buf, seed=4, offset=s)
        d = (x[s:s + chunk] - buf).abs() ** 2
        num += float(d.double().sum())
        den += float((buf.abs() ** 2).double().sum())
    rt = (num / den) ** 0.5
    print(f"C4 round trip rel_l2={rt:.3e}", flush=True)
    assert rt < 1e-5
