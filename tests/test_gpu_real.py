"""Real-data transforms (the paper's workload is real input, Section 2.1 and
Section 4): forward N reals -> N/2 + 1 bins, backward Hermitian bins -> N
reals, against the FP64 oracle applied to the same real input taken as
complex data, for every size 2^1 .. 2^16 and larger, both precisions."""
import numpy as np
import pytest
import torch

import oracle
from paper_1409_5757_amd import api, inputs
from tests.gpu_util import TOL, max_abs, rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
RDT = {torch.complex128: torch.float64, torch.complex64: torch.float32}
NPR = {torch.complex128: np.float64, torch.complex64: np.float32}


def _real_input(q, seed, cdt):
    n = 1 << q
    x = inputs.generate("uniform", seed, n // 2 + 1 if n > 1 else 1, dtype=np.complex128)
    r = np.empty(n, dtype=np.float64)
    r[0::2] = x.real[: (n + 1) // 2]
    r[1::2] = x.imag[: n // 2]
    return r.astype(NPR[cdt])


@pytest.mark.parametrize("cdt", [torch.complex128, torch.complex64])
def test_forward_every_size(cdt):
    for q in list(range(1, 17)) + [18, 20, 22]:
        n = 1 << q
        xr = _real_input(q, q, cdt)
        x = torch.from_numpy(xr).to(DEV)
        y = api.rfft(x)
        ref = oracle.fft(xr.astype(np.float64).astype(np.complex128))[: n // 2 + 1]
        got = y.cpu().numpy()
        err = rel_l2(got, ref)
        print(f"rfft q={q} {cdt}: rel_l2={err:.3e} max_abs={max_abs(got, ref):.3e}", flush=True)
        assert err <= TOL[cdt]
        np.testing.assert_array_equal(x.cpu().numpy(), xr)  # input preserved


@pytest.mark.parametrize("cdt", [torch.complex128, torch.complex64])
def test_backward_unnormalised_every_size(cdt):
    for q in list(range(1, 17)) + [20]:
        n = 1 << q
        xr = _real_input(q, 100 + q, cdt)
        spec = oracle.fft(xr.astype(np.float64).astype(np.complex128))[: n // 2 + 1]
        f = torch.from_numpy(spec.astype(np.complex128 if cdt == torch.complex128 else np.complex64)).to(DEV)
        plan = api.RealPlan(n, RDT[cdt], api.EFFT_BACKWARD, 1.0, DEV)
        y = plan.execute(f).cpu().numpy()
        ref = n * xr.astype(np.float64)
        err = rel_l2(y, ref)
        assert err <= TOL[cdt], (q, err)
        np.testing.assert_array_equal(f.cpu().numpy(), spec.astype(f.cpu().numpy().dtype))


@pytest.mark.parametrize("cdt", [torch.complex128, torch.complex64])
def test_round_trip_and_batch(cdt):
    for q in (1, 2, 9, 17):
        n = 1 << q
        xr = np.stack([_real_input(q, 7 + b, cdt) for b in range(3)])
        x = torch.from_numpy(xr).to(DEV)
        z = api.irfft(api.rfft(x), n)
        assert rel_l2(z.cpu().numpy(), xr) < (1e-14 if cdt == torch.complex128 else 2e-6)


def test_backward_ignores_imaginary_dc_and_nyquist():
    """Like other half-spectrum conventions, the imaginary parts of F_0 and
    F_{N/2} are ignored (they are zero for any real signal)."""
    n = 1 << 10
    rng = np.random.default_rng(3)
    f = rng.standard_normal(n // 2 + 1) + 1j * rng.standard_normal(n // 2 + 1)
    got = api.irfft(torch.from_numpy(f).to(DEV), n).cpu().numpy()
    g = f.copy()
    g[0] = g[0].real
    g[-1] = g[-1].real
    full = np.concatenate([g, np.conj(g[-2:0:-1])])
    ref = oracle.fft(full, +1).real / n
    assert rel_l2(got, ref) < 1e-13


def test_real_plan_errors():
    with pytest.raises(api.EfftError):
        api.RealPlan(1, torch.float64, api.EFFT_FORWARD, 1.0, DEV)   # N = 1 has no half spectrum
    with pytest.raises(api.EfftError):
        api.RealPlan(12, torch.float64, api.EFFT_FORWARD, 1.0, DEV)
    p = api.RealPlan(1024, torch.float64, api.EFFT_FORWARD, 1.0, DEV)
    assert p.passes == api.get_plan(512, torch.complex128, -1, False, 1.0, DEV).passes + 1


@pytest.mark.slow
def test_real_2p30_float32_sampled():
    """The paper's headline size and type: N = 2^30 real FP32, sampled bins
    against the FP64 oracle."""
    from tests.gpu_util import oracle_bins_from_device, sample_bins
    n = 1 << 30
    xc = torch.empty(n // 2, dtype=torch.complex64, device=DEV)
    inputs.fill_uniform_torch(xc, seed=11, lo=-0.5, hi=0.5)   # the paper's U[-0.5, 0.5] (Section 5.3)
    x = torch.view_as_real(xc).reshape(n)
    bins = sample_bins(n // 2 + 1, 6, seed=5)
    # the oracle sees the same real samples as complex data with zero imaginary part
    acc = None
    chunk = 1 << 24
    for s in range(0, n, chunk):
        h = x[s:s + chunk].double().cpu().numpy().astype(np.complex128)
        acc = oracle.dft_bins(h, bins, n=n, offset=s, acc=acc)
    ref = oracle.bins_value(acc)
    y = api.rfft(x)
    got = y[torch.from_numpy(bins).to(DEV)].cpu().numpy()
    err = rel_l2(got, ref)
    print(f"rfft 2^30 float32 sampled: rel_l2={err:.3e}", flush=True)
    assert err <= 1e-5
