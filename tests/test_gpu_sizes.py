"""Every size from the every-bin parity sizes (up to 2^24) to the largest,
2^25 .. 2^34, including the full workloads' 2^30, 2^32 and 2^34, whose
decompositions use digit shapes the other tests do not all reach.  On every
bin, the closed-form
spectrum of a sum of 8 integer-frequency tones (N e^{i phi} at each
frequency, zero elsewhere): relative L2 over all bins and the largest error
relative to N, the largest |F_k|; on uniform inputs, sampled bins against the
oracle's direct sum of Eq. "eqf" (error per bin relative to the RMS of the
spectrum, which is ||x||_2 by Parseval).  Both precisions, in place and out
of place where the device holds the arrays."""
import numpy as np
import pytest
import torch

from paper_1409_5757_amd import api, inputs
from tests.gpu_util import TOL, oracle_bins_from_device, sample_bins, tone_spectrum_errors

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

DEV = torch.device("cuda", 0)
DTYPES = [torch.complex128, torch.complex64]
SIZES = [25, 26, 27, 28, 29, 30, 31, 32, 33, 34]
SAMPLED_SIZES = [25, 26, 27, 28, 29]
CHUNK = 1 << 26


def _fits(nbytes: int) -> bool:
    free, _ = torch.cuda.mem_get_info(DEV)
    return nbytes + (4 << 30) <= free


def _transform(x: torch.Tensor, inplace: bool) -> torch.Tensor:
    p = api.get_plan(x.shape[0], x.dtype, -1, inplace, 1.0, DEV)
    if inplace:
        return p.execute(x)
    return p.execute(x, out=torch.empty_like(x))


@pytest.mark.parametrize("q", SIZES)
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.timeout(300)
def test_tones_every_bin(q, dtype):
    n = 1 << q
    eb = 16 if dtype == torch.complex128 else 8
    tol = 1e-12 if dtype == torch.complex128 else 1e-5
    ran = 0
    for inplace in (True, False):
        if not _fits(n * eb * (1 if inplace else 2)):
            continue
        x = torch.empty(n, dtype=dtype, device=DEV)
        inputs.fill_tones_torch(x, seed=q)
        y = _transform(x, inplace)
        torch.cuda.synchronize()
        rel, mabs, perr = tone_spectrum_errors(y, q, n)
        print(f"2^{q} {dtype} inplace={inplace}: every bin rel_l2={rel:.2e} max abs/N={mabs:.2e} "
              f"(tone bins {perr:.2e})", flush=True)
        assert rel <= tol and mabs < tol, (rel, mabs)
        ran += 1
        del x, y
        torch.cuda.empty_cache()
    if ran == 0:
        pytest.skip(f"2^{q} {dtype} does not fit the device in place")


@pytest.mark.parametrize("q", SAMPLED_SIZES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_uniform_sampled_bins(q, dtype):
    n = 1 << q
    x = torch.empty(n, dtype=dtype, device=DEV)
    inputs.fill_uniform_torch(x, seed=q)
    bins = sample_bins(n, 12, seed=q)
    ref = oracle_bins_from_device(x, bins)
    rms = float(torch.linalg.vector_norm(x.to(torch.complex128)))
    for inplace in (False, True):
        y = _transform(x if not inplace else x.clone(), inplace)
        err = float(np.max(np.abs(y[torch.from_numpy(bins).to(DEV)].cpu().numpy() - ref))) / rms
        print(f"2^{q} {dtype} inplace={inplace}: max sampled-bin error / rms = {err:.2e}", flush=True)
        assert err <= TOL[dtype]
        del y
    torch.cuda.empty_cache()
