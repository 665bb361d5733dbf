"""Differentiation through the transform: the backward pass of EfftFFT is the
conjugate-direction (unnormalised) transform, the exact adjoint of the
forward one.  Checked by torch.autograd.gradcheck on the FP64 path, by the
adjoint identity <F x, y> = <x, F^H y>, and on the differentiable batch
(64 signals of 2^24 complex64, loss sum |w * FFT(x) - y|^2) against central
finite differences and the analytic gradient 2 * F^H(w * (w * F x - y))."""
import numpy as np
import pytest
import torch

import oracle
from paper_1409_5757_amd import api, inputs
from tests.gpu_util import rel_l2

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def test_autograd_convention_factor():
    """PyTorch's complex gradient of L = |z|^2 is 2z (grad = dL/dRe + i dL/dIm)."""
    z = torch.tensor([0.3 - 1.2j], dtype=torch.complex128, requires_grad=True)
    (z.real ** 2 + z.imag ** 2).sum().backward()
    assert torch.allclose(z.grad, 2 * z.detach())


@pytest.mark.parametrize("n", [1, 2, 8, 64, 256])
def test_gradcheck_fp64(n):
    g = torch.Generator().manual_seed(n)
    x = torch.randn(n, dtype=torch.complex128, generator=g).to(DEV).requires_grad_(True)
    for fn in (api.fft, api.bfft, api.ifft):
        assert torch.autograd.gradcheck(fn, (x,), eps=1e-6, atol=1e-9, rtol=1e-7)


@pytest.mark.parametrize("q", [4, 13, 20])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_adjoint_identity(q, dtype):
    n = 1 << q
    x = torch.from_numpy(inputs.generate("normal", 1, n)).to(DEV).to(dtype)
    y = torch.from_numpy(inputs.generate("normal", 2, n)).to(DEV).to(dtype)
    lhs = torch.vdot(api.fft(x).to(torch.complex128), y.to(torch.complex128))
    rhs = torch.vdot(x.to(torch.complex128), api.bfft(y).to(torch.complex128))
    tol = 1e-12 if dtype == torch.complex128 else 1e-5
    assert abs(lhs - rhs) <= tol * abs(lhs)


def test_backward_matches_closed_form_small():
    """d/dx sum |F x|^2 = 2 F^H F x = 2 N x."""
    n = 4096
    x = torch.from_numpy(inputs.generate("normal", 9, n)).to(DEV).requires_grad_(True)
    torch.view_as_real(api.fft(x)).pow(2).sum().backward()
    assert (x.grad - 2 * n * x.detach()).abs().max().item() < 1e-9 * n


@pytest.mark.slow
def test_differentiable_batch_64x2p24_complex64():
    B, q = 64, 24
    n = 1 << q
    x = torch.empty(B, n, dtype=torch.complex64, device=DEV)
    y = torch.empty(B, n, dtype=torch.complex64, device=DEV)
    w = torch.empty(B, n, dtype=torch.float32, device=DEV)
    for b in range(B):
        inputs.fill_normal_torch(x[b], seed=1000 + b)
        inputs.fill_normal_torch(y[b], seed=2000 + b)
        inputs.fill_weights_torch(w[b], seed=3000 + b)
    x.requires_grad_(True)
    f = api.fft(x)
    loss = torch.view_as_real(w * f - y).pow(2).sum()
    loss.backward()
    g = x.grad.detach()
    xd = x.detach()
    del f, loss

    # analytic gradient, FP64 path (the FP64 path is itself oracle-checked)
    rows = [0, 17, 63]
    for b in rows:
        xb = xd[b].to(torch.complex128)
        d = w[b].double() * api.fft(xb) - y[b].to(torch.complex128)
        ga = 2 * api.bfft(w[b].double() * d)
        err = rel_l2(g[b].cpu().numpy(), ga.cpu().numpy())
        print(f"row {b}: autograd (FP32) vs analytic (FP64) rel_l2={err:.3e}", flush=True)
        assert err < 1e-5
    # one row entirely by the CPU FP64 oracle
    b = 17
    xh = xd[b].cpu().numpy()
    wh = w[b].cpu().numpy().astype(np.float64)
    yh = y[b].cpu().numpy().astype(np.complex128)
    dh = wh * oracle.fft(xh) - yh
    gh = 2 * oracle.fft(wh * dh, +1)
    err = rel_l2(g[b].cpu().numpy(), gh)
    print(f"row {b}: autograd vs oracle analytic rel_l2={err:.3e}", flush=True)
    assert err < 1e-5

    # central finite differences on 32 random real coordinates, loss in FP64,
    # differences of the per-element terms taken before the sum
    rng = np.random.default_rng(24)
    eps = 1e-3
    fd, ad = [], []
    for _ in range(32):
        b = int(rng.integers(0, B))
        k = int(rng.integers(0, n))
        comp = int(rng.integers(0, 2))
        xb = xd[b].to(torch.complex128)
        e = torch.zeros_like(xb)
        e[k] = eps if comp == 0 else 1j * eps
        wb = w[b].double()
        yb = y[b].to(torch.complex128)
        dp = wb * api.fft(xb + e) - yb
        dm = wb * api.fft(xb - e) - yb
        diff = (dp.real ** 2 + dp.imag ** 2) - (dm.real ** 2 + dm.imag ** 2)
        fd.append(float(diff.sum()) / (2 * eps))
        ad.append(float(g[b, k].real if comp == 0 else g[b, k].imag))
    fd, ad = np.array(fd), np.array(ad)
    err = np.linalg.norm(fd - ad) / np.linalg.norm(fd)
    print(f"finite differences vs autograd over 32 coordinates: rel_l2={err:.3e} "
          f"max abs diff / rms={np.max(np.abs(fd - ad)) / np.sqrt(np.mean(fd ** 2)):.3e}", flush=True)
    assert err < 1e-4
    assert np.max(np.abs(fd - ad)) < 1e-3 * np.sqrt(np.mean(fd ** 2))
