"""Shared helpers of the GPU tests: run the library on seeded inputs and
compare with the FP64 oracle."""
from __future__ import annotations

import numpy as np
import torch

from paper_1409_5757_amd import api, inputs

# parity bars: relative L2 error against the FP64 oracle
TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}
NP = {torch.complex128: np.complex128, torch.complex64: np.complex64}


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    d = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (d if d > 0 else 1.0))


def max_abs(a, b) -> float:
    return float(np.max(np.abs(np.asarray(a, np.complex128) - np.asarray(b, np.complex128)))) if len(a) else 0.0


def host_input(family: str, seed: int, n: int, dtype) -> np.ndarray:
    if family == "tones":
        return inputs.tones(seed, n, dtype=NP[dtype])
    return inputs.generate(family, seed, n, dtype=NP[dtype])


def run_library(x_host: np.ndarray, dtype, direction: int, inplace: bool, scale: float = 1.0):
    """Transform x_host on cuda:0; returns (result, input after the call)."""
    x = torch.from_numpy(x_host).to("cuda")
    p = api.get_plan(x_host.shape[-1], dtype, direction, inplace, scale, x.device)
    if inplace:
        p.execute(x)
        torch.cuda.synchronize()
        return x.cpu().numpy(), None
    out = p.execute(x)
    torch.cuda.synchronize()
    return out.cpu().numpy(), x.cpu().numpy()


def oracle_bins_from_device(x_dev: torch.Tensor, bins, sign: int = -1, chunk: int = 1 << 24,
                            progress_every: int = 1 << 31):
    """Eq. "eqf" at `bins` by the CPU oracle, streaming the device input to the
    host chunk by chunk (the values are exactly those the transform reads);
    prints a progress line every `progress_every` input points."""
    import oracle
    n = x_dev.shape[0]
    acc = None
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        h = x_dev[s:s + m].cpu().numpy()
        acc = oracle.dft_bins(h, bins, sign=sign, n=n, offset=s, acc=acc)
        if (s + m) % progress_every == 0 and s + m < n:
            print(f"  direct sum at {len(bins)} bins: {s + m} of {n} points", flush=True)
    return oracle.bins_value(acc)


def sample_bins(n: int, count: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    fixed = [0, 1, n // 2, n - 1] if n > 1 else [0]
    return np.unique(np.concatenate([fixed, rng.integers(0, n, count)])).astype(np.int64)


def device_rel_l2(a: torch.Tensor, b: torch.Tensor, chunk: int = 1 << 26) -> float:
    """||a - b|| / ||b|| over two device tensors, accumulated in FP64 by chunks."""
    num = 0.0
    den = 0.0
    for s in range(0, a.shape[0], chunk):
        d = (a[s:s + chunk].to(torch.complex128) - b[s:s + chunk].to(torch.complex128))
        num += float(torch.sum(d.real ** 2 + d.imag ** 2))
        bb = b[s:s + chunk].to(torch.complex128)
        den += float(torch.sum(bb.real ** 2 + bb.imag ** 2))
        del d, bb
    return (num / den) ** 0.5 if den > 0 else num ** 0.5


def tone_spectrum_errors(y, seed: int, n: int):
    """Error of the forward transform ``y`` (on the device) of
    ``inputs.fill_tones_torch(seed)`` against its exact spectrum on every bin
    (N e^{i phi} at the 8 tone bins, zero elsewhere): (relative L2 over all N
    bins, largest absolute error / N, largest tone-bin error / N).  N is the
    largest |F_k|.  The tone bins of ``y`` are zeroed."""
    f, v = inputs.tone_spectrum_peaks(seed, n)
    fi = torch.from_numpy(f).to(y.device)
    perr = np.abs(y[fi].cpu().numpy().astype(np.complex128) - v)
    y[fi] = 0
    off_sq, off_max = 0.0, 0.0
    for i in range(0, n, 1 << 26):
        a = y[i:i + (1 << 26)].abs().double()
        off_sq += float(torch.sum(a * a))
        off_max = max(off_max, float(a.max()))
    rel = ((off_sq + float(np.sum(perr ** 2))) / float(np.sum(np.abs(v) ** 2))) ** 0.5
    return rel, max(off_max, float(perr.max())) / n, float(perr.max()) / n
