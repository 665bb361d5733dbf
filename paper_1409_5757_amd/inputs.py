"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle side.

This module holds no part of the transform: it only draws numbers.  Every
value is a pure function of ``(seed, element index)``, so any chunk of an
arbitrarily long signal can be regenerated on its own, on the host (numpy) or
on the GPU (torch integer ops), with identical bits for the uniform family.

Generator: SplitMix64 used in counter mode (G. Steele, D. Lea, C. Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): the 64-bit
word for counter ``c`` under key ``K`` is ``mix64(K + (c + 1) * GAMMA)`` with
GAMMA the golden-ratio increment and ``mix64`` the published finaliser.  A
double in [0, 1) is the top 53 bits times 2^-53.

Families (the workloads' input recipes):

* ``uniform``  re, im i.i.d. U[lo, hi) (default [-1, 1)); counters 2e and 2e+1.
* ``normal``   re, im i.i.d. N(0, 1) by Box-Muller on the two uniforms of
               element e (host only: it uses libm transcendental functions).
* ``tones``    sum of ``count`` unit complex exponentials with distinct integer
               frequencies f_m in [0, N) and phases phi_m in [0, 2*pi):
               x_n = sum_m exp(i*(2*pi*((f_m*n) mod N)/N + phi_m)).  Built in
               FP64 with the phase index reduced exactly in integers.

complex64 requests draw in FP64 and round once to FP32.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK64 = (1 << 64) - 1

# one key per family, so different families with one seed are independent
_FAMILY_SALT = {"uniform": 0x0123456789ABCDEF, "normal": 0x0F1E2D3C4B5A6978,
                "weights": 0x5A5A5A5A12345678}

DEFAULT_CHUNK = 1 << 22


def _mix64_int(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * _M1) & _MASK64
    z = ((z ^ (z >> 27)) * _M2) & _MASK64
    return z ^ (z >> 31)


def family_key(seed: int, family: str) -> int:
    """64-bit key of one (seed, family) stream."""
    return _mix64_int((int(seed) * GAMMA + _FAMILY_SALT[family]) & _MASK64)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(_M1)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def unit_doubles(key: int, first_counter: int, count: int) -> np.ndarray:
    """Doubles in [0, 1) for counters first_counter .. first_counter+count-1."""
    with np.errstate(over="ignore"):
        c = np.arange(first_counter + 1, first_counter + 1 + count, dtype=np.uint64)
        z = np.uint64(key) + c * np.uint64(GAMMA)
        z = _mix64_np(z)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _chunk_values(family: str, key: int, offset: int, n: int, lo: float, hi: float) -> np.ndarray:
    u = unit_doubles(key, 2 * offset, 2 * n)
    out = np.empty(n, dtype=np.complex128)
    if family == "normal":
        u1 = 1.0 - u[0::2]  # (0, 1]
        ang = 2.0 * np.pi * u[1::2]
        r = np.sqrt(-2.0 * np.log(u1))
        out.real = r * np.cos(ang)
        out.imag = r * np.sin(ang)
    else:
        out.real = lo + (hi - lo) * u[0::2]
        out.imag = lo + (hi - lo) * u[1::2]
    return out


def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def generate(family: str, seed: int, n: int, dtype=np.complex128, offset: int = 0,
             lo: float = -1.0, hi: float = 1.0, chunk: int = DEFAULT_CHUNK) -> np.ndarray:
    """Elements [offset, offset+n) of the (family, seed) signal as a numpy array.

    ``family`` is ``"uniform"`` (re, im ~ U[lo, hi)) or ``"normal"`` (re, im ~ N(0,1)).
    """
    if family not in ("uniform", "normal"):
        raise ValueError(f"unknown family {family!r}")
    key = family_key(seed, family)
    dtype = np.dtype(dtype)
    out = np.empty(n, dtype=dtype)

    def work(start: int) -> None:
        m = min(chunk, n - start)
        v = _chunk_values(family, key, offset + start, m, lo, hi)
        out[start:start + m] = v if dtype == np.complex128 else v.astype(dtype)

    starts = list(range(0, n, chunk))
    if len(starts) <= 1:
        for s in starts:
            work(s)
    else:
        with ThreadPoolExecutor(max_workers=_workers()) as ex:
            list(ex.map(work, starts))
    return out


def real_weights(seed: int, n: int, dtype=np.float32, offset: int = 0) -> np.ndarray:
    """Real weights w ~ U[0, 1) (the loss weights of the differentiable batch)."""
    key = family_key(seed, "weights")
    return unit_doubles(key, offset, n).astype(dtype)


def tone_params(seed: int, n: int, count: int = 8):
    """Distinct integer frequencies and phases of the sparse-spectrum signal."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 0x70E5])))
    count = min(count, n)
    freqs = rng.choice(n, size=count, replace=False) if n <= (1 << 24) else \
        np.unique(rng.integers(0, n, size=4 * count, dtype=np.int64))[:count]
    while freqs.shape[0] < count:  # pragma: no cover - astronomically unlikely
        extra = rng.integers(0, n, size=count, dtype=np.int64)
        freqs = np.unique(np.concatenate([freqs, extra]))[:count]
    phases = rng.uniform(0.0, 2.0 * np.pi, size=count)
    return np.asarray(freqs, dtype=np.int64), phases


def tones(seed: int, n: int, count: int = 8, dtype=np.complex128, offset: int = 0,
          length: int | None = None, chunk: int = DEFAULT_CHUNK) -> np.ndarray:
    """Elements [offset, offset+length) of the sum-of-tones signal of length n."""
    freqs, phases = tone_params(seed, n, count)
    length = n - offset if length is None else length
    out = np.empty(length, dtype=np.dtype(dtype))

    def work(start: int) -> None:
        m = min(chunk, length - start)
        idx = np.arange(offset + start, offset + start + m, dtype=np.uint64)
        acc = np.zeros(m, dtype=np.complex128)
        mask = np.uint64(n - 1)
        with np.errstate(over="ignore"):
            for f, ph in zip(freqs, phases):
                ph_idx = (idx * np.uint64(f)) & mask  # exact (n is a power of two)
                ang = (2.0 * np.pi / n) * ph_idx.astype(np.float64) + ph
                acc += np.cos(ang) + 1j * np.sin(ang)
        out[start:start + m] = acc.astype(out.dtype)

    starts = list(range(0, length, chunk))
    if len(starts) <= 1:
        for s in starts:
            work(s)
    else:
        with ThreadPoolExecutor(max_workers=_workers()) as ex:
            list(ex.map(work, starts))
    return out


def tone_spectrum_peaks(seed: int, n: int, count: int = 8, sign: int = -1):
    """Exact nonzero bins of the forward (sign=-1) DFT of ``tones``: N*exp(i*phi) at f."""
    freqs, phases = tone_params(seed, n, count)
    if sign == -1:
        return freqs, n * np.exp(1j * phases)
    # backward transform peaks sit at (-f) mod N
    return (-freqs) % n, n * np.exp(1j * phases)


# ---------------------------------------------------------------- torch side
def _lsr(t, k: int):
    """Logical right shift of an int64 torch tensor viewed as uint64."""
    import torch
    return torch.bitwise_and(torch.bitwise_right_shift(t, k), (1 << (64 - k)) - 1)


def _to_i64(v: int) -> int:
    v &= _MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def unit_doubles_torch(key: int, first_counter: int, count: int, device):
    """Bit-identical torch version of ``unit_doubles`` (runs on any device)."""
    import torch
    c = torch.arange(first_counter + 1, first_counter + 1 + count, dtype=torch.int64, device=device)
    z = c * _to_i64(GAMMA) + _to_i64(key)
    z = z ^ _lsr(z, 30)
    z = z * _to_i64(_M1)
    z = z ^ _lsr(z, 27)
    z = z * _to_i64(_M2)
    z = z ^ _lsr(z, 31)
    return _lsr(z, 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def fill_uniform_torch(out, seed: int, offset: int = 0, lo: float = -1.0, hi: float = 1.0,
                       chunk: int = 1 << 25) -> None:
    """Fill a 1D complex torch tensor (any device) with ``generate('uniform', ...)``."""
    import torch
    key = family_key(seed, "uniform")
    n = out.shape[0]
    real_dtype = torch.float64 if out.dtype == torch.complex128 else torch.float32
    view = torch.view_as_real(out)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        u = unit_doubles_torch(key, 2 * (offset + s), 2 * m, out.device)
        v = (lo + (hi - lo) * u).view(m, 2)
        view[s:s + m].copy_(v.to(real_dtype))
        del u, v


def fill_from_host(out, family: str, seed: int, chunk: int = 1 << 24, **kw) -> None:
    """Fill a 1D complex torch tensor chunk by chunk from host-generated values."""
    import torch
    n = out.shape[0]
    np_dtype = np.complex128 if out.dtype == torch.complex128 else np.complex64
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        if family == "tones":
            v = tones(seed, n, dtype=np_dtype, offset=s, length=m, **kw)
        else:
            v = generate(family, seed, m, dtype=np_dtype, offset=s, **kw)
        out[s:s + m].copy_(torch.from_numpy(v), non_blocking=False)


def fill_normal_torch(out, seed: int, offset: int = 0, chunk: int = 1 << 25) -> None:
    """Fill a 1D complex torch tensor with i.i.d. standard normal re, im by the
    same Box-Muller recipe as ``generate('normal', ...)`` applied to the same
    counter-based uniforms (bit-identical uniforms; the transcendental
    functions of the device may round differently from the host's)."""
    import torch
    key = family_key(seed, "normal")
    n = out.shape[0]
    real_dtype = torch.float64 if out.dtype == torch.complex128 else torch.float32
    view = torch.view_as_real(out)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        u = unit_doubles_torch(key, 2 * (offset + s), 2 * m, out.device).view(m, 2)
        r = torch.sqrt(-2.0 * torch.log(1.0 - u[:, 0]))
        ang = (2.0 * np.pi) * u[:, 1]
        view[s:s + m, 0].copy_((r * torch.cos(ang)).to(real_dtype))
        view[s:s + m, 1].copy_((r * torch.sin(ang)).to(real_dtype))
        del u, r, ang


def fill_tones_torch(out, seed: int, count: int = 8, chunk: int = 1 << 25) -> None:
    """Fill a 1D complex torch tensor of length N with the sum-of-tones signal
    of ``tone_params(seed, N, count)``, synthesised on the tensor's device in
    FP64 with the phase index (f*n) mod N reduced exactly in integers."""
    import torch
    n = out.shape[0]
    freqs, phases = tone_params(seed, n, count)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        idx = torch.arange(s, s + m, dtype=torch.int64, device=out.device)
        acc = torch.zeros(m, dtype=torch.complex128, device=out.device)
        for f, ph in zip(freqs.tolist(), phases.tolist()):
            k = torch.bitwise_and(idx * int(f), n - 1).to(torch.float64)
            ang = k * (2.0 * np.pi / n) + ph
            acc += torch.complex(torch.cos(ang), torch.sin(ang))
        out[s:s + m].copy_(acc.to(out.dtype))
        del idx, acc


def fill_weights_torch(out, seed: int, offset: int = 0, chunk: int = 1 << 25) -> None:
    """Fill a 1D real torch tensor with ``real_weights(seed, ...)`` (U[0, 1))."""
    key = family_key(seed, "weights")
    n = out.shape[0]
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        out[s:s + m].copy_(unit_doubles_torch(key, offset + s, m, out.device).to(out.dtype))
