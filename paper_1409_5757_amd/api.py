"""Python front end of the gfx950 FFT library (argument marshalling only).

``fft(x)``   forward transform of Eq. "eqf" (paper, Section 1) along the last
             dimension: F_k = sum_n x_n exp(-2*pi*i*k*n/N), unnormalised.
``bfft(x)``  backward (conjugate-sign) transform, unnormalised: the adjoint.
``ifft(x)``  inverse DFT = bfft(x) / N; the 1/N = 2^-q factor is applied
             inside the library's last pass and is exact.
``rfft(x)``  real input of length N -> bins F_0 .. F_{N/2} (N/2 + 1 complex).
``irfft(X)`` N/2 + 1 Hermitian bins -> N real samples, scaled by 1/N.

Inputs are complex64 / complex128 CUDA tensors whose last dimension N is a
power of two (N = 2^q, q <= 34) or any other length 3 <= N <= 2^33 (done by
the library's chirp path; ``ifft`` then scales by the rounded 1/N).  Leading dimensions are a batch of
independent transforms, done by one batched plan (every pass of the
transform covers all rows at once).  All work runs in ``libefft.so`` on the
tensor's device, on the current torch stream; there is no CPU fallback.

``EfftFFT`` is the differentiable form: for the C-linear map y = s * A x its
backward applies s * A^H, the transform of the opposite direction with the
same scale, to the incoming gradient (PyTorch's convention for complex
autograd: grad_x = A^H grad_y).
"""
from __future__ import annotations

import collections
import ctypes
import threading

import torch

from . import _lib
from ._lib import EFFT_BACKWARD, EFFT_C64, EFFT_C128, EFFT_FORWARD, EfftError

_DTYPES = {torch.complex64: EFFT_C64, torch.complex128: EFFT_C128}


class Plan:
    """One committed transform (size, batch, dtype, direction, in/out of place,
    scale).  Each execution transforms ``batch`` contiguous signals of n points."""

    def __init__(self, n: int, dtype: torch.dtype, direction: int = EFFT_FORWARD,
                 inplace: bool = False, scale: float = 1.0, device=None, batch: int = 1):
        if dtype not in _DTYPES:
            raise TypeError(f"dtype must be torch.complex64 or torch.complex128, got {dtype}")
        self.lib = _lib.load()
        self.n = int(n)
        self.batch = int(batch)
        self.dtype = dtype
        self.direction = int(direction)
        self.inplace = bool(inplace)
        self.scale = float(scale)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            h = self.lib.efft_plan_many(self.n, self.batch, _DTYPES[dtype], self.direction,
                                        int(self.inplace), self.scale)
        if not h:
            raise EfftError(self.lib.efft_last_error(), "efft_plan_many")
        self.handle = ctypes.c_void_p(h)
        self.passes = self.lib.efft_plan_passes(self.handle)
        self.scratch_passes = self.lib.efft_plan_passes_scratch(self.handle)
        self.scratch_bytes = int(self.lib.efft_scratch_bytes(self.handle))

    def make_scratch(self) -> torch.Tensor | None:
        """A scratch tensor for ``execute(..., scratch=...)`` (None if unused)."""
        if self.scratch_bytes <= 0:
            return None
        shape = (self.n,) if self.batch == 1 else (self.batch, self.n)
        return torch.empty(shape, dtype=self.dtype, device=self.device)

    def _check(self, t: torch.Tensor, name: str):
        if t.dtype != self.dtype:
            raise TypeError(f"{name}: expected {self.dtype}, got {t.dtype}")
        if t.device != self.device:
            raise ValueError(f"{name}: expected a tensor on {self.device}, got {t.device}")
        if t.shape[-1] != self.n:
            raise ValueError(f"{name}: last dimension {t.shape[-1]} != plan size {self.n}")
        if (t.numel() // self.n if self.n else 0) % self.batch:
            raise ValueError(f"{name}: {t.numel() // self.n} rows is not a multiple of the plan batch {self.batch}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: tensor must be contiguous")

    def execute(self, x: torch.Tensor, out: torch.Tensor | None = None, stream=None,
                scratch: torch.Tensor | None = None) -> torch.Tensor:
        """Transform every length-N row of x, ``batch`` rows per library call;
        in place for in-place plans (with ``scratch``, a tensor of batch * N
        elements of the plan's dtype, one pass fewer)."""
        self._check(x, "input")
        s = ctypes.c_void_p((stream or torch.cuda.current_stream(self.device)).cuda_stream)
        rows = (x.numel() // self.n if self.n else 0) // self.batch
        xp = x.data_ptr()
        step = self.batch * self.n * x.element_size()
        if self.inplace:
            if scratch is not None:
                self._check(scratch, "scratch")
                if scratch.numel() < self.batch * self.n:
                    raise ValueError("scratch: needs batch * N elements")
                sp = ctypes.c_void_p(scratch.data_ptr())
                for r in range(rows):
                    _lib.check(self.lib.efft_exec_scratch(self.handle, ctypes.c_void_p(xp + r * step), sp, s),
                               "efft_exec_scratch")
                return x
            for r in range(rows):
                _lib.check(self.lib.efft_exec(self.handle, ctypes.c_void_p(xp + r * step), s), "efft_exec")
            return x
        if out is None:
            out = torch.empty_like(x)
        self._check(out, "output")
        op = out.data_ptr()
        for r in range(rows):
            _lib.check(self.lib.efft_exec_oop(self.handle, ctypes.c_void_p(xp + r * step),
                                              ctypes.c_void_p(op + r * step), s), "efft_exec_oop")
        return out

    def execute_events(self, x: torch.Tensor, out: torch.Tensor, events, stream=None,
                       scratch: torch.Tensor | None = None) -> None:
        """One transform of a single signal, recording caller-created hipEvents
        before each pass and after the last (``len(events) == passes + 1``)."""
        s = ctypes.c_void_p((stream or torch.cuda.current_stream(self.device)).cuda_stream)
        arr = (ctypes.c_void_p * len(events))(*events)
        sc = ctypes.c_void_p(scratch.data_ptr()) if scratch is not None else None
        _lib.check(self.lib.efft_exec_events(self.handle, ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()), sc, s, arr, len(events)),
                   "efft_exec_events")

    def device_bytes(self) -> int:
        return int(self.lib.efft_plan_bytes(self.handle))

    def close(self) -> None:
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.efft_destroy(h)
            self.handle = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order varies
        try:
            self.close()
        except Exception:
            pass


_REAL_OF = {torch.complex64: torch.float32, torch.complex128: torch.float64}
_COMPLEX_OF = {torch.float32: torch.complex64, torch.float64: torch.complex128}


class RealPlan:
    """Real-data transform of N = 2^q samples (out of place): forward maps N
    reals to N/2 + 1 bins, backward maps N/2 + 1 Hermitian bins to N reals."""

    def __init__(self, n: int, real_dtype: torch.dtype, direction: int = EFFT_FORWARD,
                 scale: float = 1.0, device=None):
        if real_dtype not in _COMPLEX_OF:
            raise TypeError(f"real dtype must be float32 or float64, got {real_dtype}")
        self.lib = _lib.load()
        self.n = int(n)
        self.real_dtype = real_dtype
        self.complex_dtype = _COMPLEX_OF[real_dtype]
        self.direction = int(direction)
        self.scale = float(scale)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else torch.device(device).index or 0)
        with torch.cuda.device(self.device):
            h = self.lib.efft_plan_real(self.n, _DTYPES[self.complex_dtype], self.direction, self.scale)
        if not h:
            raise EfftError(self.lib.efft_last_error(), "efft_plan_real")
        self.handle = ctypes.c_void_p(h)
        self.passes = self.lib.efft_plan_passes(self.handle)

    def execute(self, x: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        fwd = self.direction == EFFT_FORWARD
        in_dtype, in_len = (self.real_dtype, self.n) if fwd else (self.complex_dtype, self.n // 2 + 1)
        out_dtype, out_len = (self.complex_dtype, self.n // 2 + 1) if fwd else (self.real_dtype, self.n)
        if x.dtype != in_dtype or x.shape[-1] != in_len or x.device != self.device or not x.is_contiguous():
            raise ValueError(f"input must be a contiguous {in_dtype} tensor on {self.device} "
                             f"with last dimension {in_len}")
        if out is None:
            out = torch.empty(*x.shape[:-1], out_len, dtype=out_dtype, device=self.device)
        if out.dtype != out_dtype or out.shape[-1] != out_len or not out.is_contiguous():
            raise ValueError(f"output must be a contiguous {out_dtype} tensor with last dimension {out_len}")
        s = ctypes.c_void_p((stream or torch.cuda.current_stream(self.device)).cuda_stream)
        rows = x.numel() // in_len
        istep, ostep = in_len * x.element_size(), out_len * out.element_size()
        xp, op = x.data_ptr(), out.data_ptr()
        for r in range(rows):
            _lib.check(self.lib.efft_exec_oop(self.handle, ctypes.c_void_p(xp + r * istep),
                                              ctypes.c_void_p(op + r * ostep), s), "efft_exec_oop")
        return out

    def execute_events(self, x: torch.Tensor, out: torch.Tensor, events, stream=None) -> None:
        s = ctypes.c_void_p((stream or torch.cuda.current_stream(self.device)).cuda_stream)
        arr = (ctypes.c_void_p * len(events))(*events)
        _lib.check(self.lib.efft_exec_events(self.handle, ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()), None, s, arr, len(events)),
                   "efft_exec_events")

    def device_bytes(self) -> int:
        return int(self.lib.efft_plan_bytes(self.handle))

    def close(self) -> None:
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.efft_destroy(h)
            self.handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


# Plans made by the functional calls (fft, ifft, ...) are kept for reuse, the
# most recently used last.  The cache is bounded by a count and by the device
# bytes its plans hold (plans for lengths that are not powers of two own work
# arrays as large as the signal); the least recently used plans go first, after
# a synchronisation of their device, since work may still be queued on them.
# Plans are created (allocated) on first use: code that captures a HIP graph
# should make its plans before the capture, e.g. by one eager call or with Plan.
_cache: "collections.OrderedDict" = collections.OrderedDict()
_cache_lock = threading.Lock()
CACHE_MAX_PLANS = 64
CACHE_MAX_BYTES = 8 << 30


def _owns_work_arrays(n: int) -> bool:
    return n >= 3 and (n & (n - 1)) != 0


def _evict_locked() -> None:
    total = sum(p.device_bytes() for p in _cache.values())
    while _cache and (len(_cache) > CACHE_MAX_PLANS or total > CACHE_MAX_BYTES):
        _, old = _cache.popitem(last=False)
        total -= old.device_bytes()
        torch.cuda.synchronize(old.device)
        old.close()


def get_plan(n: int, dtype: torch.dtype, direction: int, inplace: bool, scale: float,
             device: torch.device, batch: int = 1) -> Plan:
    """Cached plan keyed by (N, batch, dtype, direction, in place, scale,
    device), and for lengths that are not powers of two also by the current
    stream: such plans own work arrays, so two streams must not share one."""
    key = (int(n), int(batch), dtype, int(direction), bool(inplace), float(scale), device)
    if _owns_work_arrays(int(n)):
        key += (torch.cuda.current_stream(device).cuda_stream,)
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            p = Plan(n, dtype, direction, inplace, scale, device, batch)
            _cache[key] = p
            _evict_locked()
        else:
            _cache.move_to_end(key)
        return p


def clear_plan_cache() -> None:
    with _cache_lock:
        for p in _cache.values():
            torch.cuda.synchronize(p.device)
            p.close()
        _cache.clear()


def _transform(x: torch.Tensor, direction: int, scale: float, inplace: bool,
               out: torch.Tensor | None = None) -> torch.Tensor:
    if not x.is_cuda:
        raise ValueError("efft transforms run on the GPU only; got a CPU tensor")
    if x.dtype not in _DTYPES:
        raise TypeError(f"dtype must be complex64 or complex128, got {x.dtype}")
    n = x.shape[-1]
    rows = x.numel() // n if n else 1
    p = get_plan(n, x.dtype, direction, inplace, scale, x.device, max(rows, 1))
    if inplace:
        return p.execute(x)
    return p.execute(x.contiguous(), out=out)


class EfftFFT(torch.autograd.Function):
    """y = scale * A_dir x, differentiable; backward applies scale * A_{-dir}."""

    @staticmethod
    def forward(ctx, x, direction: int = EFFT_FORWARD, scale: float = 1.0):
        ctx.direction = direction
        ctx.scale = scale
        return _transform(x, direction, scale, inplace=False)

    @staticmethod
    def backward(ctx, g):
        return _transform(g.contiguous(), -ctx.direction, ctx.scale, inplace=False), None, None


def fft(x: torch.Tensor, inplace: bool = False, out: torch.Tensor | None = None) -> torch.Tensor:
    """Forward DFT along the last dimension (sign -1, unnormalised)."""
    if not inplace and torch.is_grad_enabled() and x.requires_grad:
        return EfftFFT.apply(x, EFFT_FORWARD, 1.0)
    return _transform(x, EFFT_FORWARD, 1.0, inplace, out)


def bfft(x: torch.Tensor, inplace: bool = False, out: torch.Tensor | None = None) -> torch.Tensor:
    """Backward DFT along the last dimension (sign +1, unnormalised)."""
    if not inplace and torch.is_grad_enabled() and x.requires_grad:
        return EfftFFT.apply(x, EFFT_BACKWARD, 1.0)
    return _transform(x, EFFT_BACKWARD, 1.0, inplace, out)


def ifft(x: torch.Tensor, inplace: bool = False, out: torch.Tensor | None = None) -> torch.Tensor:
    """Inverse DFT along the last dimension: bfft(x) / N."""
    scale = 1.0 / x.shape[-1]
    if not inplace and torch.is_grad_enabled() and x.requires_grad:
        return EfftFFT.apply(x, EFFT_BACKWARD, scale)
    return _transform(x, EFFT_BACKWARD, scale, inplace, out)


def get_real_plan(n: int, real_dtype: torch.dtype, direction: int, scale: float,
                  device: torch.device) -> RealPlan:
    key = ("real", int(n), real_dtype, int(direction), float(scale), device)
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            p = RealPlan(n, real_dtype, direction, scale, device)
            _cache[key] = p
            _evict_locked()
        else:
            _cache.move_to_end(key)
        return p


def rfft(x: torch.Tensor) -> torch.Tensor:
    """Forward DFT of real input along the last dimension: bins 0 .. N/2."""
    if not x.is_cuda:
        raise ValueError("efft transforms run on the GPU only; got a CPU tensor")
    return get_real_plan(x.shape[-1], x.dtype, EFFT_FORWARD, 1.0, x.device).execute(x.contiguous())


def irfft(x: torch.Tensor, n: int | None = None) -> torch.Tensor:
    """Inverse of rfft: N/2 + 1 Hermitian bins -> N real samples (scaled 1/N)."""
    if not x.is_cuda:
        raise ValueError("efft transforms run on the GPU only; got a CPU tensor")
    n = 2 * (x.shape[-1] - 1) if n is None else int(n)
    if x.dtype not in _REAL_OF:
        raise TypeError(f"dtype must be complex64 or complex128, got {x.dtype}")
    return get_real_plan(n, _REAL_OF[x.dtype], EFFT_BACKWARD, 1.0 / n, x.device).execute(x.contiguous())
