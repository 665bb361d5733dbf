"""MI355X (gfx950) library for one very large 1D complex-to-complex FFT.

The transform of Eq. "eqf" (Asai & Vladimirov, "EFFT", Section 1) runs in
hand-written HIP kernels behind the C ABI of ``include/efft.h``
(``libefft.so``); this package is the thin Python binding over it.
Importing the package does not open the library; the first transform does,
and raises if it has not been built.
"""

EFFT_C64 = 1
EFFT_C128 = 2
EFFT_FORWARD = -1
EFFT_BACKWARD = 1

__all__ = ["fft", "bfft", "ifft", "rfft", "irfft", "EfftFFT", "Plan", "RealPlan", "get_plan", "schedule",
           "EFFT_C64", "EFFT_C128", "EFFT_FORWARD", "EFFT_BACKWARD"]


def __getattr__(name):
    if name in ("fft", "bfft", "ifft", "rfft", "irfft", "EfftFFT", "Plan", "RealPlan", "get_plan",
                "get_real_plan", "clear_plan_cache"):
        from . import api
        return getattr(api, name)
    if name in ("schedule", "EfftError", "load", "strerror"):
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
