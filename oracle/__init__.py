"""CPU FP64 reference for the 1D complex DFT (paper Section 1, Eq. "eqf").

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_1409_5757_amd``) never imports, links or calls it, and the two share
no code: this wrapper only marshals numpy arrays into ``efft_oracle.c``.

Functions
---------
fft(x, sign=-1)
    Radix-2 Cooley-Tukey FFT in FP64 (Section 2.2, Eqs. "eqb"/"eqct"/"eqctt"),
    returns a new complex128 array.  ``sign=-1`` is the paper's forward
    transform, ``sign=+1`` the unnormalised backward transform.
dft_bins(x, bins, sign=-1, n=None, offset=0, acc=None)
    Direct evaluation of Eq. "eqf" at chosen bins.  May be called chunk by
    chunk (``offset`` = index of the chunk's first element, ``n`` = transform
    length, ``acc`` = the accumulator returned by the previous call); finish
    with ``bins_value(acc)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "efft_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(mutant: int = 0, out_path: str | None = None) -> str:
    """Compile the oracle with gcc/OpenMP; ``mutant > 0`` plants a mistake (tests only)."""
    out = out_path or _LIB_PATH
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
           f"-DORACLE_MUTANT={int(mutant)}", _SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def _bind(lib):
    i64, dp, vp = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
    lib.oracle_fft.argtypes = [dp, i64, ctypes.c_int]
    lib.oracle_fft.restype = ctypes.c_int
    lib.oracle_fft_from_f32.argtypes = [vp, dp, i64, ctypes.c_int]
    lib.oracle_fft_from_f32.restype = ctypes.c_int
    lib.oracle_dft_bins.argtypes = [vp, ctypes.c_int, i64, i64, i64, ctypes.c_int, vp, i64, dp]
    lib.oracle_dft_bins.restype = ctypes.c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    return lib


def load(path: str | None = None):
    """Load the compiled oracle (building it first only if it is missing)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def threads(lib=None) -> int:
    return (lib or load()).oracle_threads()


def fft(x, sign: int = -1, lib=None) -> np.ndarray:
    """FP64 radix-2 FFT of a 1D complex array whose length is a power of two."""
    lib = lib or load()
    x = np.asarray(x)
    n = x.shape[0]
    if x.dtype == np.complex64:
        src = np.ascontiguousarray(x)
        out = np.empty(n, dtype=np.complex128)
        rc = lib.oracle_fft_from_f32(src.ctypes.data, out.ctypes.data, n, int(sign))
    else:
        out = np.array(x, dtype=np.complex128, copy=True, order="C")
        rc = lib.oracle_fft(out.ctypes.data, n, int(sign))
    if rc != 0:
        raise ValueError(f"oracle_fft failed (rc={rc}) for n={n}")
    return out


def dft_bins(x, bins, sign: int = -1, n: int | None = None, offset: int = 0,
             acc: np.ndarray | None = None, lib=None) -> np.ndarray:
    """Accumulate Eq. "eqf" at ``bins`` over the slice ``x`` starting at ``offset``."""
    lib = lib or load()
    x = np.ascontiguousarray(x)
    if x.dtype not in (np.complex64, np.complex128):
        x = x.astype(np.complex128)
    bins = np.ascontiguousarray(np.asarray(bins, dtype=np.int64))
    n = x.shape[0] if n is None else int(n)
    if acc is None:
        acc = np.zeros((bins.shape[0], 4), dtype=np.float64)
    rc = lib.oracle_dft_bins(x.ctypes.data, int(x.dtype == np.complex64), int(offset),
                             x.shape[0], n, int(sign), bins.ctypes.data, bins.shape[0],
                             acc.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_dft_bins failed (rc={rc})")
    return acc


def bins_value(acc: np.ndarray) -> np.ndarray:
    """Complex bin values from a Kahan accumulator returned by ``dft_bins``."""
    return (acc[:, 0] - acc[:, 1]) + 1j * (acc[:, 2] - acc[:, 3])


def dft_at(x, bins, sign: int = -1, lib=None) -> np.ndarray:
    """One-shot direct DFT of the whole array ``x`` at ``bins``."""
    return bins_value(dft_bins(x, bins, sign=sign, lib=lib))


def dft(x, sign: int = -1, lib=None) -> np.ndarray:
    """Eq. "eqf" at every bin by the direct sum: O(N^2), any length N >= 1
    (the reference for lengths that are not powers of two)."""
    x = np.asarray(x)
    return dft_at(x, np.arange(x.shape[0], dtype=np.int64), sign=sign, lib=lib)
