"""ctypes binding of ``libefft.so`` (the C ABI declared in ``include/efft.h``).

Argument marshalling only: every step of a transform runs in the library's
HIP kernels.  ``torch`` is imported before the library is opened so that the
library binds to the HIP runtime torch already loaded (same SONAME), and
stream handles taken from torch are valid inside it.  There is no fallback:
if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libefft.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "efft.h")

EFFT_C64 = 1
EFFT_C128 = 2
EFFT_FORWARD = -1
EFFT_BACKWARD = 1

_lib = None


class EfftError(RuntimeError):
    """A negative status returned by the library."""

    def __init__(self, status: int, where: str):
        self.status = status
        msg = strerror(status) if _lib is not None else str(status)
        super().__init__(f"{where}: {msg}")


def _bind(lib):
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.efft_plan.argtypes = [i64, ci, ci, ci]
    lib.efft_plan.restype = vp
    lib.efft_plan_scaled.argtypes = [i64, ci, ci, ci, ctypes.c_double]
    lib.efft_plan_scaled.restype = vp
    lib.efft_plan_many.argtypes = [i64, i64, ci, ci, ci, ctypes.c_double]
    lib.efft_plan_many.restype = vp
    lib.efft_plan_batch.argtypes = [vp]
    lib.efft_plan_batch.restype = i64
    lib.efft_plan_digits.argtypes = [i64, i64, ci, ci, ci, ctypes.c_double, ctypes.POINTER(ci), ci]
    lib.efft_plan_digits.restype = vp
    lib.efft_pass_options.argtypes = [vp, ci, ci, ctypes.POINTER(ci)]
    lib.efft_pass_options.restype = ci
    lib.efft_set_pass_options.argtypes = [vp, ci, ci, ctypes.POINTER(ci)]
    lib.efft_set_pass_options.restype = ci
    lib.efft_plan_real.argtypes = [i64, ci, ci, ctypes.c_double]
    lib.efft_plan_real.restype = vp
    lib.efft_exec.argtypes = [vp, vp, vp]
    lib.efft_exec.restype = ci
    lib.efft_exec_oop.argtypes = [vp, vp, vp, vp]
    lib.efft_exec_oop.restype = ci
    lib.efft_exec_events.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(vp), ci]
    lib.efft_exec_events.restype = ci
    lib.efft_exec_scratch.argtypes = [vp, vp, vp, vp]
    lib.efft_exec_scratch.restype = ci
    lib.efft_exec_noalloc.argtypes = [vp, vp, vp]
    lib.efft_exec_noalloc.restype = ci
    lib.efft_scratch_bytes.argtypes = [vp]
    lib.efft_scratch_bytes.restype = i64
    lib.efft_plan_passes_scratch.argtypes = [vp]
    lib.efft_plan_passes_scratch.restype = ci
    lib.efft_destroy.argtypes = [vp]
    lib.efft_destroy.restype = ci
    lib.efft_last_error.argtypes = []
    lib.efft_last_error.restype = ci
    lib.efft_strerror.argtypes = [ci]
    lib.efft_strerror.restype = ctypes.c_char_p
    lib.efft_plan_bytes.argtypes = [vp]
    lib.efft_plan_bytes.restype = i64
    lib.efft_workspace_bytes.argtypes = [vp]
    lib.efft_workspace_bytes.restype = i64
    lib.efft_plan_passes.argtypes = [vp]
    lib.efft_plan_passes.restype = ci
    lib.efft_schedule.argtypes = [i64, ci, ci, ctypes.POINTER(ci), ci, ctypes.POINTER(ci)]
    lib.efft_schedule.restype = ci
    lib.efft_stream_copy.argtypes = [vp, vp, i64, vp]
    lib.efft_stream_copy.restype = ci
    return lib


def load():
    """Open libefft.so (once).  Raises RuntimeError if it has not been built."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (bind to torch's HIP runtime first)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1409_5757_amd.build` "
                "(there is no fallback implementation)")
        _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def header_functions(path: str = HEADER) -> list[str]:
    """Names of the functions declared in include/efft.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(efft_[a-z_]+)\s*\(", text)))


def strerror(status: int) -> str:
    return load().efft_strerror(int(status)).decode()


def check(status: int, where: str) -> int:
    if status < 0:
        raise EfftError(status, where)
    return status


def schedule(n: int, dtype: int, inplace: bool):
    """(digits log2 R_1..R_m, passes) the planner would use; host only."""
    lib = load()
    buf = (ctypes.c_int * 8)()
    passes = ctypes.c_int(0)
    m = check(lib.efft_schedule(int(n), int(dtype), int(bool(inplace)), buf, 8, ctypes.byref(passes)),
              "efft_schedule")
    return [buf[i] for i in range(m)], passes.value
