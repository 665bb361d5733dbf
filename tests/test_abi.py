"""C ABI checks that need no GPU: the library loads, exports every function
include/efft.h declares, rejects invalid arguments with the documented
status, and the host-only planner returns the expected decompositions."""
import ctypes

import pytest

from paper_1409_5757_amd import _lib

C64, C128 = _lib.EFFT_C64, _lib.EFFT_C128


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_function(lib):
    names = _lib.header_functions()
    assert "efft_plan" in names and "efft_exec" in names and "efft_destroy" in names
    for n in names:
        assert hasattr(lib, n), n


def test_status_names(lib):
    codes = {0: "EFFT_OK", -1: "EFFT_ERR_SIZE", -2: "EFFT_ERR_DTYPE", -3: "EFFT_ERR_DIR",
             -4: "EFFT_ERR_NULLPTR", -5: "EFFT_ERR_ALIGN", -6: "EFFT_ERR_PLAN_KIND",
             -7: "EFFT_ERR_OVERLAP", -8: "EFFT_ERR_ALLOC", -9: "EFFT_ERR_HIP",
             -10: "EFFT_ERR_BADPLAN", -11: "EFFT_ERR_ARG"}
    for c, name in codes.items():
        assert _lib.strerror(c).startswith(name)
    assert "unknown" in _lib.strerror(-99)


@pytest.mark.parametrize("n,dtype,direction,inplace,status", [
    (0, C64, -1, 1, -1), (-8, C128, -1, 0, -1), (1 << 35, C64, -1, 1, -1),
    ((1 << 33) + 3, C128, 1, 0, -1), ((1 << 34) - 1, C64, -1, 1, -1),
    (1024, 0, -1, 1, -2), (1024, 3, -1, 1, -2), (1024, C64, 0, 1, -3), (1024, C64, 2, 0, -3),
    (12, 0, -1, 1, -2), (1000, C64, 0, 1, -3),
])
def test_plan_rejects_invalid_arguments(lib, n, dtype, direction, inplace, status):
    """Invalid arguments are rejected before any device work (runs on CPU)."""
    assert lib.efft_plan(n, dtype, direction, inplace) is None
    assert lib.efft_last_error() == status


def test_plan_scaled_rejects_bad_scale(lib):
    for s in (0.0, float("nan"), float("inf")):
        assert lib.efft_plan_scaled(1024, C64, -1, 1, s) is None
        assert lib.efft_last_error() == -11


def test_plan_many_rejects_bad_batch(lib):
    """Batch checks run before any device work (CPU)."""
    for b in (0, -1):
        assert lib.efft_plan_many(1024, b, C64, -1, 1, 1.0) is None
        assert lib.efft_last_error() == -11
    assert lib.efft_plan_many(1 << 20, (1 << 20) + 1, C64, -1, 1, 1.0) is None  # > 2^40 points
    assert lib.efft_last_error() == -1
    assert lib.efft_plan_many((1 << 33) + 1, 2, C64, -1, 1, 1.0) is None  # size check still applies
    assert lib.efft_last_error() == -1
    assert lib.efft_plan_batch(None) == -1


def test_null_and_dead_handles(lib):
    assert lib.efft_destroy(None) == 0
    assert lib.efft_exec(None, None, None) == -4
    assert lib.efft_exec_oop(None, None, None, None) == -4
    assert lib.efft_plan_passes(None) == -1
    assert lib.efft_plan_bytes(None) == -1
    fake = ctypes.create_string_buffer(256)  # never a plan
    assert lib.efft_exec(ctypes.addressof(fake), None, None) == -10
    assert lib.efft_destroy(ctypes.addressof(fake)) == -10


def test_stream_copy_rejects_invalid_arguments(lib):
    """Argument checks happen on the host before anything is enqueued (the
    addresses below are never dereferenced)."""
    a, b = 1 << 20, 1 << 24  # 16-byte aligned, far apart
    assert lib.efft_stream_copy(None, b, 64, None) == -4
    assert lib.efft_stream_copy(a, None, 64, None) == -4
    assert lib.efft_stream_copy(a + 8, b, 64, None) == -5
    assert lib.efft_stream_copy(a, b + 4, 64, None) == -5
    assert lib.efft_stream_copy(a, b, 24, None) == -11
    assert lib.efft_stream_copy(a, b, -16, None) == -11
    assert lib.efft_stream_copy(a, a + 32, 64, None) == -7
    assert lib.efft_stream_copy(a + 32, a, 64, None) == -7
    assert lib.efft_stream_copy(a, b, 0, None) == 0  # nothing to enqueue
    assert lib.efft_stream_copy(a, a, 0, None) == 0  # in place, nothing to enqueue


def _sched(n, dtype, inplace):
    return _lib.schedule(n, dtype, inplace)


@pytest.mark.parametrize("dtype", [C64, C128])
def test_schedule_covers_every_size(dtype):
    for q in range(0, 35):
        for inplace in (True, False):
            digits, passes = _sched(1 << q, dtype, inplace)
            assert sum(digits) == q
            m = len(digits)
            assert passes == m + (1 if inplace and m >= 2 else 0)
            if m >= 2:
                assert all(4 <= d <= 10 for d in digits)
            else:
                assert q <= 12
            if inplace:
                assert digits == digits[::-1], "in-place digits must be palindromic"


def test_schedule_workloads():
    """Pass counts of the benchmark workloads (one pass = one read + one write)."""
    assert _sched(1 << 20, C128, False) == ([10, 10], 2)
    assert _sched(1 << 30, C128, True) == ([10, 10, 10], 4)
    assert _sched(1 << 24, C64, False)[1] == 3
    assert _sched(1 << 32, C64, False)[1] == 4
    assert _sched(1 << 34, C64, True)[1] == 5


def test_schedule_errors():
    lib = _lib.load()
    buf = (ctypes.c_int * 8)()
    p = ctypes.c_int()
    assert lib.efft_schedule(12, C64, 1, buf, 8, ctypes.byref(p)) == -1
    assert lib.efft_schedule(16, 7, 1, buf, 8, ctypes.byref(p)) == -2
    assert lib.efft_schedule(1 << 30, C64, 1, buf, 2, ctypes.byref(p)) == -11
    assert lib.efft_schedule(16, C64, 1, None, 8, ctypes.byref(p)) == -4


def test_binding_refuses_cpu_tensors():
    import torch
    from paper_1409_5757_amd import api
    with pytest.raises(ValueError):
        api.fft(torch.zeros(16, dtype=torch.complex64))


def test_plan_digits_rejects_unusable_decompositions(lib):
    """Checked before any device work (CPU)."""
    def mk(n, inplace, digits):
        arr = (ctypes.c_int * len(digits))(*digits)
        return lib.efft_plan_digits(n, 1, C128, -1, inplace, 1.0, arr, len(digits))
    assert mk(1 << 20, 1, [8, 12]) is None and lib.efft_last_error() == -11      # not a palindrome
    assert mk(1 << 20, 0, [10, 9]) is None and lib.efft_last_error() == -11      # sum != q
    assert mk(1 << 20, 0, [3, 17]) is None and lib.efft_last_error() == -11      # digit out of range
    assert mk(1 << 26, 0, [13, 13]) is None and lib.efft_last_error() == -11     # strided digit > 12
    assert mk(1 << 13, 0, [13]) is None and lib.efft_last_error() == -11         # one digit > 12
    assert mk(1 << 30, 1, [5, 5, 5, 5, 5, 5, 0]) is None and lib.efft_last_error() == -11  # too many
    assert lib.efft_plan_digits(1 << 20, 1, C128, -1, 1, 1.0, None, 2) is None
    assert lib.efft_last_error() == -4
    assert lib.efft_pass_options(None, 0, 0, None) == -4
    assert lib.efft_set_pass_options(None, 0, 0, None) == -4


def test_tuner_decompositions():
    from paper_1409_5757_amd import tune
    assert tune.decompositions(12, True) == [[12]]
    d30 = tune.decompositions(30, True)
    assert [10, 10, 10] in d30 and all(x == x[::-1] and sum(x) == 30 for x in d30)
    assert all(4 <= v <= 12 for x in d30 for v in x) and [9, 12, 9] in d30
    assert all(v <= 10 for x in tune.decompositions(30, True, max_digit=10) for v in x)
    d32 = tune.decompositions(32, False)
    assert [8, 8, 8, 8] in d32 and [10, 10, 6, 6] in d32 and [10, 12, 10] in d32
    assert d32[0] == [10, 12, 10] or len(d32[0]) == 3
