"""CPU pins of the oracle (no GPU): the oracle is checked against the DFT's
definition (paper, Section 1, Eq. "eqf"), an arbitrary-precision evaluation
(Section 5.3's method), a library FFT, hand-worked values and identities."""
import os
import tempfile

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from tests import pins


def test_battery_passes_on_oracle(oracle_lib):
    assert pins.battery(oracle_lib) == []


@pytest.mark.parametrize("mutant", range(1, 11))
def test_battery_catches_planted_mistake(mutant):
    """Each planted mistake (sign, reordering, twiddle index, dropped twiddle,
    swapped outputs, wrong operand, skipped k=0, short bit reversal) must
    fail at least one pin."""
    with tempfile.TemporaryDirectory() as d:
        path = oracle.build(mutant=mutant, out_path=os.path.join(d, f"mut{mutant}.so"))
        lib = oracle.load(path)
        assert pins.battery(lib) != []


def test_golden_cases_exact(oracle_lib):
    for c in pins.read_golden():
        got = oracle.fft(c["x"], c["sign"])
        if c["n"] <= 4:
            assert np.array_equal(got, c["F"]), c["name"]
        else:
            np.testing.assert_allclose(got, c["F"], rtol=0, atol=1e-13)


def test_sizes_one_two_four_bit_exact_small_integers(oracle_lib):
    rng = np.random.default_rng(3)
    for n in (1, 2, 4):
        for _ in range(20):
            x = rng.integers(-8, 9, n) + 1j * rng.integers(-8, 9, n)
            for sign in (-1, 1):
                assert np.array_equal(oracle.fft(x, sign), pins.brute_dft(x, sign).round())


def test_library_fft_cross_check(oracle_lib):
    """numpy's pocketfft is a third opinion at sizes the brute force cannot reach."""
    for q in (10, 14, 18, 20):
        n = 1 << q
        rng = np.random.default_rng(q)
        x = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
        assert pins.rel_l2(oracle.fft(x), np.fft.fft(x)) < 2e-15
        assert pins.rel_l2(oracle.fft(x, +1), np.fft.ifft(x) * n) < 2e-15


def test_complex64_input_is_upcast_exactly(oracle_lib):
    rng = np.random.default_rng(11)
    x = (rng.standard_normal(1024) + 1j * rng.standard_normal(1024)).astype(np.complex64)
    np.testing.assert_array_equal(oracle.fft(x), oracle.fft(x.astype(np.complex128)))


def test_mpmath_agreement_256(oracle_lib):
    rng = np.random.default_rng(256)
    x = rng.uniform(-0.5, 0.5, 64) + 1j * rng.uniform(-0.5, 0.5, 64)
    ref = np.array([complex(v) for v in pins.mp_dft(x, dps=30)])
    assert pins.rel_l2(oracle.fft(x), ref) < 1e-15


def test_spot_mode_matches_definition(oracle_lib):
    n = 1 << 10
    rng = np.random.default_rng(5)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    bins = [0, 1, 2, 511, 512, 1023, 77]
    for sign in (-1, 1):
        ref = pins.brute_dft(x, sign)[bins]
        got = oracle.dft_at(x, bins, sign)
        assert np.max(np.abs(got - ref)) < 1e-12


def test_spot_mode_chunked_equals_one_shot(oracle_lib):
    n = 1 << 16
    rng = np.random.default_rng(9)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    bins = rng.integers(0, n, 12)
    one = oracle.dft_at(x, bins)
    acc = None
    for s in range(0, n, 5000):
        acc = oracle.dft_bins(x[s:s + 5000], bins, n=n, offset=s, acc=acc)
    chunked = oracle.bins_value(acc)
    assert np.max(np.abs(chunked - one)) < 1e-10
    full = oracle.fft(x)
    assert np.max(np.abs(one - full[bins])) < 1e-10


def test_spot_mode_complex64_input(oracle_lib):
    n = 1 << 12
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    bins = [0, 3, 4095]
    assert np.max(np.abs(oracle.dft_at(x, bins) - oracle.fft(x)[bins])) < 1e-10


def test_spot_mode_large_index_phase_reduction(oracle_lib):
    """Phase indices k*n beyond 2^64 must wrap exactly: a tone at a high
    frequency in a 2^34-length signal, sampled over a chunk far from the start,
    gives exactly the tone's contribution."""
    n = 1 << 34
    f = (1 << 33) + 12345
    offset = (1 << 34) - 4096
    idx = np.arange(offset, offset + 4096, dtype=np.uint64)
    ph = ((idx * np.uint64(f)) & np.uint64(n - 1)).astype(np.float64)
    x = np.exp(2j * np.pi * ph / n)  # the tone's samples on this slice
    val = oracle.bins_value(oracle.dft_bins(x, [f], n=n, offset=offset))
    assert abs(val[0] - 4096) < 1e-8


def test_rejects_non_power_of_two(oracle_lib):
    with pytest.raises(ValueError):
        oracle.fft(np.zeros(12, dtype=np.complex128))


@settings(max_examples=25, deadline=None)
@given(q=st.integers(min_value=0, max_value=11), seed=st.integers(0, 2**31 - 1),
       sign=st.sampled_from([-1, 1]))
def test_random_sizes_against_definition(oracle_lib, q, seed, sign):
    n = 1 << q
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    assert pins.rel_l2(oracle.fft(x, sign), pins.brute_dft(x, sign)) < 1e-14


@settings(max_examples=25, deadline=None)
@given(n=st.integers(min_value=1, max_value=400), seed=st.integers(0, 2**31 - 1),
       sign=st.sampled_from([-1, 1]))
def test_direct_dft_any_length_against_definition(oracle_lib, n, seed, sign):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)
    assert pins.rel_l2(oracle.dft(x, sign), pins.brute_dft(x, sign)) < 1e-14
