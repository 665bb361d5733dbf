"""Seeded input generators: determinism, chunk independence, and that the
torch integer path reproduces the numpy path bit for bit (CPU)."""
import numpy as np
import torch

from paper_1409_5757_amd import inputs


def test_uniform_deterministic_and_chunk_independent():
    a = inputs.generate("uniform", 3, 10000)
    b = inputs.generate("uniform", 3, 10000, chunk=777)
    c = inputs.generate("uniform", 3, 500, offset=4321)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(c, a[4321:4821])
    assert a.real.min() >= -1 and a.real.max() < 1
    assert abs(a.real.mean()) < 0.03 and abs(a.imag.mean()) < 0.03


def test_seeds_and_families_are_independent():
    a = inputs.generate("uniform", 0, 4096)
    b = inputs.generate("uniform", 1, 4096)
    c = inputs.generate("normal", 0, 4096)
    assert abs(np.corrcoef(a.real, b.real)[0, 1]) < 0.1
    assert abs(np.corrcoef(a.real, c.real)[0, 1]) < 0.1


def test_normal_moments():
    x = inputs.generate("normal", 5, 1 << 18)
    for v in (x.real, x.imag):
        assert abs(v.mean()) < 0.01 and abs(v.std() - 1) < 0.01


def test_complex64_rounds_once_from_fp64():
    a = inputs.generate("uniform", 2, 1000)
    b = inputs.generate("uniform", 2, 1000, dtype=np.complex64)
    np.testing.assert_array_equal(b, a.astype(np.complex64))


def test_torch_integer_path_matches_numpy_bitwise():
    n = 1 << 15
    ref = inputs.generate("uniform", 7, n, offset=12345)
    for dt, npdt in ((torch.complex128, np.complex128), (torch.complex64, np.complex64)):
        t = torch.empty(n, dtype=dt)
        inputs.fill_uniform_torch(t, 7, offset=12345, chunk=4096)
        np.testing.assert_array_equal(t.numpy(), ref.astype(npdt))


def test_tones_spectrum_peaks_are_exact_closed_form():
    n = 1 << 12
    x = inputs.tones(4, n)
    f, v = inputs.tone_spectrum_peaks(4, n)
    assert len(set(f.tolist())) == 8
    spec = np.fft.fft(x)
    np.testing.assert_allclose(spec[f], v, atol=1e-9)
    mask = np.ones(n, bool)
    mask[f] = False
    assert np.abs(spec[mask]).max() < 1e-9
    fb, vb = inputs.tone_spectrum_peaks(4, n, sign=+1)
    np.testing.assert_allclose((np.fft.ifft(x) * n)[fb], vb, atol=1e-9)


def test_tones_chunked():
    n = 1 << 14
    a = inputs.tones(9, n)
    b = inputs.tones(9, n, offset=1000, length=3000, chunk=512)
    np.testing.assert_array_equal(a[1000:4000], b)


def test_weights_unit_interval():
    w = inputs.real_weights(1, 10000)
    assert w.dtype == np.float32 and w.min() >= 0 and w.max() <= 1
