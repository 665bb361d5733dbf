"""Independent checks that pin the CPU oracle to facts fixed by the mathematics.

None of these routines is the oracle's algorithm: they are the plain O(N^2)
definition of Eq. "eqf" (paper, Section 1), closed-form spectra of special
signals, identities of the DFT, and values worked out by hand.  ``battery``
runs them all against an oracle library handle and returns the names of the
checks that failed; the tests require an empty list for the real oracle and a
non-empty one for every planted mutant.
"""
from __future__ import annotations

import math
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dft_small.txt")


def brute_dft(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Eq. "eqf" summed term by term, phase index (k*n) mod N reduced exactly."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    idx = np.arange(n, dtype=np.int64)
    m = np.outer(idx, idx) % n
    ang = (2.0 * math.pi / n) * m.astype(np.float64)
    w = np.cos(ang) + 1j * sign * np.sin(ang)
    return w @ x


def mp_dft(x, sign: int = -1, dps: int = 30):
    """Eq. "eqf" in mpmath at ``dps`` significant digits (the paper's arbitrary-
    precision reference of Section 5.3, with mpmath standing in for GMP)."""
    import mpmath
    with mpmath.workdps(dps):
        n = len(x)
        xs = [mpmath.mpc(float(v.real), float(v.imag)) for v in x]
        out = []
        for k in range(n):
            acc = mpmath.mpc(0)
            for j in range(n):
                acc += xs[j] * mpmath.expjpi(sign * mpmath.mpf(2 * ((k * j) % n)) / n)
            out.append(acc)
        return out


def rel_l2(a, b) -> float:
    """||a-b||_2 / ||b||_2 with squared moduli (paper, Section 5.3, Eq. "l2norm")."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def read_golden(path: str = GOLDEN):
    cases = []
    cur = None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "case":
                cur = {"name": tok[1], "n": int(tok[2]), "sign": int(tok[3])}
                cases.append(cur)
            elif tok[0] in ("x", "F"):
                vals = [complex(float(p.split(",")[0]), float(p.split(",")[1])) for p in tok[1:]]
                cur[tok[0]] = np.array(vals, dtype=np.complex128)
    return cases


def _rng(seed):
    return np.random.default_rng(seed)


def battery(lib) -> list[str]:
    """Run every pin against ``lib``; return the names of those that fail."""
    failed: list[str] = []

    def check(name, ok):
        if not ok:
            failed.append(name)

    def fft(x, sign=-1):
        return oracle.fft(x, sign, lib=lib)

    # 1. hand-worked values (exact for the integer cases up to N = 4)
    for c in read_golden():
        got = fft(c["x"], c["sign"])
        if c["n"] <= 4:
            check(f"golden:{c['name']}", np.array_equal(got, c["F"]))
        else:
            check(f"golden:{c['name']}", np.allclose(got, c["F"], rtol=0, atol=1e-13))

    # 2. brute-force definition, both signs, N = 2 .. 512
    for q in range(1, 10):
        n = 1 << q
        r = _rng(q)
        x = r.uniform(-1, 1, n) + 1j * r.uniform(-1, 1, n)
        for sign in (-1, 1):
            check(f"brute:q={q}:s={sign}", rel_l2(fft(x, sign), brute_dft(x, sign)) < 1e-14)

    # 3. arbitrary-precision definition at N = 16, 32
    for n in (16, 32):
        r = _rng(100 + n)
        x = r.uniform(-0.5, 0.5, n) + 1j * r.uniform(-0.5, 0.5, n)
        ref = np.array([complex(v) for v in mp_dft(x)], dtype=np.complex128)
        check(f"mpmath:n={n}", rel_l2(fft(x), ref) < 1e-15)

    n = 1 << 12
    r = _rng(7)
    x = r.standard_normal(n) + 1j * r.standard_normal(n)
    y = r.standard_normal(n) + 1j * r.standard_normal(n)
    fx = fft(x)

    # 4. Parseval: sum |F|^2 = N sum |x|^2
    check("parseval", abs(np.sum(np.abs(fx) ** 2) / (n * np.sum(np.abs(x) ** 2)) - 1) < 1e-13)
    # 5. linearity
    a, b = 0.75 - 0.25j, -1.5 + 2.0j
    check("linearity", rel_l2(fft(a * x + b * y), a * fx + b * fft(y)) < 1e-14)
    # 6. time shift by s multiplies bin k by exp(-2 pi i k s / N)
    s = 37
    k = np.arange(n)
    check("shift", rel_l2(fft(np.roll(x, s)), fx * np.exp(-2j * np.pi * ((k * s) % n) / n)) < 1e-13)
    # 7. modulation by exp(2 pi i f n / N) rotates the spectrum by f
    f = 101
    mod = np.exp(2j * np.pi * ((k * f) % n) / n)
    check("modulation", rel_l2(fft(x * mod), np.roll(fx, f)) < 1e-13)
    # 8. impulse at n0 -> exp(-2 pi i k n0 / N)
    n0 = 5
    imp = np.zeros(n, dtype=np.complex128)
    imp[n0] = 1
    check("impulse", np.max(np.abs(fft(imp) - np.exp(-2j * np.pi * ((k * n0) % n) / n))) < 1e-14)
    # 9. constant -> N delta_k
    cst = np.full(n, 1.0 + 0.0j)
    ref = np.zeros(n, dtype=np.complex128)
    ref[0] = n
    check("constant", np.max(np.abs(fft(cst) - ref)) < 1e-10)
    # 10. geometric r^n -> (1 - r^N) / (1 - r w^k), w = exp(-2 pi i / N)
    rr = 0.97 * np.exp(0.3j)
    g = rr ** np.arange(n)
    closed = (1 - rr ** n) / (1 - rr * np.exp(-2j * np.pi * k / n))
    check("geometric", rel_l2(fft(g), closed) < 1e-13)
    # 11. integer tones with phases: spectrum N e^{i phi} at each frequency
    freqs = np.array([3, 900, 2048, 4095])
    phases = np.array([0.1, 2.0, -1.0, 3.0])
    tone = sum(np.exp(1j * (2 * np.pi * ((k * fq) % n) / n + ph)) for fq, ph in zip(freqs, phases))
    ref = np.zeros(n, dtype=np.complex128)
    ref[freqs] = n * np.exp(1j * phases)
    check("tones", np.max(np.abs(fft(tone) - ref)) < 1e-9)
    # 12. Hermitian symmetry for real input: F_{(N-k) mod N} = conj(F_k),
    #     F_0 and F_{N/2} real (Section 2.2, Eq. "eqsym" read with the index fixed)
    xr = r.standard_normal(n).astype(np.complex128)
    fr = fft(xr)
    check("hermitian", np.max(np.abs(fr[(-k) % n] - np.conj(fr))) < 1e-11 and
          abs(fr[0].imag) < 1e-11 and abs(fr[n // 2].imag) < 1e-11)
    # 13. round trip: backward(forward(x)) / N = x
    check("roundtrip", rel_l2(fft(fx, +1) / n, x) < 1e-15)
    # 14. backward is the conjugate-sign transform: bwd(x) = conj(fwd(conj(x)))
    check("backward_conj", rel_l2(fft(x, +1), np.conj(fft(np.conj(x)))) < 1e-15)

    # Lengths that are not powers of two (the direct-sum route, oracle.dft)
    def dft(x, sign=-1):
        return oracle.dft(x, sign, lib=lib)

    # 15. brute-force definition, both signs
    for n in (3, 5, 6, 7, 12, 30, 100, 243, 1000):
        r = _rng(1000 + n)
        x = r.uniform(-1, 1, n) + 1j * r.uniform(-1, 1, n)
        for sign in (-1, 1):
            check(f"brute_any:n={n}:s={sign}", rel_l2(dft(x, sign), brute_dft(x, sign)) < 1e-14)
    # 16. arbitrary precision at N = 15
    r = _rng(15)
    x = r.uniform(-0.5, 0.5, 15) + 1j * r.uniform(-0.5, 0.5, 15)
    ref = np.array([complex(v) for v in mp_dft(x)], dtype=np.complex128)
    check("mpmath_any:n=15", rel_l2(dft(x), ref) < 1e-15)
    # 17. numpy's FFT (pocketfft, mixed radix and Bluestein) at a prime and a
    #     composite length
    for n in (9973, 3 * 5 * 7 * 11 * 4):
        r = _rng(n)
        x = r.standard_normal(n) + 1j * r.standard_normal(n)
        check(f"numpy_any:n={n}", rel_l2(dft(x), np.fft.fft(x)) < 1e-13)
    # 18. closed forms at N = 1500: impulse, and the geometric series
    n = 1500
    k = np.arange(n)
    imp = np.zeros(n, dtype=np.complex128)
    imp[7] = 1
    check("impulse_any", np.max(np.abs(dft(imp) - np.exp(-2j * np.pi * ((k * 7) % n) / n))) < 1e-14)
    g = rr ** np.arange(n)
    closed = (1 - rr ** n) / (1 - rr * np.exp(-2j * np.pi * k / n))
    check("geometric_any", rel_l2(dft(g), closed) < 1e-13)
    # 19. exact phase reduction far beyond 2^64 at a length that is not a power
    #     of two: a tone at frequency f sampled over a slice near the end sums
    #     to the slice length in the tone's bin
    n = 3 * (1 << 32) + 7
    f = (1 << 32) + 12345
    off = n - 3000
    ph = np.array([((f * j) % n) / n for j in range(off, off + 3000)])  # exact integers, then one division
    tone = np.exp(2j * np.pi * ph)
    val = oracle.bins_value(oracle.dft_bins(tone, [f], n=n, offset=off, lib=lib))[0]
    check("spot_any_phase", abs(val - 3000) < 1e-8)
    return failed
