/*
 * efft_oracle.c -- plain, slow, obviously-correct CPU reference for the
 * one-dimensional complex DFT.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only tests/, __graft_entry__.smoke() and the cpu_baseline
 * leg of bench.py use it.  It shares no code, header, table or constant with
 * the HIP library.
 *
 * What it computes (paper, Section 1, Eq. "eqf"):
 *
 *     F_k = sum_{n=0}^{N-1} x_n * exp(sign * 2*pi*i * k*n / N),
 *
 * sign = -1 for the forward transform exactly as the paper writes it, and
 * sign = +1 for the backward (conjugate-sign) transform, which the paper does
 * not define; both are unnormalised.
 *
 * Two routes, both in FP64 arithmetic on interleaved (re, im) doubles:
 *
 *  oracle_fft       -- the radix-2 Cooley-Tukey recursion of Section 2.2
 *                      (Eqs. "eqb", "eqct", "eqctt") unrolled the textbook way:
 *                      reorder the input by bit reversal (the bin map of
 *                      Section 3.2), then log2(N) levels of butterflies
 *                      F_k = E_k + W^k O_k,  F_{k+M/2} = E_k - W^k O_k.
 *                      Every twiddle W^k = exp(sign*2*pi*i*k/M) is evaluated
 *                      directly (long double cosl/sinl of an exact ratio,
 *                      rounded once), never by recurrence.
 *
 *  oracle_dft_bins  -- Eq. "eqf" itself, evaluated at chosen bins k by a
 *                      direct sum over n, with the phase index (k*n) mod N
 *                      reduced exactly in integers and Kahan-compensated
 *                      accumulation, for any length N (power of two or not;
 *                      at all N bins it is the full O(N^2) definition).
 *                      Input may be streamed in chunks, so sizes whose full
 *                      array does not fit in host memory can still be
 *                      sampled.
 *
 * Compile-time ORACLE_MUTANT=k (k > 0) plants one deliberate mistake; the
 * CPU test-suite builds those variants to show that its pins catch each one.
 * The default build (ORACLE_MUTANT undefined or 0) has no mutation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

static const long double PI_L = 3.14159265358979323846264338327950288L;

/* exp(sign * 2*pi*i * num/den) rounded to double, for any den >= 1.
 * The turn num/den is split exactly into a whole number of quarter turns and
 * a remainder below a quarter turn, and a remainder above an eighth is taken
 * from the complementary angle, so cosl/sinl only ever see [0, pi/4] and
 * every multiple of a quarter turn (1, i, -1, -i) comes out exact. */
static void unit_root(uint64_t num, uint64_t den, int sign, double *c, double *s)
{
#if ORACLE_MUTANT == 9 /* planted: the power-of-two shortcut for num mod den used for every den */
    const uint64_t u = num & (den - 1u);
#else
    const uint64_t u = num % den;                  /* num mod den */
#endif
    const uint64_t quads = (4u * u) / den;         /* whole quarter turns */
    const uint64_t rem = 4u * u - quads * den;     /* remainder, in den-ths of a quarter */
    long double cr, sr;
    if (rem == 0) {
        cr = 1.0L;
        sr = 0.0L;
    } else if (2u * rem <= den) {
        long double a = (PI_L / 2.0L) * ((long double)rem / (long double)den);
        cr = cosl(a);
        sr = sinl(a);
    } else {
        long double a = (PI_L / 2.0L) * ((long double)(den - rem) / (long double)den);
        cr = sinl(a);
        sr = cosl(a);
    }
    /* rotate by quads quarter turns: multiply by i^quads */
    long double rr = cr, ri = sr;
    switch (quads & 3u) {
    case 0: rr = cr; ri = sr; break;
    case 1: rr = -sr; ri = cr; break;
    case 2: rr = -cr; ri = -sr; break;
    default: rr = sr; ri = -cr; break;
    }
    *c = (double)rr;
    *s = (double)((long double)sign * ri);
}

static int log2_exact(int64_t n)
{
    int q = 0;
    if (n <= 0 || (n & (n - 1)) != 0) return -1;
    while (((int64_t)1 << q) < n) ++q;
    return q;
}

static uint64_t bit_reverse(uint64_t v, int bits)
{
    uint64_t r = 0;
    for (int b = 0; b < bits; ++b) {
        r = (r << 1) | (v & 1u);
        v >>= 1;
    }
    return r;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * In-place radix-2 FFT of x[2*n] (interleaved re, im), n a power of two.
 * Returns 0 on success, -1 for a size that is not a power of two, -2 when
 * the twiddle table cannot be allocated.
 */
int oracle_fft(double *x, int64_t n, int sign)
{
    const int q = log2_exact(n);
    if (q < 0) return -1;
    if (n == 1) return 0;

    /* W_N^j for j < N/2; a level of length M uses W_M^k = W_N^{k*N/M}. */
    const int64_t half_n = n / 2;
    double *w = (double *)malloc(sizeof(double) * 2 * (size_t)half_n);
    if (!w) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < half_n; ++j) {
        unit_root((uint64_t)j, (uint64_t)n, sign, &w[2 * j], &w[2 * j + 1]);
#if ORACLE_MUTANT == 1 /* planted: twiddle of the wrong sign */
        w[2 * j + 1] = -w[2 * j + 1];
#endif
    }

    /* Bit-reversal reordering: afterwards each aligned block of length M
     * holds, in order, the even-index and odd-index halves that the radix-2
     * split of Eq. "eqb" needs at every level. */
#if ORACLE_MUTANT != 2 /* planted: reordering left out */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
#if ORACLE_MUTANT == 8 /* planted: bit reversal over one bit too few */
        int64_t r = (int64_t)bit_reverse((uint64_t)i, q - 1) | (i & ((int64_t)1 << (q - 1)));
#else
        int64_t r = (int64_t)bit_reverse((uint64_t)i, q);
#endif
        if (i < r) {
            double t0 = x[2 * i], t1 = x[2 * i + 1];
            x[2 * i] = x[2 * r];
            x[2 * i + 1] = x[2 * r + 1];
            x[2 * r] = t0;
            x[2 * r + 1] = t1;
        }
    }
#endif

    /* Levels M = 2, 4, ..., N.  In each block of length M the first half is
     * E (DFT of the even samples) and the second half O (odd samples):
     *   F_k       = E_k + W_M^k O_k          (Eq. "eqct")
     *   F_{k+M/2} = E_k - W_M^k O_k          (Eq. "eqctt")   0 <= k < M/2. */
    for (int64_t m = 2; m <= n; m *= 2) {
        const int64_t h = m / 2;
        const int64_t tw_step = n / m;
#pragma omp parallel for schedule(static)
        for (int64_t b = 0; b < half_n; ++b) {
            const int64_t block = b / h;
            const int64_t k = b % h;
            const int64_t i0 = block * m + k;
            const int64_t i1 = i0 + h;
            int64_t widx = k * tw_step;
#if ORACLE_MUTANT == 3 /* planted: twiddle index off by a factor of two */
            widx = (2 * k * tw_step) % half_n;
#endif
            double wr = w[2 * widx], wi = w[2 * widx + 1];
#if ORACLE_MUTANT == 4 /* planted: twiddle dropped on the last level */
            if (m == n) { wr = 1.0; wi = 0.0; }
#endif
            const double er = x[2 * i0], ei = x[2 * i0 + 1];
            const double or_ = x[2 * i1], oi = x[2 * i1 + 1];
            const double tr = wr * or_ - wi * oi;
            const double ti = wr * oi + wi * or_;
#if ORACLE_MUTANT == 5 /* planted: butterfly outputs swapped */
            x[2 * i0] = er - tr;
            x[2 * i0 + 1] = ei - ti;
            x[2 * i1] = er + tr;
            x[2 * i1 + 1] = ei + ti;
#elif ORACLE_MUTANT == 6 /* planted: twiddle applied to the even operand instead of the odd */
            x[2 * i0] = (wr * er - wi * ei) + or_;
            x[2 * i0 + 1] = (wr * ei + wi * er) + oi;
            x[2 * i1] = (wr * er - wi * ei) - or_;
            x[2 * i1 + 1] = (wr * ei + wi * er) - oi;
#elif ORACLE_MUTANT == 7 /* planted: the k = 0 butterfly of every block skipped */
            if (k != 0) {
                x[2 * i0] = er + tr;
                x[2 * i0 + 1] = ei + ti;
                x[2 * i1] = er - tr;
                x[2 * i1 + 1] = ei - ti;
            }
#else
            x[2 * i0] = er + tr;
            x[2 * i0 + 1] = ei + ti;
            x[2 * i1] = er - tr;
            x[2 * i1 + 1] = ei - ti;
#endif
        }
    }
    free(w);
    return 0;
}

/* Same transform on complex64 input: every float is upcast exactly, the
 * transform runs in FP64, and the FP64 result is written to out[2*n]. */
int oracle_fft_from_f32(const float *in, double *out, int64_t n, int sign)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < 2 * n; ++i) out[i] = (double)in[i];
    return oracle_fft(out, n, sign);
}

/* Kahan-compensated accumulator for one complex bin. */
typedef struct {
    double sr, cr, si, ci;
} kahan_c;

static inline void kahan_add(double *s, double *c, double v)
{
    double y = v - *c;
    double t = *s + y;
    *c = (t - *s) - y;
    *s = t;
}

/*
 * Direct evaluation of Eq. "eqf" at nb chosen bins, over the input slice
 * x[offset .. offset+len) of a length-n transform.  The slice contributes
 *     sum_{j<len} x[j] * exp(sign*2*pi*i * ((k*(offset+j)) mod n) / n)
 * to acc[4*b .. 4*b+3] = (sum_re, comp_re, sum_im, comp_im) of bin bins[b]
 * (a Kahan pair per component), so a caller may stream the input in chunks
 * and call this once per chunk.  Any length n >= 1 is accepted.  The phase
 * index m = (k*j) mod n is exact integer arithmetic: for a power-of-two n the
 * wrapped 64-bit product keeps the low bits exactly; otherwise the product is
 * formed in 128 bits at the first index of a run and advanced by k (mod n)
 * from one index to the next.  The root of unity is the product of two
 * directly evaluated table entries exp(..hi*2^h/n) * exp(..lo/n), m =
 * hi*2^h + lo.  Input is FP64 (is_f32 == 0, x is double*) or complex64
 * (is_f32 != 0, x is float*, upcast exactly).  Returns 0, or -1 for a bad
 * size or slice.
 */
int oracle_dft_bins(const void *x, int is_f32, int64_t offset, int64_t len, int64_t n,
                    int sign, const int64_t *bins, int64_t nb, double *acc)
{
    if (n <= 0 || offset < 0 || len < 0 || offset + len > n) return -1;
    const int pow2 = (n & (n - 1)) == 0;
    int q = 0; /* bits of n - 1 */
    while (((int64_t)1 << q) < n) ++q;
    const int h = (q + 1) / 2;
    const int64_t n_lo = (int64_t)1 << h;
    const int64_t n_hi = (n + n_lo - 1) / n_lo; /* j with j * 2^h < n */
    const uint64_t mask = (uint64_t)n - 1u;
    double *t_lo = (double *)malloc(sizeof(double) * 2 * (size_t)n_lo);
    double *t_hi = (double *)malloc(sizeof(double) * 2 * (size_t)n_hi);
    if (!t_lo || !t_hi) {
        free(t_lo);
        free(t_hi);
        return -2;
    }
    for (int64_t j = 0; j < n_lo; ++j) unit_root((uint64_t)j, (uint64_t)n, sign, &t_lo[2 * j], &t_lo[2 * j + 1]);
    for (int64_t j = 0; j < n_hi; ++j)
        unit_root((uint64_t)j << h, (uint64_t)n, sign, &t_hi[2 * j], &t_hi[2 * j + 1]);

    const double *xd = (const double *)x;
    const float *xf = (const float *)x;
    for (int64_t b = 0; b < nb; ++b) {
        const uint64_t k = (uint64_t)(((bins[b] % n) + n) % n);
        int nth = oracle_threads();
        kahan_c *part = (kahan_c *)calloc((size_t)nth, sizeof(kahan_c));
#pragma omp parallel num_threads(nth)
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            kahan_c a = {0.0, 0.0, 0.0, 0.0};
            int64_t prev = -2;
            uint64_t m = 0;
#pragma omp for schedule(static)
            for (int64_t j = 0; j < len; ++j) {
                if (pow2) {
                    m = (k * (uint64_t)(offset + j)) & mask;
                } else if (j != prev + 1) {
#if ORACLE_MUTANT == 10 /* planted: the product wraps at 2^64 before the reduction mod n */
                    m = (k * (uint64_t)(offset + j)) % (uint64_t)n;
#else
                    m = (uint64_t)(((unsigned __int128)k * (unsigned __int128)(uint64_t)(offset + j)) % (uint64_t)n);
#endif
                } else {
                    m += k; /* (k*(j+1)) mod n from (k*j) mod n */
                    if (m >= (uint64_t)n) m -= (uint64_t)n;
                }
                prev = j;
                const uint64_t mh = m >> h, ml = m & (uint64_t)(n_lo - 1);
                const double hr = t_hi[2 * mh], hi = t_hi[2 * mh + 1];
                const double lr = t_lo[2 * ml], li = t_lo[2 * ml + 1];
                const double wr = hr * lr - hi * li;
                const double wi = hr * li + hi * lr;
                double xr, xi;
                if (is_f32) {
                    xr = (double)xf[2 * j];
                    xi = (double)xf[2 * j + 1];
                } else {
                    xr = xd[2 * j];
                    xi = xd[2 * j + 1];
                }
                kahan_add(&a.sr, &a.cr, xr * wr - xi * wi);
                kahan_add(&a.si, &a.ci, xr * wi + xi * wr);
            }
            part[tid] = a;
        }
        for (int t = 0; t < nth; ++t) {
            kahan_add(&acc[4 * b + 0], &acc[4 * b + 1], part[t].sr);
            kahan_add(&acc[4 * b + 0], &acc[4 * b + 1], -part[t].cr);
            kahan_add(&acc[4 * b + 2], &acc[4 * b + 3], part[t].si);
            kahan_add(&acc[4 * b + 2], &acc[4 * b + 3], -part[t].ci);
        }
        free(part);
    }
    free(t_lo);
    free(t_hi);
    return 0;
}
