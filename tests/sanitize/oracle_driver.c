/* Exercises every entry point of the CPU oracle (oracle/efft_oracle.c) under
 * AddressSanitizer and UndefinedBehaviorSanitizer: every power-of-two size up
 * to 2^16 in both directions, the single-precision entry, the direct sum at
 * lengths that are and are not powers of two with chunked input, bins outside
 * [0, N), and the rejected sizes and slices.  Exits 0 when every call returned
 * what its contract says and every value is finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_fft(double *x, int64_t n, int sign);
int oracle_fft_from_f32(const float *in, double *out, int64_t n, int sign);
int oracle_dft_bins(const void *x, int is_f32, int64_t offset, int64_t len, int64_t n, int sign,
                    const int64_t *bins, int64_t nb, double *acc);

static int fail(const char *what, long long a)
{
    fprintf(stderr, "FAIL %s (%lld)\n", what, a);
    return 1;
}

static int finite_all(const double *v, int64_t m)
{
    for (int64_t i = 0; i < m; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

int main(void)
{
    for (int q = 0; q <= 16; ++q) {
        const int64_t n = (int64_t)1 << q;
        double *x = malloc(sizeof(double) * 2 * (size_t)n);
        float *xf = malloc(sizeof(float) * 2 * (size_t)n);
        double *y = malloc(sizeof(double) * 2 * (size_t)n);
        if (!x || !xf || !y) return fail("malloc", q);
        for (int sign = -1; sign <= 1; sign += 2) {
            for (int64_t i = 0; i < 2 * n; ++i) {
                x[i] = (double)((i * 7919) % 2003) / 1001.0 - 1.0;
                xf[i] = (float)x[i];
            }
            if (oracle_fft(x, n, sign) != 0) return fail("oracle_fft", q);
            if (!finite_all(x, 2 * n)) return fail("oracle_fft finite", q);
            if (oracle_fft_from_f32(xf, y, n, sign) != 0) return fail("oracle_fft_from_f32", q);
            if (!finite_all(y, 2 * n)) return fail("oracle_fft_from_f32 finite", q);
        }
        free(x);
        free(xf);
        free(y);
    }
    {
        double x[2 * 12];
        for (int i = 0; i < 24; ++i) x[i] = 1.0;
        const int64_t bad[] = {0, 3, 12, -4};
        for (int i = 0; i < 4; ++i)
            if (oracle_fft(x, bad[i], -1) == 0) return fail("oracle_fft accepted size", bad[i]);
    }
    const int64_t lens[] = {1, 2, 3, 7, 12, 97, 1024, 4620, 65539};
    for (size_t li = 0; li < sizeof(lens) / sizeof(lens[0]); ++li) {
        const int64_t n = lens[li];
        double *x = malloc(sizeof(double) * 2 * (size_t)n);
        float *xf = malloc(sizeof(float) * 2 * (size_t)n);
        if (!x || !xf) return fail("malloc", n);
        for (int64_t i = 0; i < 2 * n; ++i) {
            x[i] = (double)((i * 104729) % 4099) / 2049.0 - 1.0;
            xf[i] = (float)x[i];
        }
        const int64_t bins[] = {0, 1, n - 1, n / 2, -1, n, 3 * n + 2, -5 * n - 1};
        const int64_t nb = sizeof(bins) / sizeof(bins[0]);
        for (int f32 = 0; f32 <= 1; ++f32) {
            for (int sign = -1; sign <= 1; sign += 2) {
                double acc[4 * 8] = {0};
                /* in three chunks (the last may be empty) */
                const int64_t c1 = n / 3, c2 = n - n / 3;
                const void *base = f32 ? (const void *)xf : (const void *)x;
                const size_t esz = f32 ? 2 * sizeof(float) : 2 * sizeof(double);
                if (oracle_dft_bins(base, f32, 0, c1, n, sign, bins, nb, acc) != 0 ||
                    oracle_dft_bins((const char *)base + esz * (size_t)c1, f32, c1, c2 - c1, n, sign, bins, nb, acc) != 0 ||
                    oracle_dft_bins((const char *)base + esz * (size_t)c2, f32, c2, n - c2, n, sign, bins, nb, acc) != 0)
                    return fail("oracle_dft_bins", n);
                if (!finite_all(acc, 4 * nb)) return fail("oracle_dft_bins finite", n);
            }
        }
        double acc[4] = {0};
        const int64_t b0 = 0;
        if (oracle_dft_bins(x, 0, 1, n, n, -1, &b0, 1, acc) == 0) return fail("slice past the end accepted", n);
        if (oracle_dft_bins(x, 0, -1, 1, n, -1, &b0, 1, acc) == 0) return fail("negative offset accepted", n);
        if (oracle_dft_bins(x, 0, 0, 1, 0, -1, &b0, 1, acc) == 0) return fail("n = 0 accepted", n);
        free(x);
        free(xf);
    }
    printf("oracle driver ok\n");
    return 0;
}
