// efft_mixed.hip -- lengths N = M * 2^s with a small odd factor M (3 <= M <= 15).
//
// The radix split of Section 2.2 with one radix-M level first (decimation in
// frequency), n = n1 * 2^s + n2, k = k1 + M * k2:
//     F_{k1 + M k2} = sum_{n2} W_{2^s}^{n2 k2} [ W_N^{n2 k1} sum_{n1} x_{n1 2^s + n2} W_M^{n1 k1} ],
// the inner bracket being one M-point DFT per column n2 times the twiddle
// W_N^{n2 k1}.  That gives three steps:
//   radix-M pass  work[k1 * 2^s + n2] = W_N^{n2 k1} * DFT_M(x[. * 2^s + n2])[k1]
//   M batched 2^s-point transforms of the rows of work (the power-of-two passes)
//   reorder       out[k2 * M + k1] = scale * work[k1 * 2^s + k2]
// When the rows take two or more passes, the reorder is the last of them (a
// row-to-column pass that writes the rows interleaved); the reorder kernel
// here serves rows of a single pass.
// The paper's EFFT takes the same size class (Section 2.2, Section 4), with
// the M-point transforms left to MKL; here they are direct sums in FP64.
//
// Twiddles: W_M^j (j < M) and a two-level table of W_N^m (m < N): lo[j] =
// W_N^j, hi[j] = W_N^{j 2^h}, W_N^m = hi[m >> h] * lo[m mod 2^h], every entry
// from sincospi(2m/N) in FP64 (2m/N rounded once, N not a power of two).
#include <hip/hip_runtime.h>

#include "efft_internal.hpp"

namespace efft {

namespace {

constexpr int BT = 256;

unsigned grid_for(int64_t items)
{
    const int64_t blocks = (items + BT - 1) / BT;
    return unsigned(blocks < (int64_t(1) << 20) ? blocks : (int64_t(1) << 20));
}

__global__ void __launch_bounds__(BT) table_kernel(double2 *wm, int m, double2 *lo, int64_t n_lo, double2 *hi,
                                                   int64_t n_hi, int h, int64_t n)
{
    const int64_t i = int64_t(blockIdx.x) * BT + threadIdx.x;
    double s, c;
    if (i < m) {
        sincospi(2.0 * double(i) / double(m), &s, &c);
        wm[i] = double2{c, -s};
    }
    if (i < n_lo) {
        sincospi(2.0 * double(i) / double(n), &s, &c);
        lo[i] = double2{c, -s};
    }
    if (i < n_hi) {
        sincospi(2.0 * double(i << h) / double(n), &s, &c);
        hi[i] = double2{c, -s};
    }
}

struct MixedParams {
    const void *src;
    void *dst;
    const double2 *wm, *lo, *hi;
    int64_t cols;   // 2^s
    int64_t n;      // M * 2^s
    int64_t count;  // batch * 2^s columns
    int h;
    int conj;       // backward direction
};

// One column n2 of one signal per thread: M loads at stride 2^s (adjacent
// threads read adjacent addresses), the M-point DFT in FP64, the twiddle
// W_N^{n2 k1}, M stores at stride 2^s; data loads and stores stream past the
// caches (non-temporal), which keep the twiddle tables.
template <typename V, int M>
__global__ void __launch_bounds__(BT) radix_m_kernel(MixedParams p)
{
    using T = decltype(V{}.x);
    const V *x = static_cast<const V *>(p.src);
    V *w = static_cast<V *>(p.dst);
    const int64_t stride = int64_t(gridDim.x) * BT;
    const double sg = p.conj ? -1.0 : 1.0;  // conjugate the forward roots for the backward direction
    double2 wm[M];
#pragma unroll
    for (int j = 0; j < M; ++j) wm[j] = double2{p.wm[j].x, sg * p.wm[j].y};
    const uint64_t mask_lo = (uint64_t(1) << p.h) - 1u;
    for (int64_t g = int64_t(blockIdx.x) * BT + threadIdx.x; g < p.count; g += stride) {
        const int64_t b = g / p.cols;
        const int64_t n2 = g - b * p.cols;
        const int64_t base = b * p.n + n2;
        double2 xv[M];
#pragma unroll
        for (int n1 = 0; n1 < M; ++n1) {
            const V v = load_nt(x + base + n1 * p.cols);
            xv[n1] = double2{double(v.x), double(v.y)};
        }
#pragma unroll
        for (int k1 = 0; k1 < M; ++k1) {
            double2 acc = xv[0];
#pragma unroll
            for (int n1 = 1; n1 < M; ++n1) {
                const double2 t = cmul(xv[n1], wm[(n1 * k1) % M]);
                acc = double2{acc.x + t.x, acc.y + t.y};
            }
            // W_N^{n2 k1}, n2 k1 < N
            const uint64_t mtw = uint64_t(n2) * uint64_t(k1);
            const double2 hv = p.hi[mtw >> p.h], lv = p.lo[mtw & mask_lo];
            double2 tw = cmul(hv, lv);
            tw.y *= sg;
            const double2 r = cmul(acc, tw);
            store_nt(w + base + k1 * p.cols, V{T(r.x), T(r.y)});
        }
    }
}

// out[b N + k2 M + k1] = scale * w[b N + k1 2^s + k2]: a workgroup takes 64
// consecutive k2 of one signal, reads its M rows of 64 (contiguous runs) into
// LDS and writes the 64 M outputs as one contiguous run.
constexpr int RK = 64;

template <typename V, int M>
__global__ void __launch_bounds__(BT) reorder_kernel(const V *w, V *out, int64_t cols, int64_t n, int64_t chunks,
                                                     double scale)
{
    using T = decltype(V{}.x);
    __shared__ V tile[M][RK + 1];
    for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        const int64_t per = (cols + RK - 1) / RK;  // chunks per signal
        const int64_t b = c / per;
        const int64_t k2_0 = (c - b * per) * RK;
        const int kn = int(cols - k2_0 < RK ? cols - k2_0 : RK);
        const V *src = w + b * n;
        for (int i = threadIdx.x; i < M * RK; i += BT) {
            const int k1 = i / RK, j = i - k1 * RK;
            if (j < kn) tile[k1][j] = src[int64_t(k1) * cols + k2_0 + j];
        }
        __syncthreads();
        V *dst = out + b * n + k2_0 * M;
        for (int o = threadIdx.x; o < kn * M; o += BT) {
            const int j = o / M, k1 = o - j * M;
            const V v = tile[k1][j];
            dst[o] = V{T(double(v.x) * scale), T(double(v.y) * scale)};
        }
        __syncthreads();  // the tile is rewritten by the next chunk
    }
}

template <typename V, int M>
hipError_t launch_m(const MixedParams &p, bool radix, const void *w, void *out, int64_t chunks, double scale,
                    hipStream_t stream)
{
    if (radix)
        hipLaunchKernelGGL((radix_m_kernel<V, M>), dim3(grid_for(p.count)), dim3(BT), 0, stream, p);
    else
        hipLaunchKernelGGL((reorder_kernel<V, M>),
                           dim3(unsigned(chunks < (int64_t(1) << 20) ? chunks : (int64_t(1) << 20))), dim3(BT),
                           0, stream, static_cast<const V *>(w), static_cast<V *>(out), p.cols, p.n, chunks, scale);
    return hipGetLastError();
}

template <typename V>
hipError_t dispatch_m(int m, const MixedParams &p, bool radix, const void *w, void *out, int64_t chunks,
                      double scale, hipStream_t stream)
{
    switch (m) {
    case 3: return launch_m<V, 3>(p, radix, w, out, chunks, scale, stream);
    case 5: return launch_m<V, 5>(p, radix, w, out, chunks, scale, stream);
    case 7: return launch_m<V, 7>(p, radix, w, out, chunks, scale, stream);
    case 9: return launch_m<V, 9>(p, radix, w, out, chunks, scale, stream);
    case 11: return launch_m<V, 11>(p, radix, w, out, chunks, scale, stream);
    case 13: return launch_m<V, 13>(p, radix, w, out, chunks, scale, stream);
    case 15: return launch_m<V, 15>(p, radix, w, out, chunks, scale, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_mixed_tables(double2 *wm, int m, double2 *lo, int64_t n_lo, double2 *hi, int64_t n_hi, int h,
                               int64_t n, hipStream_t stream)
{
    int64_t items = n_lo > n_hi ? n_lo : n_hi;
    if (m > items) items = m;
    hipLaunchKernelGGL(table_kernel, dim3(unsigned((items + BT - 1) / BT)), dim3(BT), 0, stream, wm, m, lo, n_lo,
                       hi, n_hi, h, n);
    return hipGetLastError();
}

hipError_t launch_radix_m(int dtype_bytes, int m, const void *x, void *w, const double2 *wm, const double2 *lo,
                          const double2 *hi, int h, int64_t cols, int64_t batch, int conj, hipStream_t stream)
{
    MixedParams p{x, w, wm, lo, hi, cols, cols * m, batch * cols, h, conj};
    if (dtype_bytes == 16) return dispatch_m<double2>(m, p, true, nullptr, nullptr, 0, 1.0, stream);
    return dispatch_m<float2>(m, p, true, nullptr, nullptr, 0, 1.0, stream);
}

hipError_t launch_reorder_m(int dtype_bytes, int m, const void *w, void *out, int64_t cols, int64_t batch,
                            double scale, hipStream_t stream)
{
    MixedParams p{nullptr, nullptr, nullptr, nullptr, nullptr, cols, cols * m, 0, 0, 0};
    const int64_t chunks = batch * ((cols + RK - 1) / RK);
    if (dtype_bytes == 16) return dispatch_m<double2>(m, p, false, w, out, chunks, scale, stream);
    return dispatch_m<float2>(m, p, false, w, out, chunks, scale, stream);
}

}  // namespace efft
