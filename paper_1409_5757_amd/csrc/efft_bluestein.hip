// efft_bluestein.hip -- transforms of a length N that is not a power of two.
//
// Eq. "eqf" (paper, Section 1) for any N, through the chirp identity
//     n*k = (n^2 + k^2 - (k - n)^2) / 2
// (Bluestein's chirp-z form).  With a_m = exp(sign*pi*i * m^2 / N),
//     F_k = a_k * sum_n (x_n a_n) * conj(a_{k-n}),
// a linear convolution of u_n = x_n a_n (n < N) with v_m = conj(a_m)
// (|m| < N).  It is evaluated as a cyclic convolution of power-of-two length
// M >= 2N - 1, where it does not wrap: U = DFT_M(u zero-padded),
// V = DFT_M(v placed at m mod M), then DFT_M^{-1}(U V), through the library's
// own power-of-two passes.  The paper's EFFT admits N = M' * 2^s with the
// bin DFTs of size M' done by MKL (Section 2.2, Section 4); this path covers
// every N >= 3 instead.
//
// With out-of-place M-point transforms, the pre-multiply and the product with
// V are applied by the transposing first pass of each transform as it loads,
// and the post-multiply by the last pass of the backward transform as it
// stores (the same products as the kernels below, which serve the in-place
// transforms).
//
// The chirp is exact in its phase: m^2 mod 2N is reduced in 128-bit integer
// arithmetic, and a_m = exp(sign*pi*i * r/N), r = m^2 mod 2N, is evaluated in
// FP64 with sincospi.
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

__global__ void __launch_bounds__(BT) chirp_kernel(double2 *a, int64_t n, int sign)
{
    const int64_t stride = int64_t(gridDim.x) * BT;
    for (int64_t j = int64_t(blockIdx.x) * BT + threadIdx.x; j < n; j += stride) {
        const unsigned __int128 sq = (unsigned __int128)uint64_t(j) * uint64_t(j);
        const uint64_t r = uint64_t(sq % (unsigned __int128)(2 * uint64_t(n)));  // j^2 mod 2N
        double s, c;
        sincospi(double(r) / double(n), &s, &c);
        a[j] = double2{c, sign * s};
    }
}

// v_m = conj(a_m) / M at m and at M - m (0 < m < N), zero elsewhere
template <typename V>
__global__ void __launch_bounds__(BT) chirp_kernel_v(V *w, const double2 *a, int64_t n, int64_t m, double inv_m)
{
    using T = decltype(V{}.x);
    const int64_t stride = int64_t(gridDim.x) * BT;
    for (int64_t j = int64_t(blockIdx.x) * BT + threadIdx.x; j < m; j += stride) {
        const int64_t idx = j < n ? j : (j > m - n ? m - j : -1);
        V out{T(0), T(0)};
        if (idx >= 0) {
            const double2 c = a[idx];
            out = V{T(c.x * inv_m), T(-c.y * inv_m)};
        }
        w[j] = out;
    }
}

// w = (x a) zero-padded to M points (products in FP64, rounded once)
template <typename V>
__global__ void __launch_bounds__(BT) premul_kernel(const V *x, V *w, const double2 *a, int64_t n, int64_t m)
{
    using T = decltype(V{}.x);
    const int64_t stride = int64_t(gridDim.x) * BT;
    for (int64_t j = int64_t(blockIdx.x) * BT + threadIdx.x; j < m; j += stride) {
        V out{T(0), T(0)};
        if (j < n) {
            const V v = x[j];
            const double2 p = cmul(double2{double(v.x), double(v.y)}, a[j]);
            out = V{T(p.x), T(p.y)};
        }
        w[j] = out;
    }
}

// w *= v (pointwise, in the storage type)
template <typename V>
__global__ void __launch_bounds__(BT) pointwise_kernel(V *w, const V *v, int64_t m)
{
    const int64_t stride = int64_t(gridDim.x) * BT;
    for (int64_t j = int64_t(blockIdx.x) * BT + threadIdx.x; j < m; j += stride) w[j] = cmul(w[j], v[j]);
}

// out = scale * a * w for the first N points (FP64 products, rounded once)
template <typename V>
__global__ void __launch_bounds__(BT) postmul_kernel(const V *w, V *out, const double2 *a, int64_t n, double scale)
{
    using T = decltype(V{}.x);
    const int64_t stride = int64_t(gridDim.x) * BT;
    for (int64_t j = int64_t(blockIdx.x) * BT + threadIdx.x; j < n; j += stride) {
        const V v = load_nt(w + j);
        const double2 c = load_nt(a + j);
        const double2 p = cmul(double2{double(v.x), double(v.y)}, double2{c.x * scale, c.y * scale});
        store_nt(out + j, V{T(p.x), T(p.y)});
    }
}

}  // namespace

hipError_t launch_chirp(double2 *a, int64_t n, int sign, hipStream_t stream)
{
    hipLaunchKernelGGL(chirp_kernel, dim3(grid_for(n)), dim3(BT), 0, stream, a, n, sign);
    return hipGetLastError();
}

hipError_t launch_chirp_v(int dtype_bytes, void *w, const double2 *a, int64_t n, int64_t m, hipStream_t stream)
{
    const double inv_m = 1.0 / double(m);  // m is a power of two: exact
    if (dtype_bytes == 16)
        hipLaunchKernelGGL(chirp_kernel_v<double2>, dim3(grid_for(m)), dim3(BT), 0, stream,
                           static_cast<double2 *>(w), a, n, m, inv_m);
    else
        hipLaunchKernelGGL(chirp_kernel_v<float2>, dim3(grid_for(m)), dim3(BT), 0, stream,
                           static_cast<float2 *>(w), a, n, m, inv_m);
    return hipGetLastError();
}

hipError_t launch_premul(int dtype_bytes, const void *x, void *w, const double2 *a, int64_t n, int64_t m,
                         hipStream_t stream)
{
    if (dtype_bytes == 16)
        hipLaunchKernelGGL(premul_kernel<double2>, dim3(grid_for(m)), dim3(BT), 0, stream,
                           static_cast<const double2 *>(x), static_cast<double2 *>(w), a, n, m);
    else
        hipLaunchKernelGGL(premul_kernel<float2>, dim3(grid_for(m)), dim3(BT), 0, stream,
                           static_cast<const float2 *>(x), static_cast<float2 *>(w), a, n, m);
    return hipGetLastError();
}

hipError_t launch_pointwise(int dtype_bytes, void *w, const void *v, int64_t m, hipStream_t stream)
{
    if (dtype_bytes == 16)
        hipLaunchKernelGGL(pointwise_kernel<double2>, dim3(grid_for(m)), dim3(BT), 0, stream,
                           static_cast<double2 *>(w), static_cast<const double2 *>(v), m);
    else
        hipLaunchKernelGGL(pointwise_kernel<float2>, dim3(grid_for(m)), dim3(BT), 0, stream,
                           static_cast<float2 *>(w), static_cast<const float2 *>(v), m);
    return hipGetLastError();
}

hipError_t launch_postmul(int dtype_bytes, const void *w, void *out, const double2 *a, int64_t n, double scale,
                          hipStream_t stream)
{
    if (dtype_bytes == 16)
        hipLaunchKernelGGL(postmul_kernel<double2>, dim3(grid_for(n)), dim3(BT), 0, stream,
                           static_cast<const double2 *>(w), static_cast<double2 *>(out), a, n, scale);
    else
        hipLaunchKernelGGL(postmul_kernel<float2>, dim3(grid_for(n)), dim3(BT), 0, stream,
                           static_cast<const float2 *>(w), static_cast<float2 *>(out), a, n, scale);
    return hipGetLastError();
}

}  // namespace efft
