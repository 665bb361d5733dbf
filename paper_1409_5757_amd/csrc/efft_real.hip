// efft_real.hip -- real-input transforms on top of the complex path.
//
// N real samples x_n are read as H = N/2 complex samples z_n = x_{2n} + i x_{2n+1}.
// With E = DFT_H(x_even) and O = DFT_H(x_odd), the H-point transform of z is
// Z_k = E_k + i O_k, and both E and O are Hermitian because their inputs are
// real, so
//     E_k = (Z_k + conj Z_{H-k}) / 2,   O_k = (Z_k - conj Z_{H-k}) / (2i),
// and the N-point spectrum follows from one radix-2 level (paper, Section 2.2,
// Eqs. "eqct"/"eqctt"):
//     F_k = E_k + W_N^k O_k,   0 <= k <= H  (F_H = E_0 - O_0).
// Bins k and H-k use the same two inputs, so one thread reads that pair and
// writes its two outputs in place -- the paper's in-place pair reassembly
// (Section 3.4, Fig. "diag:CTAssemblyPair").  The inverse (unnormalised
// backward, Hermitian input F_0..F_H) runs the same pairing in reverse:
//     Z'_k = (F_k + conj F_{H-k}) + i W_N^{-k} (F_k - conj F_{H-k}),
// after which the backward H-point transform of Z' is x_even + i x_odd, each
// scaled by N like every unnormalised backward transform.
#include <hip/hip_runtime.h>

#include "efft_internal.hpp"

namespace efft {

// Forward post-pass, in place on z[0 .. H] (z[H] is the extra output slot).
template <typename T>
__global__ void __launch_bounds__(256) r2c_post_kernel(typename vec2<T>::type *z, int64_t h, TwTable tt,
                                                       double scale, int apply_scale)
{
    using V = typename vec2<T>::type;
    const T half = T(0.5);
    const T f = apply_scale ? T(scale) : T(1);
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k <= h / 2; k += stride) {
        if (k == 0) {
            const V a = z[0];
            z[0] = V{(a.x + a.y) * f, T(0)};  // F_0 = E_0 + O_0
            z[h] = V{(a.x - a.y) * f, T(0)};  // F_H = E_0 - O_0
            continue;
        }
        const int64_t j = h - k;
        const V a = load_nt(z + k);
        const V b = load_nt(z + j);
        // E_k = (a + conj b)/2, O_k = (a - conj b)/(2i) = (-i/2)(a - conj b)
        const V e = V{half * (a.x + b.x), half * (a.y - b.y)};
        const V d = V{half * (a.x - b.x), half * (a.y + b.y)};  // (a - conj b)/2
        const V o = V{d.y, -d.x};                                // times -i
        const V wk = round_tw<V>(tw_lookup(tt, uint64_t(k)));
        const V fk = cadd(e, cmul(wk, o));
        store_nt(z + k, V{fk.x * f, fk.y * f});
        if (j != k) {
            // E_j = conj E_k, O_j = conj O_k (Hermitian), F_j = E_j + W_N^j O_j
            // with W_N^j = W_N^(N/2 - k) = -conj(W_N^k)
            const V wj = V{-wk.x, wk.y};
            const V fj = cadd(cconj(e), cmul(wj, cconj(o)));
            store_nt(z + j, V{fj.x * f, fj.y * f});
        }
    }
}

// Backward pre-pass: reads f[0 .. H] (Hermitian half spectrum), writes z[0 .. H).
template <typename T>
__global__ void __launch_bounds__(256) c2r_pre_kernel(const typename vec2<T>::type *f,
                                                      typename vec2<T>::type *z, int64_t h, TwTable tt)
{
    using V = typename vec2<T>::type;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k <= h / 2; k += stride) {
        const int64_t j = h - k;
        V a = load_nt(f + k);
        V b = load_nt(f + j);
        if (k == 0) {  // F_0 and F_{N/2} of a Hermitian spectrum are real
            a.y = T(0);
            b.y = T(0);
        }
        // s = a + conj b, d = a - conj b, Z'_k = s + i W^{-k} d
        const V s = V{a.x + b.x, a.y - b.y};
        const V d = V{a.x - b.x, a.y + b.y};
        const V wk = cconj(round_tw<V>(tw_lookup(tt, uint64_t(k))));
        const V t = cmul(wk, d);
        store_nt(z + k, V{s.x - t.y, s.y + t.x});
        if (k != 0 && j != k) {
            const V s2 = cconj(s);        // b + conj a
            const V d2 = V{-d.x, d.y};    // b - conj a = -conj(d)
            const V wj = V{-wk.x, wk.y};  // conj(W_N^(N/2 - k)) = -W_N^k, and wk = conj(W_N^k)
            const V t2 = cmul(wj, d2);
            store_nt(z + j, V{s2.x - t2.y, s2.y + t2.x});
        }
    }
}

// pairs per launch grid: one thread per pair up to 2^28 threads, then each
// thread loops (the grid stays far below the 2^32 work-item limit)
static unsigned pair_grid(int64_t h)
{
    const int64_t threads = h / 2 + 1;
    const int64_t blocks = (threads + 255) / 256;
    return unsigned(blocks < (int64_t(1) << 20) ? blocks : (int64_t(1) << 20));
}

hipError_t launch_r2c_post(int dtype_bytes, void *z, int64_t h, const TwTable &tt, double scale,
                           int apply_scale, hipStream_t stream)
{
    const unsigned grid = pair_grid(h);
    if (dtype_bytes == 16)
        hipLaunchKernelGGL(r2c_post_kernel<double>, dim3(grid), dim3(256), 0, stream,
                           static_cast<double2 *>(z), h, tt, scale, apply_scale);
    else
        hipLaunchKernelGGL(r2c_post_kernel<float>, dim3(grid), dim3(256), 0, stream,
                           static_cast<float2 *>(z), h, tt, scale, apply_scale);
    return hipGetLastError();
}

hipError_t launch_c2r_pre(int dtype_bytes, const void *f, void *z, int64_t h, const TwTable &tt,
                          hipStream_t stream)
{
    const unsigned grid = pair_grid(h);
    if (dtype_bytes == 16)
        hipLaunchKernelGGL(c2r_pre_kernel<double>, dim3(grid), dim3(256), 0, stream,
                           static_cast<const double2 *>(f), static_cast<double2 *>(z), h, tt);
    else
        hipLaunchKernelGGL(c2r_pre_kernel<float>, dim3(grid), dim3(256), 0, stream,
                           static_cast<const float2 *>(f), static_cast<float2 *>(z), h, tt);
    return hipGetLastError();
}

}  // namespace efft
