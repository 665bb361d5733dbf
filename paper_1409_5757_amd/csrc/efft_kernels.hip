// efft_kernels.hip -- the digit-reversal swap, the twiddle tables and the
// launchers of the gfx950 FFT passes.  The sub-FFT pass kernels themselves are
// in efft_stage.hpp (instantiated by efft_stage_*.hip).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "efft_internal.hpp"
#include "efft_stage.hpp"

namespace efft {

// ------------------------------------------------------------------- swap
// Workgroup (I, J, mu) exchanges tile A = rows I*TS.., cols J*TS.. of slab mu
// with tile B = rows J*TS.., cols I*TS.. of slab rev(mu), each transposed.
// The grid holds only the tile pairs with I <= J (the pair (J, I, rev(mu))
// is the same exchange); on the diagonal I == J the slabs mu and rev(mu) pair
// up and the workgroup with the smaller of the two takes them, and a tile
// paired with itself is transposed in place.  Every element is read and
// written exactly once.  (A grid over every (I, J) whose second workgroup of
// each pair returns at once launched about twice the workgroups, each
// holding the LDS of a CU while it starts and exits.)
//
// SPLIT: both tiles are loaded into registers and transposed through LDS one
// component at a time (real parts, then imaginary parts; each read overwrites
// only the component already written), so the LDS holds real numbers, half
// the bytes, and twice as many workgroups share a CU.
template <typename T, int TS, int NT, bool STREAM, bool SPLIT>
__global__ void __launch_bounds__(NT) swap_kernel(SwapParams p)
{
    using V = typename vec2<T>::type;
    constexpr int ROWS_PER_PASS = NT / TS;
    using E = typename std::conditional<SPLIT, T, V>::type;
    __shared__ E ta[TS][TS + 1];
    __shared__ E tb[TS][TS + 1];

    // grid: x = middle index mu (up to 2^24), y = tile pair I <= J numbered
    // row by row (nt * (nt + 1) / 2 of them; row I holds J = I .. nt - 1)
    const int64_t mu = order_tiles(blockIdx.x, p.M, TILE_XCD);
    int64_t I = 0, rem = blockIdx.y;
    while (rem >= p.nt - I) {
        rem -= p.nt - I;
        ++I;
    }
    const int64_t J = I + rem;
    const int64_t rmu = int64_t(digit_reverse(uint64_t(mu), p.mid));
    if (I == J && mu > rmu) return;  // taken by the workgroup of slab rmu
    const bool self = I == J && mu == rmu;

    V *x = static_cast<V *>(p.data) + int64_t(blockIdx.z) * p.n;  // signal of a batch
    const int col = threadIdx.x % TS;
    const int r0 = threadIdx.x / TS;
    // element (row a, col b) of tile A: x[((I*TS + a)*M + mu)*R + J*TS + b]
    const int64_t rowA = p.M * p.R;  // stride between consecutive outer rows
    const int64_t baseA = (I * TS * p.M + mu) * p.R + J * TS;
    const int64_t baseB = (J * TS * p.M + rmu) * p.R + I * TS;
    auto ld = [&](int64_t i) {
        if constexpr (STREAM) return load_nt(x + i);
        else return x[i];
    };
    auto st = [&](int64_t i, V v) {
        if constexpr (STREAM) store_nt(x + i, v);
        else x[i] = v;
    };
    if constexpr (SPLIT) {
        constexpr int K = TS / ROWS_PER_PASS;
        V ra[K], rb[K];
#pragma unroll
        for (int k = 0; k < K; ++k) ra[k] = ld(baseA + (r0 + k * ROWS_PER_PASS) * rowA + col);
        if (!self) {
#pragma unroll
            for (int k = 0; k < K; ++k) rb[k] = ld(baseB + (r0 + k * ROWS_PER_PASS) * rowA + col);
        }
#pragma unroll
        for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                ta[r0 + k * ROWS_PER_PASS][col] = comp ? ra[k].y : ra[k].x;
                if (!self) tb[r0 + k * ROWS_PER_PASS][col] = comp ? rb[k].y : rb[k].x;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const T xa = ta[col][r0 + k * ROWS_PER_PASS];
                if (comp)
                    ra[k].y = xa;
                else
                    ra[k].x = xa;
                if (!self) {
                    const T xb = tb[col][r0 + k * ROWS_PER_PASS];
                    if (comp)
                        rb[k].y = xb;
                    else
                        rb[k].x = xb;
                }
            }
            __syncthreads();
        }
        // ra[k] is element (col, a) of tile A: row a of B's place, and rb[k]
        // row a of A's place (a = r0 + k * ROWS_PER_PASS)
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t a = r0 + k * ROWS_PER_PASS;
            if (self) {
                st(baseA + a * rowA + col, ra[k]);
            } else {
                st(baseB + a * rowA + col, ra[k]);
                st(baseA + a * rowA + col, rb[k]);
            }
        }
        return;
    } else {
#pragma unroll
    for (int a = r0; a < TS; a += ROWS_PER_PASS) ta[a][col] = ld(baseA + a * rowA + col);
    if (!self) {
#pragma unroll
        for (int a = r0; a < TS; a += ROWS_PER_PASS) tb[a][col] = ld(baseB + a * rowA + col);
    }
    __syncthreads();
    if (self) {
#pragma unroll
        for (int a = r0; a < TS; a += ROWS_PER_PASS) st(baseA + a * rowA + col, ta[col][a]);
    } else {
#pragma unroll
        for (int a = r0; a < TS; a += ROWS_PER_PASS) {
            st(baseB + a * rowA + col, ta[col][a]);
            st(baseA + a * rowA + col, tb[col][a]);
        }
    }
    }
}

// ----------------------------------------------------------------- tables
// lo[j] = W_N^j (j < 2^h), hi[j] = W_N^(j*2^h), W_N^m = exp(-2*pi*i*m/N)
// evaluated in FP64 from the exact ratio 2m/N with sincospi.
__global__ void twiddle_table_kernel(double2 *lo, int64_t n_lo, double2 *hi, int64_t n_hi, int h,
                                     int q)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const double inv = ldexp(1.0, 1 - q);  // 2/N, exact
    if (i < n_lo) {
        double s, c;
        sincospi(double(i) * inv, &s, &c);
        lo[i] = double2{c, -s};
    }
    if (i < n_hi) {
        double s, c;
        sincospi(ldexp(double(i), h) * inv, &s, &c);
        hi[i] = double2{c, -s};
    }
}

// line32[e] = W_4096^e = exp(-2*pi*i*e/4096) from sincospi of the exact
// ratio 2e/4096 in FP64, rounded once to FP32 (the complex64 in-line twiddles)
__global__ void line32_table_kernel(float2 *t)
{
    const int e = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < LINE_TW_N) {
        double s, c;
        sincospi(double(e) * (2.0 / LINE_TW_N), &s, &c);
        t[e] = float2{float(c), float(-s)};
    }
}

// ---------------------------------------------------------------- launchers
// Set while a host-only caller checks that a kernel exists for every pass of
// a plan: the launchers then return success without launching anything.
thread_local bool g_dry_run = false;

hipError_t launch_stage_f64_lo(int layout, int logl, int lines, int sets, const StageParams &p, hipStream_t stream);
hipError_t launch_stage_f64_hi(int layout, int logl, int lines, int sets, const StageParams &p, hipStream_t stream);
hipError_t launch_stage_f32_lo(int layout, int logl, int lines, int sets, const StageParams &p, hipStream_t stream);
hipError_t launch_stage_f32_hi(int layout, int logl, int lines, int sets, const StageParams &p, hipStream_t stream);

// row layout: workgroups of about 256 threads, or one line when fewer exist
int row_lines(int dtype_bytes, int logl, int64_t nlines)
{
    (void)dtype_bytes;
    const int p = threads_per_line(logl);
    int want = p >= 256 ? 1 : 256 / p;
    return nlines >= want ? want : 1;
}

hipError_t launch_stage(int dtype_bytes, int layout, int logl, int lines, int sets,
                        const StageParams &p, hipStream_t stream)
{
    // strided layouts address a tile's lines as one block plus adjacent
    // offsets: the stride must be a power of two holding whole tiles
    if (layout != LAYOUT_ROW && layout != LAYOUT_ROW2COL &&
        (p.s <= 0 || (p.s & (p.s - 1)) != 0 || p.s % (int64_t(lines) * sets) != 0))
        return hipErrorInvalidValue;
    if (logl < 0 || logl > 12) return hipErrorInvalidValue;
    if (dtype_bytes == 16)
        return logl <= 8 ? launch_stage_f64_lo(layout, logl, lines, sets, p, stream)
                         : launch_stage_f64_hi(layout, logl, lines, sets, p, stream);
    if (dtype_bytes == 8)
        return logl <= 8 ? launch_stage_f32_lo(layout, logl, lines, sets, p, stream)
                         : launch_stage_f32_hi(layout, logl, lines, sets, p, stream);
    return hipErrorInvalidValue;
}

// The component-wise transpose of the swap, for complex64 with at least
// EFFT_SWAP_SPLIT8_MIN_M middle slabs.  Measured on gfx950 (in place, swap
// pass): 2^31 (M = 2^17) 9.24 -> 8.48 ms, 2^32 (2^16) 16.2 -> 15.1, 2^33
// (2^19) 37.4 -> 34.7, 2^34 (2^16) 59.3 -> 54.3; slower at 2^30, M = 2^10
// (3.56 -> 3.65) and 2^12 (3.06 -> 3.23); 2^28, M = 2^8, 0.95 -> 0.89.
// Complex128 (two workgroups per CU instead of one) lost at 2^30: 6.03 ->
// 7.20 ms.
#ifndef EFFT_SWAP_SPLIT8_MIN_M
#define EFFT_SWAP_SPLIT8_MIN_M (int64_t(1) << 13)
#endif

static hipError_t launch_swap_z(int dtype_bytes, const SwapParams &p, unsigned nz, hipStream_t stream)
{
    const int64_t ts = p.R / p.nt;
    const dim3 grid(unsigned(p.M), unsigned(p.nt * (p.nt + 1) / 2), nz);
#define EFFT_SWAP(T, TSV, NTV, SPL)                                                                 \
    if (ts == TSV) {                                                                                \
        if (g_dry_run) return hipSuccess;                                                           \
        if (p.nt_hint)                                                                              \
            hipLaunchKernelGGL((swap_kernel<T, TSV, NTV, true, SPL>), grid, dim3(NTV), 0, stream, p);  \
        else                                                                                        \
            hipLaunchKernelGGL((swap_kernel<T, TSV, NTV, false, SPL>), grid, dim3(NTV), 0, stream, p); \
        return hipGetLastError();                                                                   \
    }
    if (dtype_bytes == 16) {
        EFFT_SWAP(double, 64, 512, false)
        EFFT_SWAP(double, 32, 256, false)
        EFFT_SWAP(double, 16, 256, false)
    } else if (dtype_bytes == 8 && p.M >= EFFT_SWAP_SPLIT8_MIN_M) {
        EFFT_SWAP(float, 64, 512, true)
        EFFT_SWAP(float, 32, 256, true)
        EFFT_SWAP(float, 16, 256, true)
    } else if (dtype_bytes == 8) {
        EFFT_SWAP(float, 64, 512, false)
        EFFT_SWAP(float, 32, 256, false)
        EFFT_SWAP(float, 16, 256, false)
    }
#undef EFFT_SWAP
    return hipErrorInvalidValue;
}

hipError_t launch_swap(int dtype_bytes, const SwapParams &p, int64_t batch, hipStream_t stream)
{
    if (p.M > (int64_t(1) << 24) || p.nt < 1 || p.nt * (p.nt + 1) / 2 > 65535) return hipErrorInvalidValue;
    // signals of a batch along grid z, at most 65535 per launch
    for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
        SwapParams q = p;
        q.data = static_cast<char *>(p.data) + b0 * p.n * dtype_bytes;
        const hipError_t e = launch_swap_z(dtype_bytes, q, unsigned(batch - b0 < 65535 ? batch - b0 : 65535), stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void set_dry_run(bool on) { g_dry_run = on; }

hipError_t launch_line32_table(float2 *t, hipStream_t stream)
{
    hipLaunchKernelGGL(line32_table_kernel, dim3((LINE_TW_N + 255) / 256), dim3(256), 0, stream, t);
    return hipGetLastError();
}

hipError_t launch_twiddle_table(double2 *lo, int64_t n_lo, double2 *hi, int64_t n_hi, int h, int q,
                                hipStream_t stream)
{
    const int64_t n = n_lo > n_hi ? n_lo : n_hi;
    const unsigned grid = unsigned((n + 255) / 256);
    hipLaunchKernelGGL(twiddle_table_kernel, dim3(grid), dim3(256), 0, stream, lo, n_lo, hi, n_hi, h, q);
    return hipGetLastError();
}

}  // namespace efft
