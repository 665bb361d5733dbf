// efft_device.hpp -- register-level building blocks of the gfx950 FFT passes.
//
// Complex values are HIP vector types (double2 / float2, interleaved re, im).
// Every small DFT here is the forward transform of Eq. "eqf" (paper,
// Section 1) on R values held in registers, with natural-order output; the
// backward transform is obtained by conjugating on load and store, since
// DFT_+(x) = conj(DFT_-(conj(x))).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace efft {

template <typename T> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float> { using type = float2; };

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
// Complex product with its fused multiply-adds spelled out, so every kernel
// variant rounds each product identically (the compiler may not re-contract
// it differently from one instantiation to the next).
template <typename V> __device__ __forceinline__ V cmul(V a, V b)
{
    return V{fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return V{a.x, -a.y}; }
// multiply by -i = exp(-i*pi/2), the forward quarter-turn root
template <typename V> __device__ __forceinline__ V mul_mi(V a) { return V{a.y, -a.x}; }

// exp(-2*pi*i*e/16) for the constant exponents a 16-point DFT needs
template <int E, typename V> __device__ __forceinline__ V tw16(V a)
{
    using T = decltype(a.x);
    constexpr double C1 = 0.92387953251128675613;  // cos(pi/8)
    constexpr double S1 = 0.38268343236508977173;  // sin(pi/8)
    constexpr double H = 0.70710678118654752440;   // cos(pi/4)
    if constexpr (E == 0) {
        return a;
    } else if constexpr (E == 1) {  // (C1, -S1)
        return cmul(a, V{T(C1), T(-S1)});
    } else if constexpr (E == 2) {  // (H, -H)
        return V{T(H) * (a.x + a.y), T(H) * (a.y - a.x)};
    } else if constexpr (E == 3) {  // (S1, -C1)
        return cmul(a, V{T(S1), T(-C1)});
    } else if constexpr (E == 4) {  // -i
        return mul_mi(a);
    } else if constexpr (E == 6) {  // (-H, -H)
        return V{T(H) * (a.y - a.x), T(-H) * (a.x + a.y)};
    } else if constexpr (E == 9) {  // (-C1, S1)
        return cmul(a, V{T(-C1), T(S1)});
    } else {
        static_assert(E == 0, "unsupported 16-point twiddle");
        return a;
    }
}

template <typename V> __device__ __forceinline__ void dft2(V &a, V &b)
{
    V t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

template <typename V> __device__ __forceinline__ void dft4(V &a0, V &a1, V &a2, V &a3)
{
    V t0 = cadd(a0, a2), t1 = csub(a0, a2);
    V t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// 8 = 2 x 4: n = n1 + 2*n2, k = k2 + 4*k1
template <typename V> __device__ __forceinline__ void dft8(V *v)
{
    V e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    V o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    o1 = tw16<2>(o1);
    o2 = tw16<4>(o2);
    o3 = tw16<6>(o3);
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// 16 = 4 x 4: n = n1 + 4*n2, k = k2 + 4*k1
template <typename V> __device__ __forceinline__ void dft16(V *v)
{
    V y[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
        V a0 = v[n1], a1 = v[n1 + 4], a2 = v[n1 + 8], a3 = v[n1 + 12];
        dft4(a0, a1, a2, a3);
        y[n1][0] = a0; y[n1][1] = a1; y[n1][2] = a2; y[n1][3] = a3;
    }
    y[1][1] = tw16<1>(y[1][1]); y[1][2] = tw16<2>(y[1][2]); y[1][3] = tw16<3>(y[1][3]);
    y[2][1] = tw16<2>(y[2][1]); y[2][2] = tw16<4>(y[2][2]); y[2][3] = tw16<6>(y[2][3]);
    y[3][1] = tw16<3>(y[3][1]); y[3][2] = tw16<6>(y[3][2]); y[3][3] = tw16<9>(y[3][3]);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        V a0 = y[0][k2], a1 = y[1][k2], a2 = y[2][k2], a3 = y[3][k2];
        dft4(a0, a1, a2, a3);
        v[k2] = a0; v[k2 + 4] = a1; v[k2 + 8] = a2; v[k2 + 12] = a3;
    }
}

template <int R, typename V> __device__ __forceinline__ void dft(V *v)
{
    if constexpr (R == 2) dft2(v[0], v[1]);
    else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8(v);
    else if constexpr (R == 16) dft16(v);
    else static_assert(R == 1, "unsupported radix");
}

// Loads and stores with the non-temporal hint: the data of a pass is touched
// once, so it is streamed past the caches instead of displacing what is
// reused there (twiddle tables, lines of tiles still in flight).
template <typename V> __device__ __forceinline__ V load_nt(const V *p)
{
    using T = decltype(V{}.x);
    typedef T native2 __attribute__((ext_vector_type(2)));
    const native2 r = __builtin_nontemporal_load(reinterpret_cast<const native2 *>(p));
    return V{r.x, r.y};
}

template <typename V> __device__ __forceinline__ void store_nt(V *p, V v)
{
    using T = decltype(V{}.x);
    typedef T native2 __attribute__((ext_vector_type(2)));
    const native2 r = {v.x, v.y};
    __builtin_nontemporal_store(r, reinterpret_cast<native2 *>(p));
}

// Wave-uniform addressing: a pointer that is the same in every lane, moved
// into scalar registers, plus a lane's 32-bit byte offset.  The loads and
// stores then take the scalar-base form (one offset register shared by all
// of a thread's accesses) instead of one 64-bit address register each.
template <typename T> using gptr = __attribute__((address_space(1))) T *;

template <typename V> __device__ __forceinline__ gptr<V> wave_uniform(const V *p)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(a));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(a >> 32));
    return reinterpret_cast<gptr<V>>((uint64_t(hi) << 32) | lo);
}

template <typename V> __device__ __forceinline__ gptr<V> at_offset(gptr<V> base, uint32_t byte_off)
{
    return reinterpret_cast<gptr<V>>(reinterpret_cast<gptr<char>>(base) + byte_off);
}

template <typename V> __device__ __forceinline__ V load_g(gptr<V> p, int nt)
{
    using T = decltype(V{}.x);
    typedef T native2 __attribute__((ext_vector_type(2)));
    const gptr<const native2> q = reinterpret_cast<gptr<const native2>>(p);
    const native2 r = nt ? __builtin_nontemporal_load(q) : *q;
    return V{r.x, r.y};
}

template <typename V> __device__ __forceinline__ void store_g(gptr<V> p, V v, int nt)
{
    using T = decltype(V{}.x);
    typedef T native2 __attribute__((ext_vector_type(2)));
    const native2 r = {v.x, v.y};
    const gptr<native2> q = reinterpret_cast<gptr<native2>>(p);
    if (nt)
        __builtin_nontemporal_store(r, q);
    else
        *q = r;
}

// ---------------------------------------------------------------- twiddles
// FP64 table of W_N^m = exp(-2*pi*i*m/N) in three levels,
//   W_N^m = (hi[m >> h2] * mid[(m >> h) & mask_mid]) * lo[m & (2^h - 1)].
// For moderate N it is two levels in effect: h2 = h, mask_mid = 0 and mid[0]
// = 1 exactly, so the middle product changes no bit; for large N, h2 = 2h and
// mid[j] = W_N^(j 2^h), which keeps the tables a few hundred KiB (cached
// while the data streams past) where two levels would need MiBs.  One lookup
// path for both keeps the kernels free of a branch on the table shape.
struct TwTable {
    const double2 *lo;
    const double2 *hi;
    uint64_t mask_n;    // N - 1
    uint64_t mask_lo;   // 2^h - 1
    int h;
    const double2 *mid;
    uint64_t mask_mid;  // 2^h - 1, or 0 (mid[0] = 1)
    int h2;
    const float2 *line32;  // W_4096^e, e < 4096, rounded once to FP32 (complex64 in-line twiddles)
};

// entries of the FP32 line table (the longest line a pass transforms)
constexpr int LINE_TW_N = 4096;

__device__ __forceinline__ double2 tw_lookup(const TwTable &tt, uint64_t m)
{
    m &= tt.mask_n;
    const double2 a = tt.hi[m >> tt.h2];
    const double2 b = tt.mid[(m >> tt.h) & tt.mask_mid];
    const double2 c = tt.lo[m & tt.mask_lo];
    return cmul(cmul(a, b), c);
}

template <typename V> __device__ __forceinline__ V round_tw(double2 w)
{
    using T = decltype(V{}.x);
    return V{T(w.x), T(w.y)};
}

}  // namespace efft
