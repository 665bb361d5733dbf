// efft_stage.hpp -- the sub-FFT pass kernels of the decomposed 1D FFT and their
// launch templates (instantiated by the efft_stage_*.hip sources, one range of
// line lengths and one element type each, so that they compile in parallel).
//
// The length-N transform is split N = R_1 * ... * R_m (Cooley-Tukey, the
// radix-2 split of Section 2.2 applied with larger radices); each pass runs
// batched sub-FFTs of one length L = R_j along one digit of the index.  A
// pass is one read and one write of the whole array.  Inside a workgroup a
// line of L points is transformed by the Stockham autosort variant of
// Cooley-Tukey: every thread holds E = 16 points of its line in registers,
// does radix-16 (and one smaller-radix) butterflies, and exchanges through
// LDS between steps, so the line comes out in natural order.  Thread t of a
// line always holds points t + P*i (P = L/16 threads per line, i < 16) both
// when loading and when storing, which makes global accesses coalesced in
// either layout: along the line for contiguous lines, across W adjacent lines
// (one 128-byte segment per row) for strided lines.
#pragma once
#include <hip/hip_runtime.h>

#include "efft_internal.hpp"


namespace efft {

// In-line twiddles of complex64 lines from an LDS table (1) or generated in
// FP64 per butterfly (0).
#ifndef EFFT_C64_LDS_TW
#define EFFT_C64_LDS_TW 1
#endif

// An opaque copy: the compiler must assume the value changed here, so it
// recomputes what depends on it instead of keeping an earlier result alive
// in registers (an empty asm statement; no instruction is emitted).
template <typename X> __device__ __forceinline__ void opaque(X &x) { asm volatile("" : "+v"(x)); }
// Whether a pass kernel holds the wave-uniform addressing form of its strided
// loads and stores: complex128 passes never take it (the host keeps off32
// clear for them) unless EFFT_WAVE_UNIFORM_C128 is set, and leaving the code
// out of their kernels saves its address arithmetic.
template <typename V> constexpr bool uniform_code()
{
    return sizeof(decltype(V{}.x)) == 4 || EFFT_WAVE_UNIFORM_C128;
}

// The recomputation barriers (opaque copies) below keep the complex64 tiles
// of two line sets within their registers; complex128 kernels have the room
// and run faster without them (measured on gfx950, 2^30 complex128 in place,
// first pass: 8.13 -> 7.88 ms).
#ifndef EFFT_OPAQUE_C128
#define EFFT_OPAQUE_C128 0
#endif

// opaque() where the element type asks for it
template <typename V, typename X> __device__ __forceinline__ void opaque_for(X &x)
{
    if constexpr (sizeof(decltype(V{}.x)) == 4 || EFFT_OPAQUE_C128) opaque(x);
}

// LDS index of point p of a line: one padding slot per 16 points breaks the
// power-of-two strides of the Stockham writes across banks
__device__ __forceinline__ int lds_pad(int p) { return p + (p >> 4); }

template <int L, int EP = 16> struct LineGeom {
    static constexpr int E = L >= EP ? EP : L;  // points per thread
    static constexpr int P = L / E;             // threads per line
    static constexpr int PADDED = L + (L >> 4) + 2;  // padded line stride in LDS
};

// Radix of Stockham step `st` for a line of 2^LOGL points: a leading step of
// radix 2^(LOGL mod 4) when that is not 0, then radix-16 steps.
template <int LOGL> struct Radices {
    static constexpr int LEAD = (LOGL < 4) ? LOGL : (LOGL % 4);
    static constexpr int NSTEPS = (LOGL < 4) ? 1 : (LOGL / 4 + (LEAD ? 1 : 0));
    static constexpr int radix(int st)
    {
        if (LOGL < 4) return 1 << LOGL;
        if (LEAD && st == 0) return 1 << LEAD;
        return 16;
    }
    static constexpr int span(int st)  // product of the radices before step st
    {
        int s = 1;
        for (int i = 0; i < st; ++i) s *= radix(i);
        return s;
    }
};

// Complex64 twiddle powers by a chain of FP64 products (1) or by the ladder
// below (0).
#ifndef EFFT_C64_TW_CHAIN
#define EFFT_C64_TW_CHAIN 1
#endif

// u[r] *= w^r for 0 < r < R, with w^r = w^(4a) * w^b formed from
// w, w^2, w^3, w^4, w^8, w^12 in FP64 (at most four roundings each) and
// rounded once to the storage type.
template <typename V, int R>
__device__ __forceinline__ void twiddle_line(V *u, double2 w)
{
    if constexpr (sizeof(decltype(V{}.x)) == 4 && EFFT_C64_TW_CHAIN) {
        // complex64: w^r by a chain of FP64 products (at most R - 2 roundings
        // in FP64, far below the one rounding to FP32), holding two FP64
        // values instead of the ladder's six
        double2 p = w;
        u[1] = cmul(u[1], round_tw<V>(p));
#pragma unroll
        for (int r = 2; r < R; ++r) {
            p = cmul(p, w);
            u[r] = cmul(u[r], round_tw<V>(p));
        }
    } else if constexpr (R == 2) {
        u[1] = cmul(u[1], round_tw<V>(w));
    } else {
        const double2 w2 = cmul(w, w);
        const double2 w3 = cmul(w2, w);
        u[1] = cmul(u[1], round_tw<V>(w));
        u[2] = cmul(u[2], round_tw<V>(w2));
        u[3] = cmul(u[3], round_tw<V>(w3));
        if constexpr (R > 4) {
            const double2 w4 = cmul(w2, w2);
#pragma unroll
            for (int a = 1; a < R / 4; ++a) {
                const double2 c = a == 1 ? w4 : a == 2 ? cmul(w4, w4) : cmul(cmul(w4, w4), w4);
                u[4 * a] = cmul(u[4 * a], round_tw<V>(c));
                u[4 * a + 1] = cmul(u[4 * a + 1], round_tw<V>(cmul(c, w)));
                u[4 * a + 2] = cmul(u[4 * a + 2], round_tw<V>(cmul(c, w2)));
                u[4 * a + 3] = cmul(u[4 * a + 3], round_tw<V>(cmul(c, w3)));
            }
        }
    }
}

// One Stockham step on the thread's E registers.  Butterfly j = t + P*b
// (b < E/R) takes points j + (L/R)*r, i.e. registers b + (E/R)*r; after the
// twiddle W_{NS*R}^{(j mod NS)*r} and an R-point DFT, output r goes to line
// position (j/NS)*NS*R + (j mod NS) + NS*r -- into LDS, or, on the last step
// (where that position is j + (L/R)*r), back into register b + (E/R)*r.
template <typename V, int L, int R, int NS, bool TO_LDS, int EP, bool TWL>
__device__ __forceinline__ void stockham_step(V *v, V *lds_line, int t, const TwTable &tt,
                                              uint64_t n_over_l, const V *ltw)
{
    constexpr int E = LineGeom<L, EP>::E;
    constexpr int P = LineGeom<L, EP>::P;
    constexpr int NB = E / R;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + P * b;
        V u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[b + NB * r];
        if constexpr (NS > 1 && TWL) {
            // W_{NS*R}^{jm*r} = W_L^{jm*r*L/(NS*R)} from the line's table in LDS
            const int jm = j & (NS - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) u[r] = cmul(u[r], ltw[(jm * r * (L / (NS * R))) & (L - 1)]);
        } else if constexpr (NS > 1) {
            int jm = j & (NS - 1);
            opaque_for<V>(jm);
            // W_{NS*R}^{jm} = W_N^{jm * N/(NS*R)}
            const uint64_t m = uint64_t(jm) * (n_over_l * uint64_t(L / (NS * R)));
            twiddle_line<V, R>(u, tw_lookup(tt, m));
        }
        dft<R>(u);
        if constexpr (TO_LDS) {
            const int base = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
            for (int r = 0; r < R; ++r) lds_line[lds_pad(base + NS * r)] = u[r];
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) v[b + NB * r] = u[r];
        }
    }
}

template <typename V, int L, int EP>
__device__ __forceinline__ void lds_gather(V *v, const V *lds_line, int t)
{
    constexpr int E = LineGeom<L, EP>::E;
    constexpr int P = LineGeom<L, EP>::P;
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = lds_line[lds_pad(t + P * i)];
}

// The exchange between two Stockham steps done one component at a time
// through a line buffer of real numbers (half the LDS of a complex one): on
// entry v holds the step's outputs in registers (output r of butterfly b in
// register b + (E/R)*r, line position (j/NS)*NS*R + (j mod NS) + NS*r); on
// exit v holds points t + P*i.  The real parts are written, gathered, then the
// imaginary parts: each gather overwrites only the component already written.
template <typename V, int L, int R, int NS, int EP>
__device__ __forceinline__ void exchange_split(V *v, decltype(V{}.x) *lds_line, int t)
{
    constexpr int E = LineGeom<L, EP>::E;
    constexpr int P = LineGeom<L, EP>::P;
    constexpr int NB = E / R;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = t + P * b;
            const int base = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
            for (int r = 0; r < R; ++r)
                lds_line[lds_pad(base + NS * r)] = comp ? v[b + NB * r].y : v[b + NB * r].x;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const auto w = lds_line[lds_pad(t + P * i)];
            if (comp)
                v[i].y = w;
            else
                v[i].x = w;
        }
        __syncthreads();
    }
}

// All Stockham steps of a line of 2^LOGL points.  On entry v holds input
// points t + P*i; on exit outputs k = t + P*i (FINAL_TO_LDS: the outputs are
// left in LDS at natural positions instead).
template <typename V, int LOGL, bool FINAL_TO_LDS, int EP, bool TWL = false, bool SPLIT = false>
__device__ __forceinline__ void line_fft(V *v, V *lds_line, int t, const TwTable &tt,
                                         uint64_t n_over_l, const V *ltw = nullptr)
{
    constexpr int L = 1 << LOGL;
    using Rd = Radices<LOGL>;
    constexpr int NST = Rd::NSTEPS;
    static_assert(NST <= 4, "line too long");
    if constexpr (SPLIT) {
        // lds_line is a line of PADDED real numbers
        static_assert(!FINAL_TO_LDS && NST >= 2, "component exchange between steps, outputs in registers");
        using T = decltype(V{}.x);
        T *ll = reinterpret_cast<T *>(lds_line);
        stockham_step<V, L, Rd::radix(0), 1, false, EP, TWL>(v, nullptr, t, tt, n_over_l, ltw);
        exchange_split<V, L, Rd::radix(0), 1, EP>(v, ll, t);
        if constexpr (NST >= 3) {
            stockham_step<V, L, Rd::radix(1), Rd::span(1), false, EP, TWL>(v, nullptr, t, tt, n_over_l, ltw);
            exchange_split<V, L, Rd::radix(1), Rd::span(1), EP>(v, ll, t);
        }
        if constexpr (NST >= 4) {
            stockham_step<V, L, Rd::radix(2), Rd::span(2), false, EP, TWL>(v, nullptr, t, tt, n_over_l, ltw);
            exchange_split<V, L, Rd::radix(2), Rd::span(2), EP>(v, ll, t);
        }
        stockham_step<V, L, Rd::radix(NST - 1), Rd::span(NST - 1), false, EP, TWL>(v, nullptr, t, tt, n_over_l,
                                                                                    ltw);
        return;
    }
    // step 0
    if constexpr (NST == 1) {
        stockham_step<V, L, Rd::radix(0), 1, FINAL_TO_LDS, EP, TWL>(v, lds_line, t, tt, n_over_l, ltw);
        return;
    } else {
        stockham_step<V, L, Rd::radix(0), 1, true, EP, TWL>(v, lds_line, t, tt, n_over_l, ltw);
        __syncthreads();
        lds_gather<V, L, EP>(v, lds_line, t);
        __syncthreads();
        if constexpr (NST == 2) {
            stockham_step<V, L, Rd::radix(1), Rd::span(1), FINAL_TO_LDS, EP, TWL>(v, lds_line, t, tt, n_over_l, ltw);
        } else {
            stockham_step<V, L, Rd::radix(1), Rd::span(1), true, EP, TWL>(v, lds_line, t, tt, n_over_l, ltw);
            __syncthreads();
            lds_gather<V, L, EP>(v, lds_line, t);
            __syncthreads();
            if constexpr (NST == 3) {
                stockham_step<V, L, Rd::radix(2), Rd::span(2), FINAL_TO_LDS, EP, TWL>(v, lds_line, t, tt, n_over_l, ltw);
            } else {
                stockham_step<V, L, Rd::radix(2), Rd::span(2), true, EP, TWL>(v, lds_line, t, tt, n_over_l, ltw);
                __syncthreads();
                lds_gather<V, L, EP>(v, lds_line, t);
                __syncthreads();
                stockham_step<V, L, Rd::radix(3), Rd::span(3), FINAL_TO_LDS, EP, TWL>(v, lds_line, t, tt, n_over_l, ltw);
            }
        }
    }
}

// Multiply v[i] (output k = t + P*i of a line) by W_N^(g*k*scale): two table
// lookups, then W^(g*scale*(t + P*(4a + b))) = c_a * s^b with c_a = w0 * s^(4a)
// (c_{a+1} = c_a * s^4), s = W^(g*scale*P), all in FP64 and rounded once to
// the storage type.
template <typename V, int E, int P>
__device__ __forceinline__ void apply_stage_twiddle(V *v, int t, uint64_t g, uint64_t scale,
                                                    const TwTable &tt)
{
    const uint64_t gs = g * scale;
    opaque_for<V>(t);
    const double2 w0 = tw_lookup(tt, gs * uint64_t(t));
    const double2 s1 = tw_lookup(tt, gs * uint64_t(P));
    if constexpr (E == 1) {
        v[0] = cmul(v[0], round_tw<V>(w0));
    } else if constexpr (sizeof(decltype(V{}.x)) == 4 && EFFT_C64_TW_CHAIN) {
        // complex64: the same powers by a chain of FP64 products (see twiddle_line)
        double2 c = w0;
        v[0] = cmul(v[0], round_tw<V>(c));
#pragma unroll
        for (int i = 1; i < E; ++i) {
            c = cmul(c, s1);
            v[i] = cmul(v[i], round_tw<V>(c));
        }
    } else {
        const double2 s2 = cmul(s1, s1);
        const double2 s3 = cmul(s2, s1);
        const double2 s4 = cmul(s2, s2);
        double2 c = w0;
#pragma unroll
        for (int a = 0; a < (E + 3) / 4; ++a) {
            if (a > 0) c = cmul(c, s4);
#pragma unroll
            for (int b = 0; b < 4 && 4 * a + b < E; ++b) {
                const int i = 4 * a + b;
                const double2 w = b == 0 ? c : b == 1 ? cmul(c, s1) : b == 2 ? cmul(c, s2) : cmul(c, s3);
                v[i] = cmul(v[i], round_tw<V>(w));
            }
        }
    }
}

// Output scaling (last pass only) and the conjugation of the backward direction.
template <typename V, int E>
__device__ __forceinline__ void finish_outputs(V *v, const StageParams &sp)
{
    using T = decltype(V{}.x);
    if (sp.apply_scale) {
        const T f = T(sp.scale);
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = V{v[i].x * f, v[i].y * f};
    }
    if (sp.conj) {
#pragma unroll
        for (int i = 0; i < E; ++i) v[i].y = -v[i].y;
    }
}

// Workgroup -> tile order.  The hardware deals consecutive workgroups round
// robin to the 8 XCDs.  TILE_XCD hands each XCD one contiguous run of tiles,
// so neighbouring tiles (adjacent row segments) are in flight on one XCD at
// the same time; TILE_XCD_SCATTER additionally walks each XCD's run with an
// odd multiplicative stride, which spreads concurrent tiles of a pass whose
// lines are far apart in memory over more DRAM channels; `mul` is that
// stride in tiles (odd; chosen per pass by scatter_stride).
__device__ __forceinline__ int64_t order_tiles(int64_t bid, int64_t ntiles, int mode, int64_t mul = 1)
{
    // the multiplicative walk is a permutation only for a power-of-two count
    // (a batch of 3 signals, say, has 3 * 2^k tiles): use the plain XCD order
    if (mode == TILE_XCD_SCATTER && (ntiles & (ntiles - 1)) != 0) mode = TILE_XCD;
    if (mode == TILE_XCD && (ntiles & 7) == 0) return (bid & 7) * (ntiles >> 3) + (bid >> 3);
    if (mode == TILE_XCD_SCATTER && (ntiles & 63) == 0) {
        const int64_t c = ntiles >> 3, k = bid >> 3;  // c is a power of two
        return (bid & 7) * c + ((k * mul) & (c - 1));
    }
    return bid;
}

// Addresses of one tile's lines for the thread's line c (one per set).
template <int SETS> struct TileLines {
    int64_t tile;
    int64_t base[SETS], off[SETS], blk[SETS];
    int64_t ubase[SETS];  // strided layouts: base of the set's first line (the same in every lane)
};

template <int L, int LINES, int SETS, int LAYOUT>
__device__ __forceinline__ TileLines<SETS> tile_lines(int64_t tile, int c, const StageParams &sp)
{
    TileLines<SETS> a;
    a.tile = tile;
#pragma unroll
    for (int st = 0; st < SETS; ++st) {
        const int64_t line = tile * (LINES * SETS) + st * LINES + c;
        if constexpr (LAYOUT == LAYOUT_ROW2COL) {
            // the tile's lines are LINES consecutive output columns; the source
            // row of output column `line` is its digit reversal within its
            // signal (row_mul = N / L columns per signal of a batch)
            const int64_t cols = sp.row_mul;
            if (sp.ilv > 1) {
                // interleaved output: line l of a group of ilv signals is
                // output column l, i.e. column l / ilv of signal l mod ilv
                const int64_t gl = cols * sp.ilv;
                const int64_t g = line / gl, l2 = line - g * gl;
                const int64_t cc = l2 / sp.ilv, b = l2 - cc * sp.ilv;
                a.blk[st] = (g * sp.ilv + b) * cols + int64_t(digit_reverse(uint64_t(cc), sp.rev));
            } else {
                a.blk[st] = (line & ~(cols - 1)) | int64_t(digit_reverse(uint64_t(line & (cols - 1)), sp.rev));
            }
            a.off[st] = 0;
            a.base[st] = a.blk[st] * L;
        } else if constexpr (LAYOUT == LAYOUT_ROW) {
            // contiguous lines (s = 1): line l starts at l * B
            a.blk[st] = line;
            a.off[st] = 0;
            a.base[st] = line * sp.B;
        } else {
            // strided lines: the LINES lines of a set are adjacent offsets of
            // one block (s is a power of two and a multiple of LINES * SETS),
            // so the block and the first offset are the same for the whole
            // workgroup and only the line c within the set varies per lane
            const int64_t line0 = tile * (LINES * SETS) + st * LINES;
            const int ls = __builtin_ctzll(uint64_t(sp.s));
            a.blk[st] = line0 >> ls;
            a.off[st] = (line0 & (sp.s - 1)) + c;
            a.ubase[st] = a.blk[st] * sp.B + (line0 & (sp.s - 1));
            a.base[st] = a.ubase[st] + c;
        }
    }
    return a;
}

// Loads of a strided tile with wave-uniform row bases (see wave_offset_fits):
// point i of set st of a lane is at ubase[st] + s * (t0 + P * i) plus the
// lane's byte offset.
template <typename V, int E, int P, int SETS>
__device__ __forceinline__ void load_tile_uniform(V (&v)[SETS][E], const TileLines<SETS> &a, const V *src,
                                                  int64_t s, int64_t t0, uint32_t loff, int nt)
{
#pragma unroll
    for (int i = 0; i < E; ++i) {
#pragma unroll
        for (int st = 0; st < SETS; ++st)
            v[st][i] = load_g(at_offset(wave_uniform(src + (a.ubase[st] + s * (t0 + int64_t(P) * i))), loff), nt);
    }
}

template <typename V, int E, int P, int SETS>
__device__ __forceinline__ void load_tile(V (&v)[SETS][E], const TileLines<SETS> &a, const V *src, int t,
                                          int64_t s, int nt)
{
    if (nt) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
#pragma unroll
            for (int st = 0; st < SETS; ++st) v[st][i] = load_nt(src + a.base[st] + s * int64_t(t + P * i));
        }
    } else {
#pragma unroll
        for (int i = 0; i < E; ++i) {
#pragma unroll
            for (int st = 0; st < SETS; ++st) v[st][i] = src[a.base[st] + s * int64_t(t + P * i)];
        }
    }
}

// load_tile with the factors of a PreMode (transposing first passes only):
// the same products, in the same precision, as a separate pointwise pass.
template <typename V, int E, int P, int SETS>
__device__ __forceinline__ void load_tile_pre(V (&v)[SETS][E], const TileLines<SETS> &a, const V *src, int t,
                                              const StageParams &sp)
{
    using T = decltype(V{}.x);
    if (sp.pmode == PRE_MUL) {
        const V *f = static_cast<const V *>(sp.pre);
#pragma unroll
        for (int i = 0; i < E; ++i) {
#pragma unroll
            for (int st = 0; st < SETS; ++st) {
                const int64_t n = a.base[st] + sp.s * int64_t(t + P * i);
                v[st][i] = sp.nt_load ? cmul(load_nt(src + n), load_nt(f + n)) : cmul(src[n], f[n]);
            }
        }
    } else {
        const double2 *c = static_cast<const double2 *>(sp.pre);
#pragma unroll
        for (int i = 0; i < E; ++i) {
#pragma unroll
            for (int st = 0; st < SETS; ++st) {
                const int64_t n = a.base[st] + sp.s * int64_t(t + P * i);
                V r{T(0), T(0)};
                if (n < sp.n_valid) {
                    const V x = sp.nt_load ? load_nt(src + n) : src[n];
                    const double2 cn = sp.nt_load ? load_nt(c + n) : c[n];
                    const double2 pr = cmul(double2{double(x.x), double(x.y)}, cn);
                    r = V{T(pr.x), T(pr.y)};
                }
                v[st][i] = r;
            }
        }
    }
}

// The chirp path's last stores: point n = n0 + stride * i goes to
// post_out[n] times post_scale * post[n] (FP64, rounded once; the product a
// separate post-multiply pass computes) if n < n_valid, and nowhere else.
template <typename V, int E>
__device__ __forceinline__ void store_post(const V *w, int64_t n0, int64_t stride, const StageParams &sp)
{
    using T = decltype(V{}.x);
    const double2 *c = static_cast<const double2 *>(sp.post);
    V *out = static_cast<V *>(sp.post_out);
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int64_t n = n0 + stride * i;
        if (n < sp.n_valid) {
            const double2 a = load_nt(c + n);
            const double2 p = cmul(double2{double(w[i].x), double(w[i].y)},
                                   double2{a.x * sp.post_scale, a.y * sp.post_scale});
            store_nt(out + n, V{T(p.x), T(p.y)});
        }
    }
}

// Line sets of a strided tile are stored together once all are transformed
// (1) or each as soon as it is done (0).
#ifndef EFFT_SETS_STORE_TOGETHER
#define EFFT_SETS_STORE_TOGETHER 0
#endif

// Stores of E points of a thread, point i at p + stride * i (last point
// first with EFFT_STORE_REVERSE: the rows a tile loaded last, whose address
// translations are the most recent, are then written first).
#ifndef EFFT_STORE_REVERSE
#define EFFT_STORE_REVERSE 0
#endif
template <typename V, int E>
__device__ __forceinline__ void store_points(V *p, int64_t stride, const V *w, int nt)
{
    if (nt) {
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int i = EFFT_STORE_REVERSE ? E - 1 - k : k;
            store_nt(p + stride * i, w[i]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const int i = EFFT_STORE_REVERSE ? E - 1 - k : k;
            p[stride * i] = w[i];
        }
    }
}

// Transform the loaded tile and store it (the layout decides where).
// Whether a pass kernel exchanges lines between Stockham steps one component
// at a time (exchange_split): its LDS buffer is then half as large, so two
// workgroups can share a CU where the registers allow it.
// Measured on gfx950 (2^30 complex128 in place): the stride-2^10 pass of
// single-set tiles, two workgroups per CU instead of one, 6.67 -> 6.24 ms;
// the first pass is held to one workgroup per CU by the registers of its two
// line sets and does not gain, nor do the row passes (4 -> 8 workgroups per
// CU: 5.44 -> 5.68 ms) or complex64 (its tiles already share CUs).
#ifndef EFFT_SPLIT_C128
#define EFFT_SPLIT_C128 1
#endif
#ifndef EFFT_SPLIT_C64
#define EFFT_SPLIT_C64 0
#endif
// The rows-to-columns pass (LAYOUT_ROW2COL) of complex128: its final
// transpose through LDS goes one component at a time too, and it then runs
// one tile per workgroup instead of two in turn, so two workgroups share a CU
// (measured on gfx950, the last pass of the 2^30 scratch schedule: 7.99 ->
// 6.63 ms).
#ifndef EFFT_SPLIT_R2C
#define EFFT_SPLIT_R2C 1
#endif
// the same for the columns-to-rows pass (LAYOUT_COL2ROW, the out-of-place
// first pass) of complex128 (measured on gfx950: 2^30 out of place, 8.57 ->
// 7.24 ms; 2^28 2.21 -> 1.88 ms; 2^20 25 -> 21 us)
#ifndef EFFT_SPLIT_C2R
#define EFFT_SPLIT_C2R 1
#endif
// and for its form that applies factors as it loads (LAYOUT_COL2ROW_PRE, the
// chirp path's first passes: 2^28 + 1 complex128 in place, 47.0 -> 43.7 ms)
#ifndef EFFT_SPLIT_C2R_PRE
#define EFFT_SPLIT_C2R_PRE 1
#endif
template <typename V, int LOGL, int SETS, int LAYOUT> constexpr bool split_exchange()
{
    if (Radices<LOGL>::NSTEPS < 2) return false;
    if (LAYOUT == LAYOUT_ROW2COL) return sizeof(decltype(V{}.x)) == 8 && EFFT_SPLIT_R2C && SETS == 1;
    if (LAYOUT == LAYOUT_COL2ROW) return sizeof(decltype(V{}.x)) == 8 && EFFT_SPLIT_C2R && SETS == 1;
    if (LAYOUT == LAYOUT_COL2ROW_PRE) return sizeof(decltype(V{}.x)) == 8 && EFFT_SPLIT_C2R_PRE && SETS == 1;
    const bool col = LAYOUT == LAYOUT_COL || LAYOUT == LAYOUT_COL_POST;
    if (!col && LAYOUT != LAYOUT_ROW) return false;
    const int mode = sizeof(decltype(V{}.x)) == 8 ? EFFT_SPLIT_C128 : EFFT_SPLIT_C64;
    // 1: single-set strided passes; 2: also every-set strided passes; 3: also row passes
    if (mode == 1) return col && SETS == 1;
    if (mode == 2) return col;
    return mode >= 3;
}

template <typename V, int LOGL, int LINES, int SETS, int LAYOUT, int EP, bool TWL, int E>
__device__ __forceinline__ void process_tile(V (&v)[SETS][E], const TileLines<SETS> &a, V *lds, V *dst,
                                             int c, int t, int tid, const StageParams &sp, int64_t t0,
                                             uint32_t loff, const V *ltw)
{
    constexpr int L = 1 << LOGL;
    static_assert(E == LineGeom<L, EP>::E, "points per thread");
    constexpr int P = LineGeom<L, EP>::P;
    constexpr int PADDED = LineGeom<L, EP>::PADDED;
    if (sp.conj) {
#pragma unroll
        for (int st = 0; st < SETS; ++st) {
#pragma unroll
            for (int i = 0; i < E; ++i) v[st][i].y = -v[st][i].y;
        }
    }
    V *lds_line = lds + c * PADDED;
    if constexpr (LAYOUT == LAYOUT_ROW2COL) {
        // outputs land in LDS in natural order; re-read them across the tile's
        // lines (lane = line) and write output k of column `line` at
        // line + row_mul * k, so each store covers LINES consecutive elements
        constexpr bool SPLIT = split_exchange<V, LOGL, SETS, LAYOUT>();
        const int c2 = tid % LINES;
        const int t2 = tid / LINES;
        if constexpr (SPLIT) {
            // outputs k = t + P*i stay in registers; the transpose goes
            // through a buffer of real numbers, the real parts first, each
            // read overwriting only the component already written (written
            // out here and in the columns-to-rows branch: as one shared
            // helper the compiler gave these kernels 138-144 VGPRs instead of
            // 127-128, one workgroup per CU instead of two)
            using T = decltype(V{}.x);
            T *lt = reinterpret_cast<T *>(lds);
            line_fft<V, LOGL, false, EP, TWL, true>(v[0], reinterpret_cast<V *>(lt + c * PADDED), t, sp.tt,
                                                    sp.n_over_l, ltw);
#pragma unroll
            for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
                for (int i = 0; i < E; ++i) lt[c * PADDED + lds_pad(t + P * i)] = comp ? v[0][i].y : v[0][i].x;
                __syncthreads();
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    const T x = lt[c2 * PADDED + lds_pad(t2 + P * i)];
                    if (comp)
                        v[0][i].y = x;
                    else
                        v[0][i].x = x;
                }
                __syncthreads();
            }
        } else {
            line_fft<V, LOGL, true, EP, TWL>(v[0], lds_line, t, sp.tt, sp.n_over_l, ltw);
            __syncthreads();
            const V *col_lds = lds + c2 * PADDED;
#pragma unroll
            for (int i = 0; i < E; ++i) v[0][i] = col_lds[lds_pad(t2 + P * i)];
        }
        const int64_t cols = sp.row_mul;
        const int64_t line = a.tile * LINES + c2;
        int64_t col = (line & ~(cols - 1)) * L + (line & (cols - 1));  // signal * N + column
        int64_t ostride = cols;
        if (sp.ilv > 1) {  // group * (ilv N) + column l of the group, columns ilv * cols apart
            ostride = cols * sp.ilv;
            const int64_t g = line / ostride;
            col = g * ostride * L + (line - g * ostride);
        }
        finish_outputs<V, E>(v[0], sp);
        store_points<V, E>(dst + col + ostride * int64_t(t2), ostride * int64_t(P), v[0], sp.nt_store);
    } else if constexpr (LAYOUT != LAYOUT_COL2ROW && LAYOUT != LAYOUT_COL2ROW_PRE) {
#pragma unroll
        for (int st = 0; st < SETS; ++st) {
            if (st > 0) __syncthreads();  // the previous set has finished with LDS
            // each set recomputes its twiddles and LDS addresses (opaque
            // copies): keeping the first set's for the second costs more
            // registers than recomputing them
            int tl = t, cl = c;
            opaque_for<V>(tl);
            opaque_for<V>(cl);
            constexpr bool SPLIT = split_exchange<V, LOGL, SETS, LAYOUT>();
            using T = decltype(V{}.x);
            V *my_line = SPLIT ? reinterpret_cast<V *>(reinterpret_cast<T *>(lds) + cl * PADDED) : lds + cl * PADDED;
            line_fft<V, LOGL, false, EP, TWL, SPLIT>(v[st], my_line, tl, sp.tt, sp.n_over_l, ltw);
            if (sp.twmode != TW_NONE) {
                const uint64_t g = sp.twmode == TW_OFFSET ? uint64_t(a.off[st])
                                                          : digit_reverse(uint64_t(a.blk[st]), sp.rev);
                apply_stage_twiddle<V, E, P>(v[st], t, g, sp.tw_scale, sp.tt);
            }
            finish_outputs<V, E>(v[st], sp);
            if constexpr (LAYOUT == LAYOUT_COL_POST)
                store_post<V, E>(v[st], a.base[st] + sp.s * int64_t(t), sp.s * int64_t(P), sp);
            else if constexpr (SETS == 1 || !EFFT_SETS_STORE_TOGETHER)
            {
                if (uniform_code<V>() && sp.off32) {
#pragma unroll
                    for (int i = 0; i < E; ++i)
                        store_g(at_offset(wave_uniform(dst + (a.ubase[st] + sp.s * (t0 + int64_t(P) * i))), loff),
                                v[st][i], sp.nt_store);
                } else {
                    store_points<V, E>(dst + a.base[st] + sp.s * int64_t(t), sp.s * int64_t(P), v[st], sp.nt_store);
                }
            }
        }
        if constexpr (LAYOUT != LAYOUT_COL_POST && SETS > 1 && EFFT_SETS_STORE_TOGETHER) {
            // every set's outputs are kept until the last set is done, then
            // each tile row is written as one run across the sets (as it was
            // read): one address translation per row instead of one per set
            // and row, and the long runs the loads have
#pragma unroll
            for (int i = 0; i < E; ++i) {
#pragma unroll
                for (int st = 0; st < SETS; ++st) {
                    V *q = dst + a.base[st] + sp.s * int64_t(t + P * i);
                    if (sp.nt_store)
                        store_nt(q, v[st][i]);
                    else
                        *q = v[st][i];
                }
            }
        }
    } else {
        // outputs land in LDS in natural order; re-read them one contiguous
        // row per line and write that row at its digit-reversed position
        const int t2 = tid % P;
        const int c2 = tid / P;
        constexpr bool SPLIT = split_exchange<V, LOGL, SETS, LAYOUT>();
        V w[E];
        if constexpr (SPLIT) {
            // through a buffer of real numbers, one component at a time (as
            // in the rows-to-columns pass), into the same registers
            using T = decltype(V{}.x);
            T *lt = reinterpret_cast<T *>(lds);
            line_fft<V, LOGL, false, EP, TWL, true>(v[0], reinterpret_cast<V *>(lt + c * PADDED), t, sp.tt,
                                                    sp.n_over_l, ltw);
#pragma unroll
            for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
                for (int i = 0; i < E; ++i) lt[c * PADDED + lds_pad(t + P * i)] = comp ? v[0][i].y : v[0][i].x;
                __syncthreads();
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    const T x = lt[c2 * PADDED + lds_pad(t2 + P * i)];
                    if (comp)
                        v[0][i].y = x;
                    else
                        v[0][i].x = x;
                }
                __syncthreads();
            }
        } else {
            line_fft<V, LOGL, true, EP, TWL>(v[0], lds_line, t, sp.tt, sp.n_over_l, ltw);
            __syncthreads();
        }
        // one block per signal (B = N): line = signal * s + offset o2
        const int64_t line = a.tile * LINES + c2;
        const int64_t o2 = line & (sp.s - 1);
        if constexpr (SPLIT) {
#pragma unroll
            for (int i = 0; i < E; ++i) w[i] = v[0][i];
        } else {
            const V *row_lds = lds + c2 * PADDED;
#pragma unroll
            for (int i = 0; i < E; ++i) w[i] = row_lds[lds_pad(t2 + P * i)];
        }
        apply_stage_twiddle<V, E, P>(w, t2, uint64_t(o2), sp.tw_scale, sp.tt);
        finish_outputs<V, E>(w, sp);
        const int64_t row = (line - o2) * L + sp.row_mul * int64_t(digit_reverse(uint64_t(o2), sp.rev));
        store_points<V, E>(dst + row + t2, int64_t(P), w, sp.nt_store);
    }
}

// One pass: each workgroup transforms PIPE tiles of LINES * SETS lines in
// turn.  Thread (c, t) owns points t + P*i of lines c + LINES*set of a tile:
// the SETS line sets are loaded together, so a strided tile row is one
// LINES*SETS-element run, and then transformed one set at a time through the
// same LDS buffer.  With PIPE > 1 the loads of the next tile are issued
// before the current tile is transformed, so memory traffic continues while
// the CU computes.
template <int LOGL, int LINES, int EP> constexpr int stage_threads()
{
    return LINES * LineGeom<(1 << LOGL), EP>::P;
}

// Waves per SIMD a pass kernel must leave room for: the component-wise
// exchange, and the half-width complex64 tiles of 256-point lines, exist so
// that two 512-thread workgroups share a CU (4 waves per SIMD, at most 128
// VGPRs each), and the bound keeps a code change from silently taking that
// back.
template <typename T, int LOGL, int LINES, int SETS, int LAYOUT, int EP> constexpr int stage_min_waves()
{
    return ((split_exchange<typename vec2<T>::type, LOGL, SETS, LAYOUT>() ||
             (sizeof(T) == 4 && LOGL == 8 && LAYOUT == LAYOUT_COL)) &&
            stage_threads<LOGL, LINES, EP>() == 512)
               ? 4
               : 1;
}

template <typename T, int LOGL, int LINES, int SETS, int LAYOUT, int PIPE, int EP>
__global__ void __launch_bounds__((stage_threads<LOGL, LINES, EP>()),
                                  (stage_min_waves<T, LOGL, LINES, SETS, LAYOUT, EP>()))
    stage_kernel(StageParams sp)
{
    using V = typename vec2<T>::type;
    constexpr int L = 1 << LOGL;
    constexpr int E = LineGeom<L, EP>::E;
    constexpr int P = LineGeom<L, EP>::P;
    constexpr int PADDED = LineGeom<L, EP>::PADDED;
    constexpr bool NEED_LDS =
        (Radices<LOGL>::NSTEPS > 1) || (LAYOUT == LAYOUT_COL2ROW) || (LAYOUT == LAYOUT_COL2ROW_PRE) ||
        (LAYOUT == LAYOUT_ROW2COL);
    static_assert((LAYOUT != LAYOUT_COL2ROW && LAYOUT != LAYOUT_COL2ROW_PRE) || SETS == 1,
                  "one line set for row writes");
    static_assert(LAYOUT != LAYOUT_ROW2COL || SETS == 1, "one line set for column writes");
    constexpr bool SPLIT = split_exchange<V, LOGL, SETS, LAYOUT>();
    // the exchange buffer: LINES lines of complex numbers, or of real numbers
    // for the component-wise exchange (viewed through V * all the same)
    __shared__ V lds[NEED_LDS ? (SPLIT ? (LINES * PADDED + 1) / 2 : LINES * PADDED) : PADDED];
    // complex64: the in-line twiddles W_L^e of every Stockham step come from
    // a table of the line length in LDS, filled from the plan's FP32 table of
    // W_4096^e (computed in FP64, rounded once) -- no FP64 work per twiddle;
    // where the LDS has no room for it (2^12-point strided lines) they are
    // generated in FP64 as for complex128
    constexpr int LDS_EXCH = int(sizeof(V)) * (NEED_LDS ? (SPLIT ? (LINES * PADDED + 1) / 2 : LINES * PADDED) : PADDED);
    constexpr bool TWL = EFFT_C64_LDS_TW && sizeof(T) == 4 && Radices<LOGL>::NSTEPS > 1 &&
                         LDS_EXCH + L * int(sizeof(V)) <= 163840;
    __shared__ V ltw[TWL ? L : 1];
    if constexpr (TWL) {
        const float2 *g = sp.tt.line32;
        for (int e = threadIdx.x; e < L; e += int(blockDim.x)) ltw[e] = g[e * (LINE_TW_N / L)];
        // the first use follows the first exchange's barrier
    }

    const int tid = threadIdx.x;
    int c, t;
    if constexpr (LAYOUT == LAYOUT_ROW || LAYOUT == LAYOUT_ROW2COL) {
        t = tid % P;
        c = tid / P;
    } else {
        c = tid % LINES;
        t = tid / LINES;
    }
    const V *src = static_cast<const V *>(sp.src);
    V *dst = static_cast<V *>(sp.dst);
    // strided layouts: the wave's first t and the lane's byte offset from it
    // (c + s * (t - t0) elements; meaningful when sp.off32 is set)
    constexpr bool UNIFORM = uniform_code<V>();
    const int64_t t0 = UNIFORM ? (int64_t(__builtin_amdgcn_readfirstlane(tid >> 6)) * 64) / LINES : 0;
    const uint32_t loff = UNIFORM ? uint32_t((int64_t(c) + sp.s * (int64_t(t) - t0)) * int64_t(sizeof(V))) : 0;

    // virtual workgroup number of this workgroup's it-th tile: the PIPE tiles
    // of a workgroup stay on its XCD's run when the grid allows
    const int64_t groups = sp.ntiles / PIPE;
    const int64_t bid = blockIdx.x;
    auto vbid = [&](int it) -> int64_t {
        if ((groups & 7) == 0) return (bid & 7) + 8 * ((bid >> 3) * PIPE + it);
        return bid * PIPE + it;
    };

    V v[SETS][E];
    TileLines<SETS> a =
        tile_lines<L, LINES, SETS, LAYOUT>(order_tiles(vbid(0), sp.ntiles, sp.order, sp.scatter), c, sp);
    auto load = [&](V(&dst_v)[SETS][E], const TileLines<SETS> &at) {
        if constexpr (LAYOUT == LAYOUT_COL2ROW_PRE)
            load_tile_pre<V, E, P, SETS>(dst_v, at, src, t, sp);
        else if constexpr (LAYOUT == LAYOUT_COL || LAYOUT == LAYOUT_COL_POST || LAYOUT == LAYOUT_COL2ROW) {
            if (UNIFORM && sp.off32)
                load_tile_uniform<V, E, P, SETS>(dst_v, at, src, sp.s, t0, loff, sp.nt_load);
            else
                load_tile<V, E, P, SETS>(dst_v, at, src, t, sp.s, sp.nt_load);
        } else
            load_tile<V, E, P, SETS>(dst_v, at, src, t, sp.s, sp.nt_load);
    };
    load(v, a);
#pragma unroll
    for (int it = 0; it < PIPE; ++it) {
        V vn[SETS][E];
        TileLines<SETS> an;
        if (it + 1 < PIPE) {
            an = tile_lines<L, LINES, SETS, LAYOUT>(order_tiles(vbid(it + 1), sp.ntiles, sp.order, sp.scatter), c,
                                                    sp);
            load(vn, an);
        }
        if (it > 0) __syncthreads();  // the previous tile has finished with LDS
        process_tile<V, LOGL, LINES, SETS, LAYOUT, EP, TWL>(v, a, lds, dst, c, t, tid, sp, t0, loff, ltw);
        if (it + 1 < PIPE) {
#pragma unroll
            for (int st = 0; st < SETS; ++st) {
#pragma unroll
                for (int i = 0; i < E; ++i) v[st][i] = vn[st][i];
            }
            a = an;
        }
    }
}

// ---------------------------------------------------------------- launchers
// Set while a host-only caller checks that a kernel exists for every pass of
// a plan: the launchers then return success without launching anything.
extern thread_local bool g_dry_run;  // defined in efft_kernels.hip

template <typename T, int LOGL, int LINES, int SETS, int LAYOUT, int PIPE, int EP>
static hipError_t launch_pipe(const StageParams &p, hipStream_t stream)
{
    constexpr int NT = LINES * LineGeom<(1 << LOGL), EP>::P;
    if (p.ntiles % PIPE) return hipErrorInvalidValue;
    if (g_dry_run) return hipSuccess;
    hipLaunchKernelGGL((stage_kernel<T, LOGL, LINES, SETS, LAYOUT, PIPE, EP>), dim3(unsigned(p.ntiles / PIPE)),
                       dim3(NT), 0, stream, p);
    return hipGetLastError();
}

// tiles per workgroup (software pipelining depth) of each layout
#ifndef EFFT_PIPE_COL
#define EFFT_PIPE_COL 1
#endif
#ifndef EFFT_PIPE_ROW
#define EFFT_PIPE_ROW 1
#endif
#ifndef EFFT_PIPE_X
#define EFFT_PIPE_X 2
#endif

template <typename T, int LOGL, int LINES, int SETS, int LAYOUT, int EP = 16>
static hipError_t launch_one(const StageParams &p, hipStream_t stream)
{
    // a second tile in flight costs one more tile of registers: only
    // workgroups of at most 512 threads at 16 points per thread have room
    // (not where the exchange goes one component at a time: its smaller LDS
    // buffer lets two workgroups share a CU instead)
    constexpr bool ROOM = SETS == 1 && EP == 16 && LINES * LineGeom<(1 << LOGL), EP>::P <= 512 &&
                          !split_exchange<typename vec2<T>::type, LOGL, SETS, LAYOUT>();
    constexpr int PIPE = !ROOM ? 1
                         : (LAYOUT == LAYOUT_COL || LAYOUT == LAYOUT_COL_POST) ? EFFT_PIPE_COL
                         : (LAYOUT == LAYOUT_ROW) ? EFFT_PIPE_ROW : EFFT_PIPE_X;
    if (PIPE > 1 && p.ntiles >= 64 * PIPE && p.ntiles % PIPE == 0)
        return launch_pipe<T, LOGL, LINES, SETS, LAYOUT, PIPE, EP>(p, stream);
    return launch_pipe<T, LOGL, LINES, SETS, LAYOUT, 1, EP>(p, stream);
}

template <typename T, int LOGL>
static hipError_t dispatch_logl(int layout, int lines, int sets, const StageParams &p,
                                hipStream_t stream)
{
    constexpr int EB = int(2 * sizeof(T));
    constexpr int P = LineGeom<(1 << LOGL)>::P;
    constexpr int ROWW = P >= 256 ? 1 : 256 / P;
    constexpr int EPC = col_points(EB, LOGL);
    constexpr int WMAX = col_lines_max(EB, LOGL);
    constexpr int WMIN = col_lines_narrow(EB, LOGL);
    if (layout == LAYOUT_ROW) {
        if (sets != 1) return hipErrorInvalidValue;
        if (lines == ROWW) return launch_one<T, LOGL, ROWW, 1, LAYOUT_ROW>(p, stream);
        if (lines == 1) return launch_one<T, LOGL, 1, 1, LAYOUT_ROW>(p, stream);
        return hipErrorInvalidValue;
    }
    if constexpr (LOGL >= 4 && LOGL <= STRIDED_LOGL_MAX) {
        if (layout == LAYOUT_COL) {
            if (lines == WMAX && sets == 1) return launch_one<T, LOGL, WMAX, 1, LAYOUT_COL, EPC>(p, stream);
            if constexpr ((LOGL == 10 && WMAX * EB == 128) || ((LOGL == 9 || LOGL == 8) && EB == 8)) {
                if (lines == WMAX && sets == 2) return launch_one<T, LOGL, WMAX, 2, LAYOUT_COL, EPC>(p, stream);
            }
            if constexpr (LOGL == 8 && EB == 8) {  // the half-width two-set tile (col_set_lines)
                if (lines == WMAX / 2 && sets == 2) return launch_one<T, LOGL, WMAX / 2, 2, LAYOUT_COL, EPC>(p, stream);
            }
            if constexpr (LOGL == 8 && EB == 8) {  // the half-width one-set tile (col_set_lines)
                if (lines == WMAX / 2 && sets == 1) return launch_one<T, LOGL, WMAX / 2, 1, LAYOUT_COL, EPC>(p, stream);
            }
            if constexpr (WMIN != WMAX) {
                if (lines == WMIN && sets == 1) return launch_one<T, LOGL, WMIN, 1, LAYOUT_COL, EPC>(p, stream);
            }
            if constexpr (EB == 8 && LOGL == 10 && C64_SHARED_LINES != WMIN && C64_SHARED_LINES != WMAX) {
                if (lines == C64_SHARED_LINES && sets == 1)
                    return launch_one<T, LOGL, C64_SHARED_LINES, 1, LAYOUT_COL, EPC>(p, stream);
            }
            if constexpr (LOGL >= 8 && WMIN / 2 >= 2) {
                if (lines == WMIN / 2 && sets == 1) return launch_one<T, LOGL, WMIN / 2, 1, LAYOUT_COL, EPC>(p, stream);
            }
            if constexpr (LOGL >= 8 && WMIN / 4 >= 2) {
                if (lines == WMIN / 4 && sets == 1) return launch_one<T, LOGL, WMIN / 4, 1, LAYOUT_COL, EPC>(p, stream);
            }
        }
        if (layout == LAYOUT_COL_POST) {
            if (lines == WMAX && sets == 1) return launch_one<T, LOGL, WMAX, 1, LAYOUT_COL_POST, EPC>(p, stream);
            if constexpr ((LOGL == 10 && WMAX * EB == 128) || ((LOGL == 9 || LOGL == 8) && EB == 8)) {
                if (lines == WMAX && sets == 2) return launch_one<T, LOGL, WMAX, 2, LAYOUT_COL_POST, EPC>(p, stream);
            }
            if constexpr (WMIN != WMAX) {
                if (lines == WMIN && sets == 1) return launch_one<T, LOGL, WMIN, 1, LAYOUT_COL_POST, EPC>(p, stream);
            }
            if constexpr (EB == 8 && LOGL == 10 && C64_SHARED_LINES != WMIN && C64_SHARED_LINES != WMAX) {
                if (lines == C64_SHARED_LINES && sets == 1)
                    return launch_one<T, LOGL, C64_SHARED_LINES, 1, LAYOUT_COL_POST, EPC>(p, stream);
            }
        }
        if (layout == LAYOUT_COL2ROW_PRE && sets == 1) {
            if (lines == WMAX) return launch_one<T, LOGL, WMAX, 1, LAYOUT_COL2ROW_PRE, EPC>(p, stream);
            if constexpr (WMIN != WMAX) {
                if (lines == WMIN) return launch_one<T, LOGL, WMIN, 1, LAYOUT_COL2ROW_PRE, EPC>(p, stream);
            }
        }
        if (layout == LAYOUT_COL2ROW && sets == 1) {
            if (lines == WMAX) return launch_one<T, LOGL, WMAX, 1, LAYOUT_COL2ROW, EPC>(p, stream);
            if constexpr (WMIN != WMAX) {
                if (lines == WMIN) return launch_one<T, LOGL, WMIN, 1, LAYOUT_COL2ROW, EPC>(p, stream);
            }
            // narrower tiles for grids too small to fill the device
            if constexpr (LOGL >= 8 && WMIN / 2 >= 2) {
                if (lines == WMIN / 2) return launch_one<T, LOGL, WMIN / 2, 1, LAYOUT_COL2ROW, EPC>(p, stream);
            }
            if constexpr (LOGL >= 8 && WMIN / 4 >= 2) {
                if (lines == WMIN / 4) return launch_one<T, LOGL, WMIN / 4, 1, LAYOUT_COL2ROW, EPC>(p, stream);
            }
        }
        if (layout == LAYOUT_ROW2COL && sets == 1) {
            if (lines == WMAX) return launch_one<T, LOGL, WMAX, 1, LAYOUT_ROW2COL, EPC>(p, stream);
            if constexpr (WMIN != WMAX) {
                if (lines == WMIN) return launch_one<T, LOGL, WMIN, 1, LAYOUT_ROW2COL, EPC>(p, stream);
            }
        }
    }
    return hipErrorInvalidValue;
}

// dispatch_logl for the line lengths 2^LO .. 2^HI
template <typename T, int LO, int HI>
static hipError_t dispatch_range(int layout, int logl, int lines, int sets, const StageParams &p, hipStream_t stream)
{
    if constexpr (LO > HI) {
        return hipErrorInvalidValue;
    } else {
        if (logl == LO) return dispatch_logl<T, LO>(layout, lines, sets, p, stream);
        return dispatch_range<T, LO + 1, HI>(layout, logl, lines, sets, p, stream);
    }
}

// defines launcher NAME for element type T and line lengths 2^LO .. 2^HI
#define EFFT_STAGE_LAUNCHER(NAME, T, LO, HI)                                                                   \
    hipError_t NAME(int layout, int logl, int lines, int sets, const StageParams &p, hipStream_t stream)   \
    {                                                                                                      \
        return dispatch_range<T, LO, HI>(layout, logl, lines, sets, p, stream);                              \
    }

}  // namespace efft
