// efft_internal.hpp -- pass descriptors shared by the planner and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "efft_device.hpp"

namespace efft {

// How the lines of one sub-FFT pass sit in memory.
enum Layout : int {
    LAYOUT_ROW = 0,     // contiguous lines (stride 1), one or more per workgroup
    LAYOUT_COL = 1,     // strided lines; a workgroup takes W adjacent lines, so
                        // every row of its tile is one contiguous W-element run
    LAYOUT_COL2ROW = 2, // strided lines read as LAYOUT_COL, each written back
                        // as a contiguous row at a digit-reversed row index
    LAYOUT_ROW2COL = 3, // contiguous rows read from a scratch array, each
                        // written as a strided column of the output, in
                        // natural order (the last pass of a scratch plan)
    LAYOUT_COL2ROW_PRE = 4, // LAYOUT_COL2ROW whose loads apply the factors of
                            // sp.pmode (separate kernels, so the plain
                            // transposing pass keeps its own code)
    LAYOUT_COL_POST = 5     // LAYOUT_COL whose outputs n < n_valid go to
                            // post_out times post_scale * post[n] (FP64), and
                            // the others nowhere: the chirp path's last pass
};

// Twiddle applied to output k of line (block b, offset o) of a pass.
enum TwMode : int {
    TW_NONE = 0,
    TW_OFFSET = 1,   // W_N^(o * k * scale)
    TW_REVBLOCK = 2  // W_N^(rev(b) * k * scale), rev = digit reversal of b
};

// What a LAYOUT_COL2ROW_PRE pass applies to each point it loads (point n of the
// signal): the factors of a pointwise product, or the chirp of a length that
// is not a power of two, with zero padding beyond the signal.
enum PreMode : int {
    PRE_NONE = 0,
    PRE_MUL = 1,   // src[n] * pre[n] (pre in the storage type)
    PRE_CHIRP = 2  // n < n_valid: src[n] * pre[n] in FP64 (pre: double2), rounded once; else 0
};

// Order in which workgroups visit the tiles of a pass (see order_tiles).
enum TileOrder : int { TILE_LINEAR = 0, TILE_XCD = 1, TILE_XCD_SCATTER = 2 };

// Digit list of a mixed-radix index, lowest digit first, each 2^bits[i].
struct Digits {
    int nd;
    int bits[6];
};

__host__ __device__ inline uint64_t digit_reverse(uint64_t v, const Digits &d)
{
    // v = d_0 + 2^b0 d_1 + ...; result has d_{nd-1} lowest, ..., d_0 highest
    uint64_t r = 0;
    for (int i = 0; i < d.nd; ++i) {
        const uint64_t digit = v & ((uint64_t(1) << d.bits[i]) - 1u);
        v >>= d.bits[i];
        r = (r << d.bits[i]) | digit;
    }
    return r;
}

// One sub-FFT pass.  Line l (0 <= l < N/L) is split as l = blk * s + o with
// 0 <= o < s; its element i sits at blk * B + o + s * i, B = s * L.
struct StageParams {
    const void *src;
    void *dst;
    int64_t s;
    int64_t B;
    int64_t ntiles;      // tiles of the pass (the grid has ntiles / PIPE workgroups)
    uint64_t n_over_l;   // N / L, scales the in-line Stockham twiddles
    uint64_t tw_scale;   // see TwMode
    int64_t row_mul;     // LAYOUT_COL2ROW: line o's row starts at row_mul * rev(o);
                         // LAYOUT_ROW2COL: column stride of the output
    const void *pre;     // LAYOUT_COL2ROW_PRE: factors applied on load (see PreMode)
    int64_t n_valid;     // PRE_CHIRP: points of the source signal; LAYOUT_COL_POST: points kept
    const void *post;    // LAYOUT_COL_POST: double2 factors (the chirp)
    void *post_out;      // LAYOUT_COL_POST: destination of the n_valid kept points
    double post_scale;   // LAYOUT_COL_POST: multiplies the factors
    int pmode;           // PreMode
    int64_t ilv;         // LAYOUT_ROW2COL: signals interleaved in the output (1: none).
                         // With ilv = M, bin k of signal b of each group of M signals
                         // lands at k * M + b of that group's M * N outputs
    Digits rev;          // digits of o (COL2ROW), of blk (TW_REVBLOCK) or of the
                         // output column index (ROW2COL, whose source row is its reversal)
    TwTable tt;
    double scale;        // multiplies every output when apply_scale is set
    int twmode;
    int conj;            // 1: backward direction (conjugate on load and store)
    int apply_scale;
    int order;           // TileOrder
    int64_t scatter;     // TILE_XCD_SCATTER: odd stride, in tiles, of each XCD's walk
    int nt_load;         // 1: data loads carry the non-temporal (streaming) hint
    int nt_store;        // 1: data stores carry it
    int off32;           // strided layouts: a lane's offset within its wave's rows fits 32 bits
                         // (set by the launcher; see wave_offset_fits)
};

// Strided tiles address point i of a lane as a wave-uniform row base plus the
// lane's offset c + s * (t - t0) within its wave (t0 the wave's first t): the
// base lives in scalar registers and every load and store of the lane shares
// one 32-bit offset register, so a tile's 16 to 32 loads can be in flight
// without a 64-bit address register each.  That needs the offset below 2^32
// bytes, which holds for every plan of the workloads; other plans take 64-bit
// addresses.
// Measured on gfx950 (2^30 points in place, first pass): complex64 gains
// (5.75 -> 5.58 ms with two line sets), complex128 loses (8.08 -> 9.00 ms),
// so complex128 keeps 64-bit addresses.
#ifndef EFFT_WAVE_UNIFORM
#define EFFT_WAVE_UNIFORM 1
#endif
#ifndef EFFT_WAVE_UNIFORM_C128
#define EFFT_WAVE_UNIFORM_C128 0
#endif
inline bool wave_offset_fits(int layout, int lines, int64_t s, int dtype_bytes)
{
    if (layout == LAYOUT_ROW || layout == LAYOUT_ROW2COL) return false;
    if (dtype_bytes == 16 && !EFFT_WAVE_UNIFORM_C128) return false;
    const int64_t rows = lines >= 64 ? 1 : 64 / lines;  // distinct t in one wave
    const int64_t bound = (int64_t(lines) + s * (rows - 1)) * dtype_bytes;
    return bound < (int64_t(1) << 31);
}

// Tiled in-place digit reversal of a [R][M][R] array: element (a, mu, b)
// swaps with (b, rev(mu), a).
struct SwapParams {
    void *data;
    int64_t R;     // outer digit size (first and last digit)
    int64_t M;     // product of the middle digits (1 if none)
    int64_t nt;    // R / tile
    Digits mid;    // middle digits, lowest first
    int64_t n;     // elements per signal (R * M * R)
    int nt_hint;   // 1: loads and stores carry the non-temporal (streaming) hint
};

// Tile edge of the digit-reversal swap: 64 x 64 tiles (512-byte runs for
// complex64, 1 KiB for complex128) when the outer digit allows; measured
// 1.2x faster than 32 x 32 for complex128 at N = 2^30.
#ifndef EFFT_SWAP_TS16
#define EFFT_SWAP_TS16 64
#endif
#ifndef EFFT_SWAP_TS8
#define EFFT_SWAP_TS8 64
#endif
inline int64_t swap_tile(int dtype_bytes, int64_t R)
{
    const int64_t ts = dtype_bytes == 16 ? EFFT_SWAP_TS16 : EFFT_SWAP_TS8;
    return R < ts ? R : ts;
}

// kernel launchers (efft_kernels.hip); return hipSuccess or the launch error
hipError_t launch_stage(int dtype_bytes, int layout, int logl, int lines, int sets,
                        const StageParams &p, hipStream_t stream);
// batch signals of p.n elements each, contiguous
hipError_t launch_swap(int dtype_bytes, const SwapParams &p, int64_t batch, hipStream_t stream);
hipError_t launch_twiddle_table(double2 *lo, int64_t n_lo, double2 *hi, int64_t n_hi, int h,
                                int q, hipStream_t stream);
// W_4096^e in FP32 for e < LINE_TW_N
hipError_t launch_line32_table(float2 *t, hipStream_t stream);
hipError_t launch_r2c_post(int dtype_bytes, void *z, int64_t h, const TwTable &tt, double scale,
                           int apply_scale, hipStream_t stream);
hipError_t launch_c2r_pre(int dtype_bytes, const void *f, void *z, int64_t h, const TwTable &tt,
                          hipStream_t stream);
// lengths that are not powers of two (chirp form, efft_bluestein.hip):
// a[j] = exp(sign*pi*i * (j^2 mod 2N)/N) for j < n (FP64)
hipError_t launch_chirp(double2 *a, int64_t n, int sign, hipStream_t stream);
// w[0..m) = conj(a_j)/m at j and m - j (0 <= j < n), zero elsewhere
hipError_t launch_chirp_v(int dtype_bytes, void *w, const double2 *a, int64_t n, int64_t m, hipStream_t stream);
// w[0..m) = (x a) zero-padded
hipError_t launch_premul(int dtype_bytes, const void *x, void *w, const double2 *a, int64_t n, int64_t m,
                         hipStream_t stream);
// w *= v over m points
hipError_t launch_pointwise(int dtype_bytes, void *w, const void *v, int64_t m, hipStream_t stream);
// out[0..n) = scale * a * w
hipError_t launch_postmul(int dtype_bytes, const void *w, void *out, const double2 *a, int64_t n, double scale,
                          hipStream_t stream);
// lengths N = M * 2^s with a small odd M (efft_mixed.hip): tables W_M^j and
// the two-level W_N table; the radix-M pass (x -> w) and the reorder pass
// (w -> out, times scale), for `batch` contiguous signals
hipError_t launch_mixed_tables(double2 *wm, int m, double2 *lo, int64_t n_lo, double2 *hi, int64_t n_hi, int h,
                               int64_t n, hipStream_t stream);
hipError_t launch_radix_m(int dtype_bytes, int m, const void *x, void *w, const double2 *wm, const double2 *lo,
                          const double2 *hi, int h, int64_t cols, int64_t batch, int conj, hipStream_t stream);
hipError_t launch_reorder_m(int dtype_bytes, int m, const void *w, void *out, int64_t cols, int64_t batch,
                            double scale, hipStream_t stream);
// while on (per host thread), launch_stage / launch_swap only check that a
// kernel exists for the arguments and launch nothing
void set_dry_run(bool on);

// Smallest q whose twiddle table takes three levels: two levels at q = 34
// need 4 MiB, as much as one XCD's L2, and the first pass of 2^34 complex64
// then read 1.46x its bytes from HBM (table misses); three levels at q >= 33
// take at most 144 KiB.
#ifndef EFFT_TW3_MIN_Q
#define EFFT_TW3_MIN_Q 33
#endif
constexpr int TW3_MIN_Q = EFFT_TW3_MIN_Q;

// LDS budget of one workgroup tile (one workgroup per CU on gfx950's 160 KB)
constexpr int TILE_LDS_BYTES = 143360;

// Points per thread of the strided layouts.  Setting EFFT_C64_COL_POINTS to
// 32 gives complex64 lines of 256 points or more half the threads; measured on
// gfx950 it was no faster (within 2%), and its second line set or prefetched
// tile spills registers, so the default is 16 everywhere.
#ifndef EFFT_C64_COL_POINTS
#define EFFT_C64_COL_POINTS 16
#endif
__host__ __device__ constexpr int col_points(int dtype_bytes, int logl)
{
    return (dtype_bytes == 8 && logl >= 8) ? EFFT_C64_COL_POINTS : 16;
}

// threads per line of L = 2^logl points at ep points per thread
__host__ __device__ constexpr int line_threads(int logl, int ep)
{
    return (1 << logl) >= ep ? (1 << logl) / ep : 1;
}

// Lines per workgroup set of the strided layouts when the tile is made as
// wide as the LDS budget and the thread budget (1024, or 512 at 32 points per
// thread) allow: each tile row is then one long contiguous run.  Shorter
// lines get wider tiles.
__host__ __device__ constexpr int col_lines_max(int dtype_bytes, int logl)
{
    const int l = 1 << logl;
    const int ep = col_points(dtype_bytes, logl);
    const int p = line_threads(logl, ep);
    const int padded = l + (l >> 4) + 2;
    int w = (ep == 32 ? 512 : 1024) / p;
    while (w > 1 && w * padded * dtype_bytes > TILE_LDS_BYTES) w >>= 1;
    if (w > 256) w = 256;
    return w;
}
// the narrow tile: one 128-byte segment per row
__host__ __device__ constexpr int col_lines_min(int dtype_bytes) { return dtype_bytes == 16 ? 8 : 16; }
// the narrow tile of a line length: lines of 2^11 and 2^12 points fill the
// LDS with fewer lines than one 128-byte segment
__host__ __device__ constexpr int col_lines_narrow(int dtype_bytes, int logl)
{
    return col_lines_min(dtype_bytes) < col_lines_max(dtype_bytes, logl) ? col_lines_min(dtype_bytes)
                                                                          : col_lines_max(dtype_bytes, logl);
}

// Longest strided line (log2) the kernels hold: 2^12 points, 4 complex64 or
// 2 complex128 lines per tile (32-byte tile rows).  The planner's own
// decompositions keep strided digits at 2^10 or less (wider tile rows); a
// caller-chosen decomposition may use up to 2^12.
constexpr int STRIDED_LOGL_MAX = 12;

// Measured on gfx950: a pass that reads and writes the same strided lines
// gains from long tile rows only at large strides (at a 2^24-element stride
// 512-byte rows ran 1.7x faster than 128-byte rows), while at small strides
// and for passes that write contiguous rows the narrow tile wins, because its
// smaller LDS footprint lets several workgroups share a CU.
constexpr int64_t WIDE_TILE_STRIDE = int64_t(1) << 17;

// Tile order of a strided pass (measured: the scattered order is 5-10%
// faster from a 2^17-element stride up, the plain XCD order below it)
inline int col_order(int64_t stride) { return stride >= WIDE_TILE_STRIDE ? TILE_XCD_SCATTER : TILE_XCD; }

// Stride of the scattered walk.  Measured on gfx950 over 7 .. 4099: strided
// passes whose tile rows are 256-byte runs (complex128 lines of 1024 points
// in two sets of 8, complex64 lines of 512 points 32 wide) run best at 127 -
// 129 tiles (2^30 complex128 in place, first pass 8.03 -> 7.78 ms; 2^34
// complex64, 81.3 -> 78.5 ms), while the transposing first pass of 2^32
// complex64 (512-byte rows) lost 17% there and keeps 1031.
// Strided passes with 512-byte tile rows (complex64 512-point lines in two
// sets of 32) keep 1031: at 2^34 in place, first pass, 129 gave 76.6-76.8 ms
// and 517 75.8 ms against 75.0-75.8 ms.
#ifndef EFFT_SCATTER_512
#define EFFT_SCATTER_512 1031
#endif
inline int64_t scatter_stride(int layout, int lines, int sets, int dtype_bytes)
{
    const bool col = layout == LAYOUT_COL || layout == LAYOUT_COL_POST;
    if (col && lines * sets * dtype_bytes == 256) return 129;
    if (col && lines * sets * dtype_bytes == 512) return EFFT_SCATTER_512;
    return 1031;
}

// Lines per workgroup for complex64 lines of 1024 points at a small stride:
// the 16-line tile fills the LDS, one workgroup per CU; an 8-line tile lets
// two share a CU, so one computes while the other streams (measured on
// gfx950, 2^30 complex64 in place: the stride-2^10 pass 3.92 -> 3.51 ms; the
// same change loses at large strides and for complex128 or shorter lines).
constexpr int C64_SHARED_LINES = 8;

// lines per workgroup of a strided pass (column_pass: a LAYOUT_COL pass,
// which reads and writes the same strided lines)
// Complex64 lines of 256 or 512 points take the widest tile (512- and
// 256-byte tile rows) at every stride that holds it, in every strided layout
// (1): measured on gfx950 by the tuner, 2^32 complex64 out of place 61.0 ->
// 58.1 ms (all four passes wider), 2^34 complex64 in place second pass
// 49.0 -> 48.3 ms.  (0): the wide tile only where lines are far apart.
#ifndef EFFT_C64_WIDE_SHORT
#define EFFT_C64_WIDE_SHORT 1
#endif

// Complex128 lines of 512 points written as rows (the transposing first pass
// of out-of-place plans whose first digit is 2^9): 16 lines (256-byte runs)
// from a 2^17-element stride, 8 below.  Measured on gfx950 (bitwise the same
// output): 2^26 out of place 0.474 -> 0.435 ms, 2^27 0.912 -> 0.846 ms, but
// 2^25 (stride 2^16) 0.215 -> 0.224 ms.
#ifndef EFFT_C128_WIDE_ROWS9
#define EFFT_C128_WIDE_ROWS9 1
#endif

inline int col_lines(int dtype_bytes, int logl, int64_t stride, bool same_positions, bool column_pass = false)
{
    const int w = col_lines_max(dtype_bytes, logl);
    if (EFFT_C64_WIDE_SHORT && dtype_bytes == 8 && (logl == 8 || logl == 9) && stride >= w) return w;
    if (same_positions && stride >= WIDE_TILE_STRIDE && stride >= w) return w;
    if (EFFT_C128_WIDE_ROWS9 && !same_positions && dtype_bytes == 16 && logl == 9 && stride >= WIDE_TILE_STRIDE)
        return w;
    if (column_pass && dtype_bytes == 8 && logl == 10 && stride >= C64_SHARED_LINES) return C64_SHARED_LINES;
    return col_lines_narrow(dtype_bytes, logl);
}

// Line sets per workgroup of LAYOUT_COL passes: where even the widest tile of
// 1024-point lines is a single 128-byte segment (8 complex128 or 16 complex64
// lines), a second set loaded together makes each tile row a 256-byte run at
// large strides.  The register file has room for it: 512 threads of 199
// VGPRs (complex128), 1024 threads of 122 (complex64).  At these strides
// every tile row is a separate address translation, so the longer runs also
// halve the translations per byte.
#ifndef EFFT_COL_SETS
#define EFFT_COL_SETS 2
#endif
#ifndef EFFT_C64_COL_SETS
#define EFFT_C64_COL_SETS 2
#endif
// Complex64 lines of 512 points: two sets of 32 lines (512-byte runs) at
// large strides (1), or one set of 32 (0).  Measured on gfx950, 2^34
// complex64 in place: first pass 79.1 -> 75.3 ms.
#ifndef EFFT_C64_SETS9
#define EFFT_C64_SETS9 1
#endif
// Complex64 lines of 256 points: two line sets at large strides (1), or one
// (0); col_set_lines below sets the lines per set.  Measured on gfx950 with
// sets of 64 lines (1 KiB runs): the last pass of 2^32 out of place (stride
// 2^24) 16.2 -> 15.0 ms, the second pass of 2^34 in place (stride 2^17) 51.0
// -> 49.2 ms.
#ifndef EFFT_C64_SETS8
#define EFFT_C64_SETS8 1
#endif
#ifndef EFFT_SETS_MIN_STRIDE
#define EFFT_SETS_MIN_STRIDE (int64_t(1) << 16)
#endif
inline int col_sets(int dtype_bytes, int logl, int lines, int64_t stride)
{
    if (lines != col_lines_max(dtype_bytes, logl) || stride < EFFT_SETS_MIN_STRIDE) return 1;
    if (logl == 9 && dtype_bytes == 8) return EFFT_C64_SETS9 ? 2 : 1;
    if (logl == 8 && dtype_bytes == 8) return EFFT_C64_SETS8 ? 2 : 1;
    const int want = dtype_bytes == 16 ? EFFT_COL_SETS : EFFT_C64_COL_SETS;
    return (want >= 2 && logl == 10 && lines * dtype_bytes == 128) ? 2 : 1;
}

// Lines per set of the widest strided tile of complex64 lines of 256 points
// (64 lines, 1024 threads, one workgroup per CU): half of them (512 threads)
// so that the LDS holds two workgroups per CU, for two-set tiles and for
// one-set tiles at strides from EFFT_C64_HALF_ONE_MIN_STRIDE.  Measured on
// gfx950 (bitwise the same output): two sets, 2^34 complex64 in place second
// pass (stride 2^17) 50.3 -> 47.6 ms, 2^32 out of place strided passes 13.93
// -> 13.57 and 14.96 -> 14.63 ms; one set, the 2^34 third pass (stride 2^9)
// 49.35 -> 47.12 ms, but the 2^32 out-of-place second pass (stride 2^8)
// 12.15 -> 12.51 ms.  Half-width tiles of 512-point lines (two sets of 16,
// 256-byte runs) lost at the 2^25 stride of the 2^34 first pass (75.7 -> 106
// ms), and a half-width transposing first pass gained nothing (2^32, 15.81 ->
// 15.76 ms).
#ifndef EFFT_C64_HALF_SETS8
#define EFFT_C64_HALF_SETS8 1
#endif
#ifndef EFFT_C64_HALF_ONE_MIN_STRIDE
#define EFFT_C64_HALF_ONE_MIN_STRIDE (int64_t(1) << 9)
#endif
inline int col_set_lines(int dtype_bytes, int logl, int lines, int sets, int64_t stride)
{
    if (dtype_bytes != 8 || logl != 8 || lines != col_lines_max(dtype_bytes, logl)) return lines;
    if (sets == 2) return EFFT_C64_HALF_SETS8 ? lines / 2 : lines;
    return stride >= EFFT_C64_HALF_ONE_MIN_STRIDE ? lines / 2 : lines;
}

// Non-temporal hints of a pass (measured on gfx950 at 2^30 points: they speed
// up the large-stride column passes by about 10%, the row passes by about 5%,
// and the stores of every pass; only the loads of small-stride column passes,
// whose tiles share cache lines with their neighbours, are better cached).
// The transposing first pass of complex64 tiles with 512-byte rows is faster
// with neither hint (2^32 out of place: 16.75 -> 15.81 ms; the complex128
// transposing pass loses without them, 2.23 -> 2.48 ms at 2^28).
#ifndef EFFT_NT_MODE
#define EFFT_NT_MODE 1  // 0: never, 1: as above, 2: always
#endif
inline void set_stream_hints(StageParams &sp, int layout, int lines, int dtype_bytes)
{
    sp.nt_store = EFFT_NT_MODE >= 1;
    sp.nt_load = EFFT_NT_MODE >= 2 || (EFFT_NT_MODE == 1 && !(layout == LAYOUT_COL && sp.s < WIDE_TILE_STRIDE));
    if (EFFT_NT_MODE == 1 && layout == LAYOUT_COL2ROW && dtype_bytes == 8 && lines * dtype_bytes >= 512)
        sp.nt_load = sp.nt_store = 0;
}
#ifndef EFFT_NT_SWAP
#define EFFT_NT_SWAP 1
#endif

// lines per workgroup of the row layout for a given line length
int row_lines(int dtype_bytes, int logl, int64_t nlines);

// threads per line
inline int threads_per_line(int logl) { return logl >= 4 ? (1 << (logl - 4)) : 1; }

}  // namespace efft
