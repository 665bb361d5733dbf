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
    LAYOUT_COL2ROW = 2  // strided lines read as LAYOUT_COL, each written back
                        // as a contiguous row at a digit-reversed row index
};

// Twiddle applied to output k of line (block b, offset o) of a pass.
enum TwMode : int {
    TW_NONE = 0,
    TW_OFFSET = 1,   // W_N^(o * k * scale)
    TW_REVBLOCK = 2  // W_N^(rev(b) * k * scale), rev = digit reversal of b
};

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
    int64_t ntiles;      // workgroups in the grid
    uint64_t n_over_l;   // N / L, scales the in-line Stockham twiddles
    uint64_t tw_scale;   // see TwMode
    int64_t row_mul;     // LAYOUT_COL2ROW: line o's row starts at row_mul * rev(o)
    Digits rev;          // digits of o (COL2ROW) or of blk (TW_REVBLOCK)
    TwTable tt;
    double scale;        // multiplies every output when apply_scale is set
    int twmode;
    int conj;            // 1: backward direction (conjugate on load and store)
    int apply_scale;
};

// Tiled in-place digit reversal of a [R][M][R] array: element (a, mu, b)
// swaps with (b, rev(mu), a).
struct SwapParams {
    void *data;
    int64_t R;     // outer digit size (first and last digit)
    int64_t M;     // product of the middle digits (1 if none)
    int64_t nt;    // R / tile
    Digits mid;    // middle digits, lowest first
};

// kernel launchers (efft_kernels.hip); return hipSuccess or the launch error
hipError_t launch_stage(int dtype_bytes, int layout, int logl, int lines, const StageParams &p,
                        hipStream_t stream);
hipError_t launch_swap(int dtype_bytes, const SwapParams &p, hipStream_t stream);
hipError_t launch_twiddle_table(double2 *lo, int64_t n_lo, double2 *hi, int64_t n_hi, int h,
                                int q, hipStream_t stream);

// lines per workgroup of the column layouts: one 128-byte row segment
inline int col_lines(int dtype_bytes) { return dtype_bytes == 16 ? 8 : 16; }

// lines per workgroup of the row layout for a given line length
int row_lines(int dtype_bytes, int logl, int64_t nlines);

// threads per line
inline int threads_per_line(int logl) { return logl >= 4 ? (1 << (logl - 4)) : 1; }

}  // namespace efft
