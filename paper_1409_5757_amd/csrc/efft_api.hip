// efft_api.hip -- planner, executor and C ABI (include/efft.h).
//
// Decomposition.  N = 2^q is split into digits N = R_1 * ... * R_m, R_1 the
// digit of the slowest-varying input index.  Each pass transforms one digit
// with batched L = R_j point sub-FFTs (a multi-radix generalisation of the
// radix-2 split of Section 2.2, Eqs. "eqct"/"eqctt"; the paper's
// scatter -> bin DFTs -> reassembly stages of Section 2.3 are the same
// factorisation with R = 2 reassembly levels).
//
// In place (decimation in frequency): pass j works inside blocks of
// B_j = R_j...R_m points on lines of stride s_j = R_{j+1}...R_m, multiplying
// output k_j of line o by W_{B_j}^{o*k_j}.  The result is in digit-reversed
// order; the digits are chosen palindromic (R_j = R_{m+1-j}) so that the
// reversal is an involution, done in place by one pass that swaps tile pairs
// (the read-set = write-set idea of the paper's pair reassembly, Section 3.4).
//
// Out of place: the first pass reads x along the slowest digit and writes
// each transformed line as a contiguous row of `out` at a digit-reversed row
// index; later passes then work in place on `out` along strided columns and
// leave natural order, so no reordering pass is needed.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <unordered_set>
#include <vector>

#include "../../include/efft.h"
#include "efft_internal.hpp"

using namespace efft;

namespace {

constexpr uint64_t PLAN_MAGIC = 0x45464654504c414eULL;  // "EFFTPLAN"
constexpr int MAX_DIGITS = 6;

// which array a pass reads or writes
enum Buf { BUF_IN = 0, BUF_OUT = 1, BUF_SCRATCH = 2 };

struct Pass {
    bool swap;
    int src, dst;  // Buf
    int layout, logl, lines, sets;
    StageParams sp;  // src/dst filled at exec time
    SwapParams wp;   // data filled at exec time
};

thread_local int g_last_error = EFFT_OK;
std::mutex g_reg_mu;
std::unordered_set<const void *> g_registry;

bool registered(const void *p)
{
    std::lock_guard<std::mutex> lk(g_reg_mu);
    return g_registry.count(p) != 0;
}

// largest line (log2) per layout: strided lines are limited by LDS for a
// W-line tile, contiguous lines by LDS for one line
int col_max(int dtype_bytes) { return dtype_bytes == 16 ? 10 : 10; }
// largest strided digit of a caller-chosen decomposition
int col_max_digits(int dtype_bytes)
{
    (void)dtype_bytes;
    return STRIDED_LOGL_MAX;
}
int row_max(int dtype_bytes) { return dtype_bytes == 16 ? 12 : 12; }

int log2_exact(int64_t n)
{
    if (n <= 0 || (n & (n - 1)) != 0) return -1;
    int q = 0;
    while ((int64_t(1) << q) < n) ++q;
    return q;
}

// Balanced palindromic digits for the in-place plan.
int plan_digits_inplace(int q, int eb, int *d)
{
    if (q <= row_max(eb)) {
        d[0] = q;
        return 1;
    }
    const int cm = col_max(eb);
    for (int m = 2; m <= MAX_DIGITS; ++m) {
        const int half = m / 2, center = m % 2;
        // search all palindromes of this length; keep the one with the
        // smallest largest digit, ties to the larger outer digit
        int best_max = 1 << 30, best[MAX_DIGITS] = {0};
        bool found = false;
        int dig[MAX_DIGITS];
        // enumerate the first `half` digits and the center in [4, cm]: every
        // strided pass then has lines of at least 16 points and a stride of at
        // least 16 lines
        int total = 1;
        for (int i = 0; i < half; ++i) total *= (cm - 3);
        for (int idx = 0; idx < total; ++idx) {
            int rem = idx, sum = 0;
            for (int i = 0; i < half; ++i) {
                dig[i] = 4 + rem % (cm - 3);
                rem /= (cm - 3);
                dig[m - 1 - i] = dig[i];
                sum += 2 * dig[i];
            }
            if (center) {
                const int c = q - sum;
                if (c < 4 || c > cm) continue;
                dig[half] = c;
            } else if (sum != q) {
                continue;
            }
            int mx = 0;
            for (int i = 0; i < m; ++i) mx = dig[i] > mx ? dig[i] : mx;
            if (mx < best_max || (mx == best_max && dig[0] > best[0])) {
                best_max = mx;
                for (int i = 0; i < m; ++i) best[i] = dig[i];
                found = true;
            }
        }
        if (found) {
            for (int i = 0; i < m; ++i) d[i] = best[i];
            return m;
        }
    }
    return -1;
}

// Balanced digits for the out-of-place plan (every digit >= 4 when m > 1).
int plan_digits_oop(int q, int eb, int *d)
{
    if (q <= row_max(eb)) {
        d[0] = q;
        return 1;
    }
    const int cm = col_max(eb);
    int m = (q + cm - 1) / cm;
    if (m < 2) m = 2;
    if (m > MAX_DIGITS) return -1;
    for (int i = 0; i < m; ++i) d[i] = q / m + (i < q % m ? 1 : 0);
    return m;
}

int plan_digits(int q, int eb, int inplace, int *d)
{
    return inplace ? plan_digits_inplace(q, eb, d) : plan_digits_oop(q, eb, d);
}

int dtype_bytes(int dtype) { return dtype == EFFT_C128 ? 16 : dtype == EFFT_C64 ? 8 : 0; }

}  // namespace

enum PlanKind { KIND_C2C = 0, KIND_R2C = 1, KIND_C2R = 2, KIND_CHIRP = 3, KIND_MIXED = 4 };

struct efft_plan_s {
    uint64_t magic;
    int64_t n;
    int64_t batch;  // contiguous signals of n points per execution
    int q, dtype, dir, inplace, eb;
    int m;
    int digits[MAX_DIGITS];
    std::vector<Pass> passes;
    // in-place plans: the same transform with a caller-provided scratch array
    // of N elements, one pass shorter (empty when that gains nothing)
    std::vector<Pass> scratch_passes;
    double scale;
    double2 *tables;
    int64_t table_bytes;
    // real-input plans: an N/2-point complex plan plus the pairing pass, which
    // uses W_N^k from this plan's own table (tt_real)
    int kind;
    efft_plan_s *inner;
    TwTable tt_real;
    // lengths that are not powers of two (KIND_CHIRP): the chirp a_j (FP64),
    // the transformed kernel V = DFT_M(v)/M and a work array of M points, with
    // forward (inner) and backward (inner2) in-place M-point plans
    int64_t m_pad;
    efft_plan_s *inner2;
    double2 *chirp;
    void *vhat, *work, *work2;  // work2: second work array of out-of-place inner plans
    // out-of-place inner plans: their passes with the premultiplication by the
    // chirp (forward) and the product with V (backward) done by the first
    // pass as it loads, so neither takes a pass of its own
    std::vector<Pass> chirp_fwd, chirp_bwd;
    bool chirp_post;  // chirp_bwd's last pass also post-multiplies into the output
    // N = M * 2^s with a small odd M (KIND_MIXED): tables (W_M, lo, hi of W_N)
    // in `tables`, rows of 2^s points transformed by `inner` (batch M), work
    int m_odd, h_mixed;
    int64_t cols;
    // the rows' scratch schedule run in place on `work`, its last pass writing
    // the rows interleaved into the output (natural order, times scale); empty
    // when the rows take one pass (then a reorder pass follows them)
    std::vector<Pass> mixed_passes;
    int device;  // HIP device current when the plan was made (its tables live there)
};

namespace {

StageParams base_params(const efft_plan_s *p, const TwTable &tt)
{
    StageParams sp{};
    sp.tt = tt;
    sp.conj = p->dir == EFFT_BACKWARD ? 1 : 0;
    sp.twmode = TW_NONE;
    sp.rev.nd = 0;
    sp.scale = 1.0;
    sp.apply_scale = 0;
    sp.order = TILE_XCD;
    sp.ilv = 1;
    return sp;
}

void build_passes_unscaled(efft_plan_s *p, const TwTable &tt);

// The output scale is applied by the last sub-FFT pass (a trailing
// digit-reversal pass only permutes).
void build_scratch_passes(efft_plan_s *p, const TwTable &tt);

void apply_scale_to_last(std::vector<Pass> &v, double scale)
{
    if (scale == 1.0) return;
    for (size_t i = v.size(); i-- > 0;) {
        if (!v[i].swap) {
            v[i].sp.apply_scale = 1;
            v[i].sp.scale = scale;
            return;
        }
    }
}

void set_hints(std::vector<Pass> &v, int eb)
{
    for (Pass &ps : v) {
        if (ps.swap)
            ps.wp.nt_hint = EFFT_NT_SWAP;
        else
            set_stream_hints(ps.sp, ps.layout, ps.lines * ps.sets, eb);
    }
}

// A strided single-set pass whose grid has fewer workgroups than the device
// has CUs leaves CUs idle (2^20 points: 128 tiles of 8 complex128 lines for
// 256 CUs): halve its lines while the grid is that small and a kernel for the
// narrower tile exists.  Measured on 2^20 complex128 out of place: 0.042 ms
// -> 0.038 ms with 256; thresholds of 512 and 1024 (tiles of 2 lines) were
// slower than 256 (0.040 ms), and 2^22 and complex64 at 2^20 did not change.
#ifndef EFFT_SMALL_GRID_TILES
#define EFFT_SMALL_GRID_TILES 256
#endif
int64_t tiles_for(const efft_plan_s *p, const Pass &ps, int lines, int sets);
void narrow_small_grids(const efft_plan_s *p, std::vector<Pass> &v)
{
    for (Pass &ps : v) {
        if (ps.swap || ps.sets != 1 || (ps.layout != LAYOUT_COL && ps.layout != LAYOUT_COL2ROW)) continue;
        while (ps.sp.ntiles < EFFT_SMALL_GRID_TILES && ps.lines > 2) {
            Pass q = ps;
            q.lines = ps.lines / 2;
            q.sp.ntiles = tiles_for(p, q, q.lines, 1);
            if (q.sp.ntiles < 0) break;
            set_dry_run(true);
            const hipError_t e = launch_stage(p->eb, q.layout, q.logl, q.lines, 1, q.sp, nullptr);
            set_dry_run(false);
            if (e != hipSuccess) break;
            ps = q;
        }
    }
}

// A pass copied from plan `p` whose layout was changed afterwards (the chirp
// path's fused first and last passes) may have been narrowed for a layout
// with more tile widths: double its lines until a kernel for the new layout
// exists.  False if none does.
bool widen_to_kernel(const efft_plan_s *p, Pass &ps)
{
    for (;;) {
        set_dry_run(true);
        const hipError_t e = launch_stage(p->eb, ps.layout, ps.logl, ps.lines, ps.sets, ps.sp, nullptr);
        set_dry_run(false);
        if (e == hipSuccess) return true;
        const int64_t nt = tiles_for(p, ps, ps.lines * 2, ps.sets);
        if (nt < 0) return false;
        ps.lines *= 2;
        ps.sp.ntiles = nt;
    }
}

void build_passes(efft_plan_s *p, const TwTable &tt)
{
    build_passes_unscaled(p, tt);
    // the first pass reads the input; every later pass works in place on out
    for (size_t i = 0; i < p->passes.size(); ++i) {
        p->passes[i].src = i == 0 ? BUF_IN : BUF_OUT;
        p->passes[i].dst = BUF_OUT;
    }
    apply_scale_to_last(p->passes, p->scale);
    p->scratch_passes.clear();
    if (p->inplace && p->m >= 2) {
        build_scratch_passes(p, tt);
        apply_scale_to_last(p->scratch_passes, p->scale);
    }
    // a batch of contiguous signals: every sub-FFT pass's lines simply
    // continue into the next signal (blocks of the same structure), so only
    // the tile count grows; the swap runs one grid layer per signal
    for (std::vector<Pass> *v : {&p->passes, &p->scratch_passes}) {
        for (Pass &ps : *v) {
            if (ps.swap)
                ps.wp.n = p->n;
            else
                ps.sp.ntiles *= p->batch;
        }
        narrow_small_grids(p, *v);
    }
    set_hints(p->passes, p->eb);
    set_hints(p->scratch_passes, p->eb);
}

// Scratch schedule of an in-place plan: the sub-FFT passes of digits
// 1 .. m-1 run as in the in-place schedule, the first from the data into the
// scratch array and the others in place on it; the last digit's pass reads
// contiguous rows of the scratch array and writes each transformed row as a
// column of the data array at its natural position, so no digit-reversal
// pass is needed.
void build_scratch_passes(efft_plan_s *p, const TwTable &tt)
{
    const int m = p->m;
    for (int j = 0; j + 1 < m; ++j) {
        Pass ps = p->passes[size_t(j)];
        ps.src = j == 0 ? BUF_IN : BUF_SCRATCH;
        ps.dst = BUF_SCRATCH;
        p->scratch_passes.push_back(ps);
    }
    const int64_t n = p->n;
    const int dl = p->digits[m - 1];
    const int64_t L = int64_t(1) << dl;
    Pass ps{};
    ps.swap = false;
    ps.src = BUF_SCRATCH;
    ps.dst = BUF_OUT;
    ps.logl = dl;
    ps.layout = LAYOUT_ROW2COL;
    ps.lines = col_lines(p->eb, dl, n / L, true);
    ps.sets = 1;
    ps.sp = base_params(p, tt);
    ps.sp.s = 1;
    ps.sp.B = L;
    ps.sp.n_over_l = uint64_t(n / L);
    ps.sp.row_mul = n / L;
    ps.sp.rev.nd = 0;
    for (int i = 0; i + 1 < m; ++i) ps.sp.rev.bits[ps.sp.rev.nd++] = p->digits[i];  // k_1 lowest
    ps.sp.order = col_order(n / L);
    ps.sp.ntiles = (n / L) / ps.lines;
    p->scratch_passes.push_back(ps);
}

void build_passes_unscaled(efft_plan_s *p, const TwTable &tt)
{
    const int64_t n = p->n;
    const int m = p->m;
    const int *d = p->digits;
    p->passes.clear();
    if (p->inplace) {
        for (int j = 0; j < m; ++j) {
            Pass ps{};
            ps.swap = false;
            ps.logl = d[j];
            const int64_t L = int64_t(1) << d[j];
            int64_t s = 1;
            for (int i = j + 1; i < m; ++i) s <<= d[i];
            ps.sp = base_params(p, tt);
            ps.sp.s = s;
            ps.sp.B = s * L;
            ps.sp.n_over_l = uint64_t(n / L);
            ps.sets = 1;
            if (s == 1) {
                ps.layout = LAYOUT_ROW;
                ps.lines = row_lines(p->eb, d[j], n / L);
            } else {
                ps.layout = LAYOUT_COL;
                ps.lines = col_lines(p->eb, d[j], s, true, true);
                ps.sets = col_sets(p->eb, d[j], ps.lines, s);
                ps.lines = col_set_lines(p->eb, d[j], ps.lines, ps.sets, s);
                ps.sp.order = col_order(s);
                ps.sp.twmode = TW_OFFSET;
                ps.sp.tw_scale = uint64_t(n / (s * L));
            }
            ps.sp.ntiles = (n / L) / (ps.lines * ps.sets);
            p->passes.push_back(ps);
        }
        if (m >= 2) {
            Pass ps{};
            ps.swap = true;
            ps.wp.R = int64_t(1) << d[0];
            int64_t M = 1;
            ps.wp.mid.nd = 0;
            for (int i = m - 2; i >= 1; --i) {  // lowest digit first
                ps.wp.mid.bits[ps.wp.mid.nd++] = d[i];
                M <<= d[i];
            }
            ps.wp.M = M;
            const int64_t ts = swap_tile(p->eb, ps.wp.R);
            ps.wp.nt = ps.wp.R / ts;
            p->passes.push_back(ps);
        }
        return;
    }
    // out of place
    if (m == 1) {
        Pass ps{};
        ps.swap = false;
        ps.logl = d[0];
        ps.layout = LAYOUT_ROW;
        ps.lines = row_lines(p->eb, d[0], 1);
        ps.sets = 1;
        ps.sp = base_params(p, tt);
        ps.sp.s = 1;
        ps.sp.B = n;
        ps.sp.n_over_l = 1;
        ps.sp.ntiles = 1;
        p->passes.push_back(ps);
        return;
    }
    {  // first pass: lines along digit 1, rows written at R_1 * rev(o)
        Pass ps{};
        ps.swap = false;
        ps.logl = d[0];
        ps.layout = LAYOUT_COL2ROW;
        ps.lines = col_lines(p->eb, d[0], n >> d[0], false);
        ps.sets = 1;
        const int64_t L = int64_t(1) << d[0];
        ps.sp = base_params(p, tt);
        ps.sp.s = n / L;
        ps.sp.B = n;
        ps.sp.n_over_l = uint64_t(n / L);
        ps.sp.tw_scale = 1;
        ps.sp.row_mul = L;
        ps.sp.order = col_order(n / L);
        ps.sp.rev.nd = 0;
        for (int i = m - 1; i >= 1; --i) ps.sp.rev.bits[ps.sp.rev.nd++] = d[i];  // o = n_m + R_m n_{m-1} + ...
        ps.sp.ntiles = (n / L) / ps.lines;
        p->passes.push_back(ps);
    }
    int64_t C = int64_t(1) << d[0];
    for (int j = 1; j < m; ++j) {
        Pass ps{};
        ps.swap = false;
        ps.logl = d[j];
        ps.layout = LAYOUT_COL;
        ps.lines = col_lines(p->eb, d[j], C, true, true);
        ps.sets = col_sets(p->eb, d[j], ps.lines, C);
        ps.lines = col_set_lines(p->eb, d[j], ps.lines, ps.sets, C);
        const int64_t L = int64_t(1) << d[j];
        ps.sp = base_params(p, tt);
        ps.sp.order = col_order(C);
        ps.sp.s = C;
        ps.sp.B = C * L;
        ps.sp.n_over_l = uint64_t(n / L);
        if (j + 1 < m) {
            ps.sp.twmode = TW_REVBLOCK;
            ps.sp.tw_scale = uint64_t(C);
            ps.sp.rev.nd = 0;
            for (int i = j + 1; i < m; ++i) ps.sp.rev.bits[ps.sp.rev.nd++] = d[i];  // H = n_{j+1} + ...
        }
        ps.sp.ntiles = (n / L) / (ps.lines * ps.sets);
        p->passes.push_back(ps);
        C *= L;
    }
}

int validate_ptr(const efft_plan_s *p, const void *ptr)
{
    if (!ptr) return EFFT_ERR_NULLPTR;
    if (reinterpret_cast<uintptr_t>(ptr) % uintptr_t(p->eb) != 0) return EFFT_ERR_ALIGN;
    return EFFT_OK;
}

int run_c2c(const efft_plan_s *p, const void *in, void *out, hipStream_t stream, void **events,
            int nevents);
int run_passes(const std::vector<Pass> &passes, int64_t batch, int eb, const void *in, void *out,
               void *scratch, hipStream_t stream, void **events, int nevents);

int total_passes(const efft_plan_s *p)
{
    if (p->kind == KIND_C2C) return int(p->passes.size());
    if (p->kind == KIND_CHIRP)  // (premul,) M-point forward, (product,) M-point backward, postmul
        return int(p->inner->passes.size()) + int(p->inner2->passes.size()) +
               (p->chirp_fwd.empty() ? 3 : p->chirp_post ? 0 : 1);
    if (p->kind == KIND_MIXED)  // radix-M pass, the rows' passes (and a reorder)
        return p->mixed_passes.empty() ? int(p->inner->passes.size()) + 2 : int(p->mixed_passes.size()) + 1;
    return int(p->inner->passes.size()) + 1;
}

// N = M * 2^s: radix-M pass into the work array, then the batched 2^s-point
// rows in place on it; the rows' last pass writes them interleaved into the
// output in natural order (times scale), or, for rows of one pass, a reorder
// pass does.
int run_mixed(const efft_plan_s *p, const void *in, void *out, hipStream_t stream, void **events, int nevents)
{
    const int np = total_passes(p);
    if (events && nevents < np + 1) return EFFT_ERR_ARG;
    auto rec = [&](int i) {
        return !events || hipEventRecord(static_cast<hipEvent_t>(events[i]), stream) == hipSuccess;
    };
    const int64_t n_lo = int64_t(1) << p->h_mixed;
    const double2 *wm = p->tables, *lo = p->tables + p->m_odd, *hi = lo + n_lo;
    if (!rec(0) || launch_radix_m(p->eb, p->m_odd, in, p->work, wm, lo, hi, p->h_mixed, p->cols, p->batch,
                                  p->dir == EFFT_BACKWARD ? 1 : 0, stream) != hipSuccess)
        return EFFT_ERR_HIP;
    if (!p->mixed_passes.empty())  // in = scratch = work: the rows' passes in place, the last into out
        return run_passes(p->mixed_passes, p->inner->batch, p->eb, p->work, out, p->work, stream,
                          events ? events + 1 : nullptr, events ? np : 0);
    const int ni = int(p->inner->passes.size());
    const int r = run_c2c(p->inner, p->work, p->work, stream, events ? events + 1 : nullptr, events ? ni + 1 : 0);
    if (r != EFFT_OK) return r;
    if (!rec(ni + 1) ||
        launch_reorder_m(p->eb, p->m_odd, p->work, out, p->cols, p->batch, p->scale, stream) != hipSuccess)
        return EFFT_ERR_HIP;
    return rec(np) ? EFFT_OK : EFFT_ERR_HIP;
}

// Chirp plan: per signal, w = (x a) zero-padded; w = DFT_M(w); w *= V;
// w = DFT_M^-(w) (the 1/M is in V); out = scale * a * w[0 .. N).  With
// out-of-place M-point plans the first two products happen in the first
// pass of each transform, as it loads, and the last in the last pass of the
// backward transform, as it stores.
int run_chirp(const efft_plan_s *p, const void *in, void *out, hipStream_t stream, void **events, int nevents)
{
    const int np = total_passes(p);
    if (events && (nevents < np + 1 || p->batch != 1)) return EFFT_ERR_ARG;
    auto rec = [&](int i) {
        return !events || hipEventRecord(static_cast<hipEvent_t>(events[i]), stream) == hipSuccess;
    };
    const int nf = int(p->inner->passes.size()), nb = int(p->inner2->passes.size());
    for (int64_t b = 0; b < p->batch; ++b) {
        const char *x = static_cast<const char *>(in) + b * p->n * p->eb;
        char *y = static_cast<char *>(out) + b * p->n * p->eb;
        if (!p->chirp_fwd.empty()) {
            // x -> work2 (premultiplied and zero-padded as loaded), work2 ->
            // work (times V as loaded; the last pass post-multiplies straight
            // into y, else a post-multiply pass follows)
            int r = run_passes(p->chirp_fwd, 1, p->eb, x, p->work2, nullptr, stream, events, events ? nf + 1 : 0);
            if (r != EFFT_OK) return r;
            std::vector<Pass> bwd = p->chirp_bwd;
            if (p->chirp_post) bwd.back().sp.post_out = y;
            r = run_passes(bwd, 1, p->eb, p->work2, p->work, nullptr, stream, events ? events + nf : nullptr,
                           events ? nb + 1 : 0);
            if (r != EFFT_OK) return r;
            if (!p->chirp_post &&
                (launch_postmul(p->eb, p->work, y, p->chirp, p->n, p->scale, stream) != hipSuccess || !rec(np)))
                return EFFT_ERR_HIP;
            continue;
        }
        if (!rec(0) || launch_premul(p->eb, x, p->work, p->chirp, p->n, p->m_pad, stream) != hipSuccess)
            return EFFT_ERR_HIP;
        // out-of-place inner plans (when the device has room): work -> work2 -> work
        void *mid = p->work2 ? p->work2 : p->work;
        int r = run_c2c(p->inner, p->work, mid, stream, events ? events + 1 : nullptr, events ? nf + 1 : 0);
        if (r != EFFT_OK) return r;
        if (!rec(nf + 1) || launch_pointwise(p->eb, mid, p->vhat, p->m_pad, stream) != hipSuccess)
            return EFFT_ERR_HIP;
        r = run_c2c(p->inner2, mid, p->work, stream, events ? events + nf + 2 : nullptr, events ? nb + 1 : 0);
        if (r != EFFT_OK) return r;
        if (!rec(nf + nb + 2) || launch_postmul(p->eb, p->work, y, p->chirp, p->n, p->scale, stream) != hipSuccess)
            return EFFT_ERR_HIP;
        if (!rec(np)) return EFFT_ERR_HIP;
    }
    return EFFT_OK;
}

int run(const efft_plan_s *p, const void *in, void *out, hipStream_t stream, void **events,
        int nevents)
{
    if (p->kind == KIND_C2C) return run_c2c(p, in, out, stream, events, nevents);
    if (p->kind == KIND_CHIRP) return run_chirp(p, in, out, stream, events, nevents);
    if (p->kind == KIND_MIXED) return run_mixed(p, in, out, stream, events, nevents);
    const int np = total_passes(p);
    if (events && nevents < np + 1) return EFFT_ERR_ARG;
    const int64_t h = p->n / 2;
    if (p->kind == KIND_R2C) {
        // the N reals are read as N/2 complex points; out[0 .. N/2) receives
        // their transform, then the pairing pass completes out[0 .. N/2]
        const int r = run_c2c(p->inner, in, out, stream, events, events ? nevents - 1 : 0);
        if (r != EFFT_OK) return r;
        if (launch_r2c_post(p->eb, out, h, p->tt_real, p->scale, p->scale != 1.0 ? 1 : 0, stream) != hipSuccess)
            return EFFT_ERR_HIP;
        if (events && hipEventRecord(static_cast<hipEvent_t>(events[np]), stream) != hipSuccess)
            return EFFT_ERR_HIP;
        return EFFT_OK;
    }
    // C2R: pairing pass from in[0 .. N/2] into out[0 .. N/2), then the
    // in-place backward N/2-point transform of out
    if (events && hipEventRecord(static_cast<hipEvent_t>(events[0]), stream) != hipSuccess) return EFFT_ERR_HIP;
    if (launch_c2r_pre(p->eb, in, out, h, p->tt_real, stream) != hipSuccess) return EFFT_ERR_HIP;
    return run_c2c(p->inner, out, out, stream, events ? events + 1 : nullptr, events ? nevents - 1 : 0);
}

int run_passes(const std::vector<Pass> &passes, int64_t batch, int eb, const void *in, void *out,
               void *scratch, hipStream_t stream, void **events, int nevents)
{
    if (events && nevents < int(passes.size()) + 1) return EFFT_ERR_ARG;
    for (size_t i = 0; i < passes.size(); ++i) {
        Pass ps = passes[i];
        if (events && hipEventRecord(static_cast<hipEvent_t>(events[i]), stream) != hipSuccess)
            return EFFT_ERR_HIP;
        void *bufs[3] = {const_cast<void *>(in), out, scratch};
        hipError_t e;
        if (ps.swap) {
            ps.wp.data = bufs[ps.dst];
            e = launch_swap(eb, ps.wp, batch, stream);
        } else {
            ps.sp.src = bufs[ps.src];
            ps.sp.dst = bufs[ps.dst];
            ps.sp.scatter = scatter_stride(ps.layout, ps.lines, ps.sets, eb);
            ps.sp.off32 = EFFT_WAVE_UNIFORM && wave_offset_fits(ps.layout, ps.lines, ps.sp.s, eb) ? 1 : 0;
            e = launch_stage(eb, ps.layout, ps.logl, ps.lines, ps.sets, ps.sp, stream);
        }
        if (e != hipSuccess) return EFFT_ERR_HIP;
    }
    if (events && hipEventRecord(static_cast<hipEvent_t>(events[passes.size()]), stream) != hipSuccess)
        return EFFT_ERR_HIP;
    return EFFT_OK;
}

int run_c2c(const efft_plan_s *p, const void *in, void *out, hipStream_t stream, void **events,
            int nevents)
{
    return run_passes(p->passes, p->batch, p->eb, in, out, nullptr, stream, events, nevents);
}

const efft_plan_s *live(const efft_plan_t *plan)
{
    if (!plan || !registered(plan)) return nullptr;
    return plan->magic == PLAN_MAGIC ? plan : nullptr;
}

// largest length that is not a power of two: its padded length 2^ceil(log2(2n-1))
// is at most 2^EFFT_MAX_LOG2N
constexpr int64_t MAX_CHIRP_N = (int64_t(1) << (EFFT_MAX_LOG2N - 1));

int validate_args(int q, int dtype, int dir, double scale)
{
    if (q < 0 || q > EFFT_MAX_LOG2N) return EFFT_ERR_SIZE;
    if (!dtype_bytes(dtype)) return EFFT_ERR_DTYPE;
    if (dir != EFFT_FORWARD && dir != EFFT_BACKWARD) return EFFT_ERR_DIR;
    if (!(scale == scale) || scale == 0.0 || scale - scale != 0.0) return EFFT_ERR_ARG;  // NaN, 0, inf
    return EFFT_OK;
}

// A private non-blocking stream for the kernels that build a plan's tables:
// plan creation waits for them without synchronising the whole device, so
// work on the caller's other streams keeps running.
struct SetupStream {
    hipStream_t s = nullptr;
    bool ok;
    SetupStream() { ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess; }
    ~SetupStream()
    {
        if (s) (void)hipStreamDestroy(s);
    }
    // wait for everything enqueued; false if creation, a launch or the wait failed
    bool finish(bool launched)
    {
        const bool done = ok && hipStreamSynchronize(s) == hipSuccess;
        if (!(done && launched)) (void)hipGetLastError();
        return done && launched;
    }
};

// FP64 table of W_N^m for N = 2^q on the current device: two levels,
// lo[2^h] and hi[2^(q-h)] with h = ceil(q/2) (and mid = {1}), or from
// q = TW3_MIN_Q on three, lo[2^h], mid[2^h] and hi[2^(q-2h)] with
// h = ceil(q/3) (see TwTable).
// Built on a stream of the library's own, which the call waits for (the
// tables must be complete before the plan is returned), so that other streams
// of the device keep running.
int make_tables(efft_plan_s *p, int q, TwTable *tt)
{
    const bool three = q >= TW3_MIN_Q;
    const int h = three ? (q + 2) / 3 : (q + 1) / 2;
    const int64_t n_lo = int64_t(1) << h;
    const int64_t n_mid = three ? n_lo : 1;  // two levels: mid = {1}
    const int64_t n_hi = int64_t(1) << (q - (three ? 2 * h : h));
    // the FP32 line table (LINE_TW_N float2) follows the FP64 tables
    p->table_bytes = (n_lo + n_mid + n_hi) * int64_t(sizeof(double2)) + LINE_TW_N * int64_t(sizeof(float2));
    if (hipMalloc(reinterpret_cast<void **>(&p->tables), size_t(p->table_bytes)) != hipSuccess) {
        (void)hipGetLastError();
        p->tables = nullptr;
        return EFFT_ERR_ALLOC;
    }
    double2 *lo = p->tables, *mid = lo + n_lo, *hi = mid + n_mid;
    float2 *line32 = reinterpret_cast<float2 *>(hi + n_hi);
    SetupStream ss;
    // lo[j] = W^j and mid[j] = W^(j 2^h) (or hi[j] = W^(j 2^h) for two levels);
    // for three levels then hi[j] = W^(j 2^(2h)); for two, mid[0] = W^0 = 1
    bool launched = ss.ok &&
                    launch_twiddle_table(lo, n_lo, three ? mid : hi, three ? n_mid : n_hi, h, q, ss.s) == hipSuccess;
    if (launched)
        launched = (three ? launch_twiddle_table(nullptr, 0, hi, n_hi, 2 * h, q, ss.s)
                          : launch_twiddle_table(mid, 1, nullptr, 0, h, q, ss.s)) == hipSuccess;
    if (launched) launched = launch_line32_table(line32, ss.s) == hipSuccess;
    if (!ss.finish(launched)) {
        (void)hipFree(p->tables);
        p->tables = nullptr;
        return EFFT_ERR_HIP;
    }
    tt->lo = lo;
    tt->hi = hi;
    tt->mid = mid;
    tt->h = h;
    tt->h2 = three ? 2 * h : h;
    tt->mask_n = (uint64_t(1) << q) - 1u;
    tt->mask_lo = uint64_t(n_lo) - 1u;
    tt->mask_mid = three ? uint64_t(n_lo) - 1u : 0;
    tt->line32 = line32;
    return EFFT_OK;
}

// every pass of the plan's schedules has a kernel (host-side dry run)
bool kernels_exist(const efft_plan_s *p)
{
    set_dry_run(true);
    bool ok = true;
    for (const std::vector<Pass> *v : {&p->passes, &p->scratch_passes}) {
        for (const Pass &ps : *v) {
            const hipError_t e = ps.swap ? launch_swap(p->eb, ps.wp, 1, nullptr)
                                         : launch_stage(p->eb, ps.layout, ps.logl, ps.lines, ps.sets, ps.sp, nullptr);
            if (e != hipSuccess) ok = false;
        }
    }
    set_dry_run(false);
    return ok;
}

// A caller-chosen decomposition: log2 digits summing to q, each strided
// digit within the strided kernels' range [4, STRIDED_LOGL_MAX], a one-digit plan
// within the row kernels' range, and palindromic for an in-place plan (the
// digit-reversal swap needs it).
bool digits_usable(int q, int eb, int inplace, const int *d, int m)
{
    if (m < 1 || m > MAX_DIGITS) return false;
    int sum = 0;
    for (int i = 0; i < m; ++i) sum += d[i];
    if (sum != q) return false;
    if (m == 1) return q <= row_max(eb);
    for (int i = 0; i < m; ++i) {
        if (d[i] < 4 || d[i] > col_max_digits(eb)) return false;
        if (inplace && d[i] != d[m - 1 - i]) return false;
    }
    return true;
}

efft_plan_s *create_c2c(int64_t n, int64_t batch, int dtype, int dir, int inplace, double scale, int *status,
                        const int *digits = nullptr, int ndigits = 0)
{
    efft_plan_s *p = new (std::nothrow) efft_plan_s();
    if (!p) {
        *status = EFFT_ERR_ALLOC;
        return nullptr;
    }
    p->magic = PLAN_MAGIC;
    p->n = n;
    p->batch = batch;
    p->q = log2_exact(n);
    p->dtype = dtype;
    p->dir = dir;
    p->inplace = inplace ? 1 : 0;
    p->eb = dtype_bytes(dtype);
    p->scale = scale;
    p->kind = KIND_C2C;
    p->inner = nullptr;
    if (digits) {
        if (!digits_usable(p->q, p->eb, p->inplace, digits, ndigits)) {
            delete p;
            *status = EFFT_ERR_ARG;
            return nullptr;
        }
        p->m = ndigits;
        for (int i = 0; i < ndigits; ++i) p->digits[i] = digits[i];
    } else {
        p->m = plan_digits(p->q, p->eb, p->inplace, p->digits);
    }
    if (p->m < 1) {
        delete p;
        *status = EFFT_ERR_SIZE;
        return nullptr;
    }
    if (digits) {  // a kernel must exist for every pass of a chosen decomposition
        TwTable none{};
        build_passes(p, none);
        if (!kernels_exist(p)) {
            delete p;
            *status = EFFT_ERR_ARG;
            return nullptr;
        }
    }
    TwTable tt{};
    *status = make_tables(p, p->q, &tt);
    if (*status != EFFT_OK) {
        delete p;
        return nullptr;
    }
    build_passes(p, tt);
    return p;
}

// tile counts of a sub-FFT pass for `lines` x `sets` lines per workgroup;
// -1 if tiles would straddle blocks or the lines do not divide evenly
int64_t tiles_for(const efft_plan_s *p, const Pass &ps, int lines, int sets)
{
    const int64_t nlines = p->n >> ps.logl;  // lines per signal
    const int64_t w = int64_t(lines) * sets;
    if (w < 1 || nlines % w) return -1;
    if (ps.layout != LAYOUT_ROW && ps.layout != LAYOUT_ROW2COL && ps.sp.s % w)
        return -1;  // a tile of strided lines stays inside one block
    return nlines / w * p->batch;
}

void free_plan(efft_plan_s *p)
{
    if (!p) return;
    p->magic = 0;
    if (p->tables) (void)hipFree(p->tables);
    if (p->chirp) (void)hipFree(p->chirp);
    if (p->vhat) (void)hipFree(p->vhat);
    if (p->work) (void)hipFree(p->work);
    if (p->work2) (void)hipFree(p->work2);
    free_plan(p->inner);
    free_plan(p->inner2);
    delete p;
}

// Plan for N = M * 2^s, M odd and 3 <= M <= 15: the two tables, a work array
// of batch * N points and the batched plan of the 2^s-point rows.
efft_plan_s *create_mixed(int64_t n, int64_t batch, int dtype, int dir, int inplace, double scale, int *status)
{
    int64_t cols = 1;
    while ((n / cols) % 2 == 0) cols *= 2;
    const int mo = int(n / cols);
    efft_plan_s *p = new (std::nothrow) efft_plan_s();
    if (!p) {
        *status = EFFT_ERR_ALLOC;
        return nullptr;
    }
    p->magic = PLAN_MAGIC;
    p->n = n;
    p->batch = batch;
    p->q = -1;
    p->dtype = dtype;
    p->dir = dir;
    p->inplace = inplace ? 1 : 0;
    p->eb = dtype_bytes(dtype);
    p->scale = scale;
    p->kind = KIND_MIXED;
    p->m_odd = mo;
    p->cols = cols;
    int bits = 0;
    while ((int64_t(1) << bits) < n) ++bits;
    p->h_mixed = (bits + 1) / 2;
    const int64_t n_lo = int64_t(1) << p->h_mixed, n_hi = (n + n_lo - 1) / n_lo;
    p->inner = create_c2c(cols, batch * mo, dtype, dir, 1, 1.0, status);
    if (!p->inner) {
        free_plan(p);
        return nullptr;
    }
    if (!p->inner->scratch_passes.empty()) {
        // the rows' scratch schedule with its last pass (rows written as
        // columns at their natural positions) interleaving the M rows of each
        // signal: bin k1 + M k2 = row k1, bin k2 lands at k2 * M + k1
        p->mixed_passes = p->inner->scratch_passes;
        Pass &last = p->mixed_passes.back();
        if (last.swap || last.layout != LAYOUT_ROW2COL) {
            free_plan(p);
            *status = EFFT_ERR_HIP;
            return nullptr;
        }
        last.sp.ilv = mo;
        if (scale != 1.0) {
            last.sp.apply_scale = 1;
            last.sp.scale = scale;
        }
    }
    p->table_bytes = (mo + n_lo + n_hi) * int64_t(sizeof(double2)) + batch * n * p->eb;
    if (hipMalloc(reinterpret_cast<void **>(&p->tables), size_t(mo + n_lo + n_hi) * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->work, size_t(batch * n) * size_t(p->eb)) != hipSuccess) {
        (void)hipGetLastError();
        free_plan(p);
        *status = EFFT_ERR_ALLOC;
        return nullptr;
    }
    SetupStream ss;
    if (!ss.finish(ss.ok && launch_mixed_tables(p->tables, mo, p->tables + mo, n_lo, p->tables + mo + n_lo, n_hi,
                                                p->h_mixed, n, ss.s) == hipSuccess)) {
        free_plan(p);
        *status = EFFT_ERR_HIP;
        return nullptr;
    }
    *status = EFFT_OK;
    return p;
}

// Plan for a length n >= 3 that is not a power of two: two in-place plans of
// M = 2^ceil(log2(2n - 1)) points, the chirp and the transformed kernel are
// built here (on the current device), once.
efft_plan_s *create_chirp(int64_t n, int64_t batch, int dtype, int dir, int inplace, double scale, int *status)
{
    int64_t m = 1;
    while (m < 2 * n - 1) m *= 2;
    efft_plan_s *p = new (std::nothrow) efft_plan_s();
    if (!p) {
        *status = EFFT_ERR_ALLOC;
        return nullptr;
    }
    p->magic = PLAN_MAGIC;
    p->n = n;
    p->batch = batch;
    p->q = -1;
    p->dtype = dtype;
    p->dir = dir;
    p->inplace = inplace ? 1 : 0;
    p->eb = dtype_bytes(dtype);
    p->scale = scale;
    p->kind = KIND_CHIRP;
    p->m_pad = m;
    // Out-of-place M-point plans need fewer passes (no digit-reversal pass,
    // no palindrome constraint) but a second work array: used when the three
    // M-point arrays and the chirp take at most half of the device's memory,
    // a fixed rule per device so that results do not depend on what else is
    // allocated.
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        total_b = 0;
    }
    const bool oop = double(3 * m * int64_t(dtype_bytes(dtype)) + n * int64_t(sizeof(double2))) <= 0.5 * double(total_b);
    p->inner = create_c2c(m, 1, dtype, EFFT_FORWARD, oop ? 0 : 1, 1.0, status);
    if (p->inner) p->inner2 = create_c2c(m, 1, dtype, EFFT_BACKWARD, oop ? 0 : 1, 1.0, status);
    if (!p->inner || !p->inner2) {
        free_plan(p);
        return nullptr;
    }
    const size_t eb = size_t(p->eb);
    if (hipMalloc(reinterpret_cast<void **>(&p->chirp), size_t(n) * sizeof(double2)) != hipSuccess ||
        hipMalloc(&p->vhat, size_t(m) * eb) != hipSuccess || hipMalloc(&p->work, size_t(m) * eb) != hipSuccess ||
        (oop && hipMalloc(&p->work2, size_t(m) * eb) != hipSuccess)) {
        (void)hipGetLastError();
        free_plan(p);
        *status = EFFT_ERR_ALLOC;
        return nullptr;
    }
    p->table_bytes = int64_t(n) * int64_t(sizeof(double2)) + (oop ? 3 : 2) * m * int64_t(eb);
    if (oop && p->inner->passes.front().layout == LAYOUT_COL2ROW &&
        p->inner2->passes.front().layout == LAYOUT_COL2ROW) {
        p->chirp_fwd = p->inner->passes;
        p->chirp_fwd.front().layout = LAYOUT_COL2ROW_PRE;
        p->chirp_fwd.front().sp.pmode = PRE_CHIRP;
        p->chirp_fwd.front().sp.pre = p->chirp;
        p->chirp_fwd.front().sp.n_valid = n;
        p->chirp_bwd = p->inner2->passes;
        p->chirp_bwd.front().layout = LAYOUT_COL2ROW_PRE;
        p->chirp_bwd.front().sp.pmode = PRE_MUL;
        p->chirp_bwd.front().sp.pre = p->vhat;
        Pass &last = p->chirp_bwd.back();
        p->chirp_post = p->chirp_bwd.size() >= 2 && last.layout == LAYOUT_COL;
        if (p->chirp_post) {
            last.layout = LAYOUT_COL_POST;
            last.sp.post = p->chirp;
            last.sp.post_scale = p->scale;
            last.sp.n_valid = n;
        }
        if (!widen_to_kernel(p->inner, p->chirp_fwd.front()) || !widen_to_kernel(p->inner2, p->chirp_bwd.front()) ||
            (p->chirp_post && !widen_to_kernel(p->inner2, p->chirp_bwd.back()))) {
            // no fused kernel for these tiles: separate pre- and post-multiply passes
            p->chirp_fwd.clear();
            p->chirp_bwd.clear();
            p->chirp_post = false;
        }
    }
    // V = DFT_M(v) / M, formed in the work array and transformed into vhat
    // (in place when the inner plans are)
    void *vsrc = oop ? p->work : p->vhat;
    SetupStream ss;
    if (!ss.finish(ss.ok && launch_chirp(p->chirp, n, dir, ss.s) == hipSuccess &&
                   launch_chirp_v(p->eb, vsrc, p->chirp, n, m, ss.s) == hipSuccess &&
                   run_c2c(p->inner, vsrc, p->vhat, ss.s, nullptr, 0) == EFFT_OK)) {
        free_plan(p);
        *status = EFFT_ERR_HIP;
        return nullptr;
    }
    *status = EFFT_OK;
    return p;
}

void register_plan(efft_plan_s *p)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        dev = -1;
    }
    p->device = dev;
    std::lock_guard<std::mutex> lk(g_reg_mu);
    g_registry.insert(p);
}

// ------------------------------------------------ fixed device scratch array
// The scratch array of efft_exec_noalloc: a fixed device array in place of
// the caller-owned one of efft_exec_scratch, for callers that cannot
// allocate.  Each device the library runs on holds its own copy for the life
// of the process.  Host code never passes the array's name to a kernel (on
// the host it only stands for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device on the first efft_exec_noalloc call there.
static __device__ __align__(256) unsigned char scratch[EFFT_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// device address of the fixed scratch array on `dev` (the current device)
int fixed_scratch(int dev, void **ptr)
{
    if (dev < 0 || dev >= MAX_DEVICES) return EFFT_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *a = nullptr;
        if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) {
            (void)hipGetLastError();
            return EFFT_ERR_HIP;
        }
        g_scratch_ptr[dev] = a;
    }
    *ptr = g_scratch_ptr[dev];
    return EFFT_OK;
}

// bytes of the input and output arrays of one execution
int64_t in_bytes(const efft_plan_s *p)
{
    if (p->kind == KIND_R2C) return p->n * p->eb / 2;
    if (p->kind == KIND_C2R) return (p->n / 2 + 1) * p->eb;
    return p->batch * p->n * p->eb;
}
int64_t out_bytes(const efft_plan_s *p)
{
    if (p->kind == KIND_R2C) return (p->n / 2 + 1) * p->eb;
    if (p->kind == KIND_C2R) return p->n * p->eb / 2;
    return p->batch * p->n * p->eb;
}

int validate_scratch(const efft_plan_s *p, const void *data, const void *scratch)
{
    int v = validate_ptr(p, scratch);
    if (v != EFFT_OK) return v;
    const uintptr_t a = reinterpret_cast<uintptr_t>(data), b = reinterpret_cast<uintptr_t>(scratch);
    const uintptr_t bytes = uintptr_t(p->batch) * uintptr_t(p->n) * uintptr_t(p->eb);
    return (a < b + bytes && b < a + bytes) ? EFFT_ERR_OVERLAP : EFFT_OK;
}

bool overlaps(const efft_plan_s *p, const void *in, const void *out)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
    return a < b + uintptr_t(out_bytes(p)) && b < a + uintptr_t(in_bytes(p));
}

}  // namespace

extern "C" {

efft_plan_t *efft_plan(int64_t n, int dtype, int dir, int inplace)
{
    return efft_plan_scaled(n, dtype, dir, inplace, 1.0);
}

efft_plan_t *efft_plan_scaled(int64_t n, int dtype, int dir, int inplace, double scale)
{
    return efft_plan_many(n, 1, dtype, dir, inplace, scale);
}

efft_plan_t *efft_plan_many(int64_t n, int64_t batch, int dtype, int dir, int inplace, double scale)
{
    const bool chirp = n >= 3 && n <= MAX_CHIRP_N && log2_exact(n) < 0;
    const int q = chirp ? 1 : log2_exact(n);  // the remaining checks are size-independent
    int status = validate_args(q, dtype, dir, scale);
    if (status == EFFT_OK && batch < 1) status = EFFT_ERR_ARG;
    if (status == EFFT_OK && (batch > (int64_t(1) << 40) / n)) status = EFFT_ERR_SIZE;  // 2^40 points
    if (status != EFFT_OK) {
        g_last_error = status;
        return nullptr;
    }
    int64_t odd = n;
    while (odd > 0 && odd % 2 == 0) odd /= 2;
    const bool mixed = chirp && odd <= 15;  // N = M * 2^s with a small odd M: one radix-M pass
    efft_plan_s *p = mixed   ? create_mixed(n, batch, dtype, dir, inplace, scale, &status)
                     : chirp ? create_chirp(n, batch, dtype, dir, inplace, scale, &status)
                             : create_c2c(n, batch, dtype, dir, inplace, scale, &status);
    if (!p) {
        g_last_error = status;
        return nullptr;
    }
    register_plan(p);
    g_last_error = EFFT_OK;
    return p;
}

efft_plan_t *efft_plan_real(int64_t n, int dtype, int dir, double scale)
{
    const int q = log2_exact(n);
    int status = validate_args(q, dtype, dir, scale);
    if (status == EFFT_OK && q < 1) status = EFFT_ERR_SIZE;
    if (status != EFFT_OK) {
        g_last_error = status;
        return nullptr;
    }
    efft_plan_s *p = new (std::nothrow) efft_plan_s();
    if (!p) {
        g_last_error = EFFT_ERR_ALLOC;
        return nullptr;
    }
    p->magic = PLAN_MAGIC;
    p->n = n;
    p->batch = 1;
    p->q = q;
    p->dtype = dtype;
    p->dir = dir;
    p->inplace = 0;
    p->eb = dtype_bytes(dtype);
    p->scale = scale;
    p->kind = dir == EFFT_FORWARD ? KIND_R2C : KIND_C2R;
    status = make_tables(p, q, &p->tt_real);
    if (status != EFFT_OK) {
        delete p;
        g_last_error = status;
        return nullptr;
    }
    // R2C: out-of-place forward N/2-point transform, scale applied by the
    // pairing pass; C2R: in-place backward N/2-point transform on the output,
    // scale applied by its last pass
    p->inner = create_c2c(n / 2, 1, dtype, dir, dir == EFFT_BACKWARD ? 1 : 0,
                          dir == EFFT_BACKWARD ? scale : 1.0, &status);
    if (!p->inner) {
        (void)hipFree(p->tables);
        delete p;
        g_last_error = status;
        return nullptr;
    }
    register_plan(p);
    g_last_error = EFFT_OK;
    return p;
}

int efft_exec(const efft_plan_t *plan, void *data, void *stream)
{
    const efft_plan_s *p = live(plan);
    if (!p) return plan ? EFFT_ERR_BADPLAN : EFFT_ERR_NULLPTR;
    if (!p->inplace) return EFFT_ERR_PLAN_KIND;
    const int v = validate_ptr(p, data);
    if (v != EFFT_OK) return v;
    return run(p, data, data, static_cast<hipStream_t>(stream), nullptr, 0);
}

int efft_exec_oop(const efft_plan_t *plan, const void *in, void *out, void *stream)
{
    const efft_plan_s *p = live(plan);
    if (!p) return plan ? EFFT_ERR_BADPLAN : EFFT_ERR_NULLPTR;
    if (p->inplace) return EFFT_ERR_PLAN_KIND;
    int v = validate_ptr(p, in);
    if (v == EFFT_OK) v = validate_ptr(p, out);
    if (v != EFFT_OK) return v;
    if (overlaps(p, in, out)) return EFFT_ERR_OVERLAP;
    return run(p, in, out, static_cast<hipStream_t>(stream), nullptr, 0);
}

int efft_exec_events(const efft_plan_t *plan, const void *in, void *out, void *scratch, void *stream,
                     void **events, int nevents)
{
    const efft_plan_s *p = live(plan);
    if (!p) return plan ? EFFT_ERR_BADPLAN : EFFT_ERR_NULLPTR;
    if (!events) return EFFT_ERR_NULLPTR;
    int v = validate_ptr(p, in);
    if (v == EFFT_OK) v = validate_ptr(p, out);
    if (v != EFFT_OK) return v;
    if (p->inplace && in != out) return EFFT_ERR_PLAN_KIND;
    if (!p->inplace && overlaps(p, in, out)) return EFFT_ERR_OVERLAP;
    if (scratch && !p->scratch_passes.empty()) {
        v = validate_scratch(p, out, scratch);
        if (v != EFFT_OK) return v;
        return run_passes(p->scratch_passes, p->batch, p->eb, in, out, scratch, static_cast<hipStream_t>(stream),
                          events, nevents);
    }
    return run(p, in, out, static_cast<hipStream_t>(stream), events, nevents);
}

int efft_exec_scratch(const efft_plan_t *plan, void *data, void *scratch, void *stream)
{
    const efft_plan_s *p = live(plan);
    if (!p) return plan ? EFFT_ERR_BADPLAN : EFFT_ERR_NULLPTR;
    if (!p->inplace) return EFFT_ERR_PLAN_KIND;
    int v = validate_ptr(p, data);
    if (v != EFFT_OK) return v;
    if (p->scratch_passes.empty()) return run(p, data, data, static_cast<hipStream_t>(stream), nullptr, 0);
    v = validate_scratch(p, data, scratch);
    if (v != EFFT_OK) return v;
    return run_passes(p->scratch_passes, p->batch, p->eb, data, data, scratch, static_cast<hipStream_t>(stream),
                      nullptr, 0);
}

int efft_exec_noalloc(const efft_plan_t *plan, void *data, void *stream)
{
    const efft_plan_s *p = live(plan);
    if (!p) return plan ? EFFT_ERR_BADPLAN : EFFT_ERR_NULLPTR;
    if (!p->inplace) return EFFT_ERR_PLAN_KIND;
    const int v = validate_ptr(p, data);
    if (v != EFFT_OK) return v;
    if (p->scratch_passes.empty()) return run(p, data, data, static_cast<hipStream_t>(stream), nullptr, 0);
    if (p->batch * p->n * p->eb > int64_t(EFFT_NOALLOC_SCRATCH_BYTES)) return EFFT_ERR_SIZE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return EFFT_ERR_HIP;
    }
    if (dev != p->device) return EFFT_ERR_ARG;
    void *ws = nullptr;
    const int r = fixed_scratch(dev, &ws);
    if (r != EFFT_OK) return r;
    return run_passes(p->scratch_passes, p->batch, p->eb, data, data, ws, static_cast<hipStream_t>(stream),
                      nullptr, 0);
}

int64_t efft_scratch_bytes(const efft_plan_t *plan)
{
    const efft_plan_s *p = live(plan);
    if (!p) return -1;
    return p->scratch_passes.empty() ? 0 : p->batch * p->n * p->eb;
}

int efft_plan_passes_scratch(const efft_plan_t *plan)
{
    const efft_plan_s *p = live(plan);
    if (!p) return -1;
    return p->scratch_passes.empty() ? total_passes(p) : int(p->scratch_passes.size());
}

int efft_destroy(efft_plan_t *plan)
{
    if (!plan) return EFFT_OK;
    {
        std::lock_guard<std::mutex> lk(g_reg_mu);
        if (!g_registry.erase(plan)) return EFFT_ERR_BADPLAN;
    }
    free_plan(plan);
    return EFFT_OK;
}

int efft_last_error(void) { return g_last_error; }

const char *efft_strerror(int status)
{
    switch (status) {
    case EFFT_OK: return "EFFT_OK: success";
    case EFFT_ERR_SIZE: return "EFFT_ERR_SIZE: n must be 2^q (0 <= q <= 34) or another length 3 <= n <= 2^33";
    case EFFT_ERR_DTYPE: return "EFFT_ERR_DTYPE: dtype must be EFFT_C64 or EFFT_C128";
    case EFFT_ERR_DIR: return "EFFT_ERR_DIR: dir must be EFFT_FORWARD (-1) or EFFT_BACKWARD (+1)";
    case EFFT_ERR_NULLPTR: return "EFFT_ERR_NULLPTR: required pointer is NULL";
    case EFFT_ERR_ALIGN: return "EFFT_ERR_ALIGN: data pointer not aligned to one element";
    case EFFT_ERR_PLAN_KIND: return "EFFT_ERR_PLAN_KIND: in-place/out-of-place mismatch";
    case EFFT_ERR_OVERLAP: return "EFFT_ERR_OVERLAP: input and output ranges overlap";
    case EFFT_ERR_ALLOC: return "EFFT_ERR_ALLOC: device allocation failed";
    case EFFT_ERR_HIP: return "EFFT_ERR_HIP: HIP call or kernel launch failed";
    case EFFT_ERR_BADPLAN: return "EFFT_ERR_BADPLAN: not a live plan";
    case EFFT_ERR_ARG: return "EFFT_ERR_ARG: invalid argument";
    default: return "unknown efft status";
    }
}

int64_t efft_plan_bytes(const efft_plan_t *plan)
{
    const efft_plan_s *p = live(plan);
    if (!p) return -1;
    return p->table_bytes + (p->inner ? p->inner->table_bytes : 0) + (p->inner2 ? p->inner2->table_bytes : 0);
}

efft_plan_t *efft_plan_digits(int64_t n, int64_t batch, int dtype, int dir, int inplace, double scale,
                              const int *log2_digits, int m)
{
    const int q = log2_exact(n);
    int status = validate_args(q, dtype, dir, scale);
    if (status == EFFT_OK && (batch < 1 || !log2_digits)) status = batch < 1 ? EFFT_ERR_ARG : EFFT_ERR_NULLPTR;
    if (status == EFFT_OK && batch > (int64_t(1) << 40) / n) status = EFFT_ERR_SIZE;
    if (status != EFFT_OK) {
        g_last_error = status;
        return nullptr;
    }
    efft_plan_s *p = create_c2c(n, batch, dtype, dir, inplace, scale, &status, log2_digits, m);
    if (!p) {
        g_last_error = status;
        return nullptr;
    }
    register_plan(p);
    g_last_error = EFFT_OK;
    return p;
}

int efft_pass_options(const efft_plan_t *plan, int scratch, int pass, int *opts)
{
    const efft_plan_s *p = live(plan);
    if (!p) return plan ? EFFT_ERR_BADPLAN : EFFT_ERR_NULLPTR;
    if (!opts) return EFFT_ERR_NULLPTR;
    if (p->kind != KIND_C2C) return EFFT_ERR_PLAN_KIND;
    const std::vector<Pass> &v = scratch ? p->scratch_passes : p->passes;
    if (pass < 0 || pass >= int(v.size())) return EFFT_ERR_ARG;
    const Pass &ps = v[size_t(pass)];
    if (ps.swap) {
        opts[0] = -1;
        opts[1] = opts[2] = opts[3] = 0;
        opts[4] = opts[5] = ps.wp.nt_hint;
    } else {
        opts[0] = ps.layout;
        opts[1] = ps.lines;
        opts[2] = ps.sets;
        opts[3] = ps.sp.order;
        opts[4] = ps.sp.nt_load;
        opts[5] = ps.sp.nt_store;
    }
    return EFFT_OK;
}

int efft_set_pass_options(efft_plan_t *plan, int scratch, int pass, const int *opts)
{
    efft_plan_s *p = const_cast<efft_plan_s *>(live(plan));
    if (!p) return plan ? EFFT_ERR_BADPLAN : EFFT_ERR_NULLPTR;
    if (!opts) return EFFT_ERR_NULLPTR;
    if (p->kind != KIND_C2C) return EFFT_ERR_PLAN_KIND;
    std::vector<Pass> &v = scratch ? p->scratch_passes : p->passes;
    if (pass < 0 || pass >= int(v.size())) return EFFT_ERR_ARG;
    for (int i = 3; i < 6; ++i)
        if (opts[i] < 0) return EFFT_ERR_ARG;
    if (opts[3] > TILE_XCD_SCATTER || opts[4] > 1 || opts[5] > 1) return EFFT_ERR_ARG;
    Pass ps = v[size_t(pass)];
    if (ps.swap) {
        ps.wp.nt_hint = opts[4];
    } else {
        const int64_t nt = tiles_for(p, ps, opts[1], opts[2]);
        if (nt < 0) return EFFT_ERR_ARG;
        ps.lines = opts[1];
        ps.sets = opts[2];
        ps.sp.ntiles = nt;
        ps.sp.order = opts[3];
        ps.sp.nt_load = opts[4];
        ps.sp.nt_store = opts[5];
        set_dry_run(true);
        const hipError_t e = launch_stage(p->eb, ps.layout, ps.logl, ps.lines, ps.sets, ps.sp, nullptr);
        set_dry_run(false);
        if (e != hipSuccess) return EFFT_ERR_ARG;  // no kernel for this combination
    }
    v[size_t(pass)] = ps;
    return EFFT_OK;
}

int64_t efft_workspace_bytes(const efft_plan_t *plan) { return efft_plan_bytes(plan); }

int64_t efft_plan_batch(const efft_plan_t *plan)
{
    const efft_plan_s *p = live(plan);
    return p ? p->batch : -1;
}

int efft_plan_passes(const efft_plan_t *plan)
{
    const efft_plan_s *p = live(plan);
    return p ? total_passes(p) : -1;
}

int efft_schedule(int64_t n, int dtype, int inplace, int *log2_radix, int max_digits, int *passes)
{
    const int q = log2_exact(n);
    if (q < 0 || q > EFFT_MAX_LOG2N) return EFFT_ERR_SIZE;
    const int eb = dtype_bytes(dtype);
    if (!eb) return EFFT_ERR_DTYPE;
    if (!log2_radix || !passes) return EFFT_ERR_NULLPTR;
    // build the plan's passes without device tables and check that a kernel
    // instantiation exists for each of them
    efft_plan_s probe{};
    probe.magic = PLAN_MAGIC;
    probe.n = n;
    probe.batch = 1;
    probe.q = q;
    probe.dtype = dtype;
    probe.dir = EFFT_FORWARD;
    probe.inplace = inplace ? 1 : 0;
    probe.eb = eb;
    probe.scale = 1.0;
    probe.kind = KIND_C2C;
    probe.m = plan_digits(q, eb, probe.inplace, probe.digits);
    if (probe.m < 1) return EFFT_ERR_SIZE;
    if (probe.m > max_digits) return EFFT_ERR_ARG;
    TwTable tt{};
    build_passes(&probe, tt);
    set_dry_run(true);
    int status = EFFT_OK;
    std::vector<Pass> all = probe.passes;
    all.insert(all.end(), probe.scratch_passes.begin(), probe.scratch_passes.end());
    for (const Pass &ps : all) {
        const hipError_t e = ps.swap ? launch_swap(eb, ps.wp, 1, nullptr)
                                     : launch_stage(eb, ps.layout, ps.logl, ps.lines, ps.sets, ps.sp, nullptr);
        if (e != hipSuccess) status = EFFT_ERR_SIZE;
    }
    set_dry_run(false);
    if (status != EFFT_OK) return status;
    for (int i = 0; i < probe.m; ++i) log2_radix[i] = probe.digits[i];
    *passes = int(probe.passes.size());
    return probe.m;
}

}  // extern "C"
