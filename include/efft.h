/*
 * efft.h -- C ABI of an MI355X (gfx950) library for one very large in-memory
 * one-dimensional complex-to-complex FFT, N = 2^q points.
 *
 * Operation (Asai & Vladimirov, "EFFT", Section 1, Eq. "eqf"):
 *
 *     F_k = sum_{n=0}^{N-1} x_n * exp(sign * 2*pi*i * k*n / N),   0 <= k < N,
 *
 * with sign = -1 (EFFT_FORWARD, the paper's transform as written) or
 * sign = +1 (EFFT_BACKWARD, the conjugate-sign transform; the paper defines
 * only the forward one).  Neither direction is scaled: backward(forward(x))
 * equals N*x, and the backward transform is the exact adjoint of the forward
 * one.  Input and output are in natural order (F_k at index k).
 *
 * The plan/execute split follows the paper's usage flow of a transform
 * handle that is created once, committed, and then reused (Section 2.1,
 * Listing "code:dfti"; Section 3.1, the handles built once at initialisation
 * because creating them costs more than a transform).  Like the paper's
 * EFFT_Transform (Section 4, Listing "code:efftheader"), the transform size is
 * the only required parameter; the decomposition (the paper's number of
 * splits) is chosen internally.
 *
 * Data layout: interleaved complex (re, im), the layout of torch.complex64 /
 * torch.complex128 and of the paper's stride-2 complex arrays (Section 3.4):
 *   EFFT_C64  -- float  re, im (8 bytes per element), FP32 storage and
 *                arithmetic; every twiddle factor is generated in FP64 and
 *                rounded once to FP32.
 *   EFFT_C128 -- double re, im (16 bytes per element), FP64 throughout.
 *
 * Memory: every data pointer is a device pointer in the calling process's
 * current HIP device, owned by the caller, and must be aligned to one element
 * (8 bytes for EFFT_C64, 16 for EFFT_C128).  The paper's EFFT allocates its
 * own 64-byte-aligned array (Section 3.1); here the caller allocates, and the
 * kernels need only element alignment.  A power-of-two or real-data plan owns only its FP64 twiddle
 * tables (at most a few hundred KiB); a plan for another length also owns
 * work arrays (see efft_plan and efft_plan_bytes).  Everything a plan owns is
 * allocated on the device that is current when the plan is created, and
 * efft_destroy frees it.
 *
 * Asynchrony and threads: the exec calls only enqueue kernels on the given
 * stream (a hipStream_t; NULL selects the default stream) and return;
 * device-side faults surface at the caller's next synchronisation.  Plan
 * creation waits for its own table-building kernels on a private stream of
 * the library (no device-wide synchronisation).  A power-of-two or real-data
 * plan holds no scratch memory and may be executed concurrently from several
 * streams; a plan that owns work arrays (lengths that are not powers of two)
 * must not have two executions in flight at once.  efft_set_pass_options
 * changes a plan and must not overlap any execution of it.  Error statuses
 * from plan creation are kept per host thread (efft_last_error).
 *
 * Errors: every function that returns int returns EFFT_OK (0) or one of the
 * negative EFFT_ERR_* codes below; efft_strerror names them.
 */
#ifndef EFFT_H
#define EFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct efft_plan_s efft_plan_t; /* opaque */

/* element types (interleaved complex) */
enum { EFFT_C64 = 1, EFFT_C128 = 2 };

/* direction = sign of the exponent in Eq. "eqf" */
enum { EFFT_FORWARD = -1, EFFT_BACKWARD = 1 };

/* status codes */
enum {
    EFFT_OK = 0,
    EFFT_ERR_SIZE = -1,      /* n is neither 2^q (0 <= q <= EFFT_MAX_LOG2N) nor 3 <= n <= 2^(EFFT_MAX_LOG2N-1) */
    EFFT_ERR_DTYPE = -2,     /* dtype is neither EFFT_C64 nor EFFT_C128 */
    EFFT_ERR_DIR = -3,       /* dir is neither EFFT_FORWARD nor EFFT_BACKWARD */
    EFFT_ERR_NULLPTR = -4,   /* a required pointer is NULL */
    EFFT_ERR_ALIGN = -5,     /* a data pointer is not aligned to one element */
    EFFT_ERR_PLAN_KIND = -6, /* efft_exec on an out-of-place plan or the reverse */
    EFFT_ERR_OVERLAP = -7,   /* out-of-place input and output ranges overlap */
    EFFT_ERR_ALLOC = -8,     /* device allocation for the plan failed */
    EFFT_ERR_HIP = -9,       /* a HIP call or kernel launch failed */
    EFFT_ERR_BADPLAN = -10,  /* handle is not a live plan (never made, or destroyed) */
    EFFT_ERR_ARG = -11       /* any other invalid argument */
};

/* largest supported q: 2^34 complex64 (128 GiB) is the largest enormous
 * transform that fits one 288 GB device in place */
#define EFFT_MAX_LOG2N 34

/*
 * Create a plan for an N-point transform.  n = N = 2^q (0 <= q <= 34), or any
 * other length 3 <= N <= 2^33;
 * dtype = EFFT_C64 or EFFT_C128; dir = EFFT_FORWARD or EFFT_BACKWARD;
 * inplace != 0 makes an in-place plan (executed with efft_exec), inplace == 0
 * an out-of-place plan (executed with efft_exec_oop).  Builds the FP64 twiddle
 * tables on the current device and waits for that to finish.  Returns NULL on
 * failure, with the reason in efft_last_error().
 *
 * A length N = M * 2^s with an odd M <= 15 (the paper's EFFT takes N =
 * M * 2^s, Section 2.2 and Section 4, with MKL doing the M-point bin DFTs)
 * runs one radix-M pass (direct M-point sums in FP64 and the twiddle
 * W_N^{n2 k1}) and the M batched 2^s-point transforms of the rows, whose last
 * pass writes the rows interleaved into the output in natural order (rows of
 * at most 2^12 points, which take a single pass, are followed by a reorder
 * pass instead); such a plan owns the tables and a work array of N points
 * per signal, so at most one execution of it may be in flight at a time.
 * Any other length is
 * transformed through the chirp identity n*k = (n^2 + k^2 - (k-n)^2)/2:
 * F_k = a_k sum_n (x_n a_n) conj(a_{k-n}), a_m = exp(sign*pi*i*m^2/N), a
 * linear convolution done as a cyclic one of length M = 2^ceil(log2(2N-1))
 * with the library's power-of-two passes.  Such a plan owns, on the device,
 * the chirp (N FP64 complex values), the transformed convolution kernel and
 * a work array (M elements of dtype each; see efft_plan_bytes), so at most
 * one execution of it may be in flight at a time.  Each execution runs, per
 * signal: a pre-multiply, an M-point forward transform, a pointwise product,
 * an M-point backward transform and a post-multiply pass.  When the M-point
 * transforms run out of place (the device has room for a second work array),
 * the pre-multiply and the pointwise product are applied by the first pass
 * of each transform as it loads and the post-multiply by the last pass as it
 * stores, so they add no pass of their own.
 */
efft_plan_t *efft_plan(int64_t n, int dtype, int dir, int inplace);

/*
 * As efft_plan, with every output multiplied by `scale` inside the last
 * sub-FFT pass (no extra pass over the data).  scale = 1/N turns the
 * backward transform into the inverse DFT; for N = 2^q that factor is exact.
 * scale must be finite and nonzero (else EFFT_ERR_ARG).
 */
efft_plan_t *efft_plan_scaled(int64_t n, int dtype, int dir, int inplace, double scale);

/*
 * Batched plan: `batch` independent transforms of n points each (the paper's
 * "many transforms" mode, Section 2.1), signal b at elements
 * [b*n, (b+1)*n) of every array the exec calls take; each exec call then
 * transforms all of them with the same number of passes as one signal.
 * n, dtype, dir, inplace and scale as for efft_plan_scaled; batch >= 1 (else
 * EFFT_ERR_ARG) and batch * n <= 2^40 (else EFFT_ERR_SIZE).  A scratch array
 * for efft_exec_scratch then holds batch * n elements.  efft_plan_scaled is
 * efft_plan_many with batch = 1.
 */
efft_plan_t *efft_plan_many(int64_t n, int64_t batch, int dtype, int dir, int inplace, double scale);

/* Signals per execution of a plan (1 unless made by efft_plan_many); -1 if
 * plan is not a live plan. */
int64_t efft_plan_batch(const efft_plan_t *plan);

/*
 * As efft_plan_many for N = 2^q, with the decomposition N = 2^d_0 * ... *
 * 2^d_{m-1} chosen by the caller (log2_digits[i] = d_i, slowest input digit
 * first) instead of by the planner -- the GPU form of the paper's tuning
 * scan over the number of splits (Section 5.2, Fig. "fig:heatmap"; see
 * efft_set_pass_options for the other knobs).  The digits must sum to q;
 * with m = 1, q <= 12; with m > 1 every digit lies in [4, 12] and an in-place
 * plan needs a palindrome (d_i = d_{m-1-i}).  Returns NULL with EFFT_ERR_ARG
 * for an unusable decomposition, EFFT_ERR_NULLPTR if log2_digits is NULL, and
 * the codes of efft_plan_many otherwise.
 */
efft_plan_t *efft_plan_digits(int64_t n, int64_t batch, int dtype, int dir, int inplace, double scale,
                              const int *log2_digits, int m);

/*
 * Launch options of pass `pass` (0-based) of a power-of-two plan's schedule:
 * scratch = 0 selects the plain schedule (efft_exec / efft_exec_oop),
 * scratch = 1 the scratch schedule (efft_exec_scratch).  opts[0..5]:
 *   opts[0] layout (read only: 0 contiguous lines, 1 strided lines,
 *           2 strided lines written as rows, 3 rows written as strided
 *           lines, -1 the digit-reversal swap),
 *   opts[1] lines per line set of a workgroup, opts[2] line sets per
 *           workgroup, opts[3] tile order (0 linear, 1 one contiguous run
 *           per XCD, 2 the same walked with an odd stride),
 *   opts[4] non-temporal loads, opts[5] non-temporal stores (0/1; for the
 *           swap opts[4] sets both).
 * efft_pass_options reads them; efft_set_pass_options replaces them if a
 * kernel exists for the combination (else EFFT_ERR_ARG, plan unchanged).
 * They decide which workgroup transforms which lines and how memory is
 * accessed, never the arithmetic: every valid setting gives bit-identical
 * results.  Setting options must not overlap an execution of the plan.
 * EFFT_ERR_PLAN_KIND for real-input plans and lengths that are not powers of
 * two.
 */
int efft_pass_options(const efft_plan_t *plan, int scratch, int pass, int *opts);
int efft_set_pass_options(efft_plan_t *plan, int scratch, int pass, const int *opts);

/*
 * Real-data plan for N = 2^q real samples (1 <= q <= 34), always out of
 * place, executed with efft_exec_oop.  The paper's EFFT transforms real data
 * (Section 2.1 "code:dfti", Section 4); this keeps the standard half-spectrum
 * layout rather than MKL's packed "perm" order:
 *   dir = EFFT_FORWARD  (real to complex): in = N reals (float for EFFT_C64,
 *       double for EFFT_C128), out = N/2 + 1 complex bins F_0 .. F_{N/2} of
 *       Eq. "eqf" (the rest follow from F_{N-k} = conj F_k);
 *   dir = EFFT_BACKWARD (complex to real): in = N/2 + 1 complex bins taken as
 *       the half of a Hermitian spectrum (the imaginary parts of F_0 and
 *       F_{N/2} are ignored), out = N reals of the unnormalised backward
 *       transform (N * x for in = the forward transform of x).
 * Every output is multiplied by scale (1/N makes the backward transform the
 * inverse).  Computed as one N/2-point complex transform plus one pass that
 * combines bins k and N/2 - k in place (one radix-2 level, Section 2.2, Eqs.
 * "eqct"/"eqctt"; the pair reassembly of Section 3.4).  Input and output must
 * not overlap; in is not written.  Returns NULL on failure (efft_last_error).
 */
efft_plan_t *efft_plan_real(int64_t n, int dtype, int dir, double scale);

/*
 * In-place transform of data[0 .. N) (device pointer, N elements of the
 * plan's dtype), enqueued on stream: the compute step of the paper's
 * create/commit/compute flow (Section 2.1, Listing "code:dfti",
 * DftiComputeForward) and of EFFT_Transform's RunTransform() (Section 4,
 * Listing "code:efftheader"), with the result in the data array itself.  The
 * in-place path is a sequence of batched sub-FFT passes followed by one tiled
 * digit-reversal pass; it needs no memory beyond the data array itself.
 * EFFT_ERR_NULLPTR for a NULL plan or data, EFFT_ERR_BADPLAN for a handle
 * that is not a live plan, EFFT_ERR_PLAN_KIND for an out-of-place plan,
 * EFFT_ERR_ALIGN for data not aligned to one element, EFFT_ERR_HIP if a
 * launch fails; nothing is enqueued on an argument error.
 */
int efft_exec(const efft_plan_t *plan, void *data, void *stream);

/*
 * Out-of-place transform: reads in[0 .. N), writes out[0 .. N), enqueued on
 * stream (for real-data plans the array sizes are those of efft_plan_real).
 * in is never written (the input is preserved, as the paper's
 * EFFT_Transform keeps Data() separate from Result(), Section 4).  The two
 * ranges must not overlap.
 */
int efft_exec_oop(const efft_plan_t *plan, const void *in, void *out, void *stream);

/*
 * In-place transform like efft_exec, using a caller-owned device scratch
 * array of efft_scratch_bytes(plan) bytes (N elements; it must not overlap
 * data).  With scratch the digit-reversal pass disappears: the last sub-FFT
 * pass reads rows of the scratch array and writes its results straight to
 * their natural positions in data, so the transform makes one pass fewer over
 * memory.  This trades the extra array for speed, as the paper's EFFT does
 * with its scratch array (Section 3.1).  The scratch contents are undefined
 * afterwards.  For plans that gain nothing from scratch (N <= 2^12),
 * efft_scratch_bytes returns 0 and this call is efft_exec (scratch may be NULL).
 */
int efft_exec_scratch(const efft_plan_t *plan, void *data, void *scratch, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * transform of efft_exec_scratch with the scratch array taken from a fixed
 * array of EFFT_NOALLOC_SCRATCH_BYTES bytes that the library holds on each
 * device it runs on, until the process ends.  This call allocates nothing
 * and frees nothing; it needs batch * N * element bytes <= that size (else
 * EFFT_ERR_SIZE, nothing enqueued; 2^22 complex128 or 2^23 complex64
 * points), an in-place plan (else EFFT_ERR_PLAN_KIND), and the plan's device
 * to be the current one (else EFFT_ERR_ARG).  Results are bit-identical to
 * efft_exec_scratch.  Every call on one device shares that device's array:
 * two calls whose executions overlap in time on one device (different
 * streams, or different host threads) race and give undefined results; calls
 * ordered on one stream are safe.  Nothing in the array needs clearing
 * between calls: the first pass writes every element it later reads.  For
 * plans that gain nothing from scratch this call is efft_exec.
 */
#define EFFT_NOALLOC_SCRATCH_BYTES (64LL << 20)
int efft_exec_noalloc(const efft_plan_t *plan, void *data, void *stream);

/* Scratch bytes efft_exec_scratch uses (0 if none helps); -1 for a bad handle. */
int64_t efft_scratch_bytes(const efft_plan_t *plan);

/* Kernel launches of one efft_exec_scratch call; -1 for a bad handle. */
int efft_plan_passes_scratch(const efft_plan_t *plan);

/*
 * Same work as efft_exec (in == out, in-place plan; with scratch != NULL as
 * efft_exec_scratch) or efft_exec_oop (other plans), additionally recording
 * events[i] (hipEvent_t, created by the caller) on stream just before kernel
 * pass i and events[npass] after the last one, so that per-pass durations can
 * be read with hipEventElapsedTime.  nevents must be at least the number of
 * passes + 1 (efft_plan_passes, or efft_plan_passes_scratch with scratch).
 * Chirp-path plans (lengths with an odd factor above 15) accept events only
 * with a batch of 1 (else EFFT_ERR_ARG).
 */
int efft_exec_events(const efft_plan_t *plan, const void *in, void *out, void *scratch, void *stream,
                     void **events, int nevents);

/* Free everything the plan owns on the device (its tables and, for lengths
 * that are not powers of two, its work arrays), as the paper's
 * ~EFFT_Transform() releases the transform's buffers (Section 4, Listing
 * "code:efftheader").
 * The caller must make sure no execution of the plan is still running.  NULL
 * is a no-op returning EFFT_OK; a handle that is not a live plan (already
 * destroyed) returns EFFT_ERR_BADPLAN. */
int efft_destroy(efft_plan_t *plan);

/* Status of the last efft_plan call on this host thread. */
int efft_last_error(void);

/* Static, human-readable name of a status code. */
const char *efft_strerror(int status);

/* Device bytes held by the plan (its twiddle tables, and for a length that is
 * not a power of two also the chirp, kernel and work arrays); -1 for a bad
 * handle. */
int64_t efft_plan_bytes(const efft_plan_t *plan);

/* The same figure under the name of a workspace query: device bytes a plan
 * owns and keeps for its whole life (it allocates nothing at execution). */
int64_t efft_workspace_bytes(const efft_plan_t *plan);

/* Number of kernel launches one execution enqueues (for a chirp-path plan,
 * which runs the signals of a batch one after another, per signal); -1 for a
 * bad handle. */
int efft_plan_passes(const efft_plan_t *plan);

/*
 * Host-only description of the decomposition a power-of-two plan would use
 * (no device needed; other lengths return EFFT_ERR_SIZE).  Writes the digit sizes log2(R_1), ..., log2(R_m) of
 * N = R_1 * ... * R_m (R_1 is the digit of the slowest-varying input index,
 * transformed first) into log2_radix[0 .. m), at most max_digits of them, and
 * returns m, or a negative status for invalid arguments.  *passes receives the
 * number of kernel launches (m sub-FFT passes, plus one digit-reversal pass
 * for in-place plans with m >= 2).  It also checks, without launching
 * anything, that the library holds a kernel for every pass of that plan, and
 * returns EFFT_ERR_SIZE if not.
 */
int efft_schedule(int64_t n, int dtype, int inplace, int *log2_radix, int max_digits,
                  int *passes);

/*
 * Memory-bandwidth reference: copies `bytes` bytes from src to dst, enqueued
 * on `stream` (a hipStream_t; NULL is the default stream).  The paper sets
 * EFFT beside the STREAM benchmark (Section 5.4, Fig. "fig:parallel-perf");
 * this is the GPU counterpart, a streaming copy with the access style of the
 * transform's passes (16-byte accesses with the non-temporal hint), which the
 * benchmark reports as the achievable copy bandwidth.  dst and src are device
 * pointers, both 16-byte aligned (else EFFT_ERR_ALIGN), non-NULL (else
 * EFFT_ERR_NULLPTR), with ranges that do not overlap (else
 * EFFT_ERR_OVERLAP) unless dst == src, which rewrites the range in place
 * (the access pattern of an in-place pass); bytes must be a non-negative
 * multiple of 16 (else
 * EFFT_ERR_ARG), and 0 enqueues nothing.  EFFT_ERR_HIP if the launch fails.
 * The arguments are checked on the host before anything is enqueued.
 */
int efft_stream_copy(void *dst, const void *src, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* EFFT_H */
