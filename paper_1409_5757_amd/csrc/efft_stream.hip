// efft_stream.hip -- the memory-bandwidth reference of the benchmark.
//
// The paper sets EFFT beside the STREAM benchmark to assess how well a
// bandwidth-bound transform uses the memory system (Section 5.4,
// Fig. "fig:parallel-perf").  The GPU counterpart is a plain streaming copy
// with the access style of the transform's passes: 16-byte loads and stores
// with the non-temporal hint, consecutive lanes on consecutive addresses,
// each workgroup loading its whole chunk before storing it, and as many
// workgroups per CU as the passes have.  With dst == src it rewrites the
// range in place, the pattern of an in-place pass.
#include <hip/hip_runtime.h>

#include "../../include/efft.h"
#include "efft_internal.hpp"

namespace efft {
namespace {

constexpr int BT = 256;

// One workgroup copies one contiguous chunk of BT * UNROLL 16-byte elements:
// every thread issues all UNROLL loads (consecutive lanes on consecutive
// addresses, one wave-wide 1 KiB run per load), then all UNROLL stores, the
// access pattern of a contiguous-line pass, and the workgroup ends (the
// hardware refills the CU with the next chunk).  The tail chunk is guarded.
template <int UNROLL>
__global__ void __launch_bounds__(BT) stream_copy_kernel(double2 *dst, const double2 *src, int64_t n)
{
    const int64_t base = int64_t(blockIdx.x) * BT * UNROLL + threadIdx.x;
    double2 v[UNROLL];
    if (base + int64_t(BT) * (UNROLL - 1) < n) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) v[u] = load_nt(src + base + int64_t(u) * BT);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) store_nt(dst + base + int64_t(u) * BT, v[u]);
    } else {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t i = base + int64_t(u) * BT;
            if (i < n) v[u] = load_nt(src + i);
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t i = base + int64_t(u) * BT;
            if (i < n) store_nt(dst + i, v[u]);
        }
    }
}

// Two 16-byte loads per thread (8 KiB per workgroup) and 40 KiB of LDS
// reserved per workgroup (unused; it caps a CU at four workgroups, as the
// exchange buffers of the transform's passes cap them).  Measured on gfx950,
// copying 8 GiB: 6.47 TB/s, against 6.05 (4 loads, same cap), 5.84 (4 loads,
// no cap), 5.74 (8 loads), 5.51 (16 loads, no cap) and 5.16 (16 loads, two
// workgroups per CU); the grid-stride loop with 4 loads it replaces ran at
// 5.78.
#ifndef EFFT_COPY_UNROLL
#define EFFT_COPY_UNROLL 2
#endif
constexpr int UNROLL = EFFT_COPY_UNROLL;
#ifndef EFFT_COPY_LDS_KB
#define EFFT_COPY_LDS_KB 40
#endif

}  // namespace
}  // namespace efft

extern "C" int efft_stream_copy(void *dst, const void *src, int64_t bytes, void *stream)
{
    if (!dst || !src) return EFFT_ERR_NULLPTR;
    if (reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16) return EFFT_ERR_ALIGN;
    if (bytes < 0 || bytes % 16) return EFFT_ERR_ARG;
    const uintptr_t d = reinterpret_cast<uintptr_t>(dst), s = reinterpret_cast<uintptr_t>(src);
    // dst == src rewrites the range in place (the access pattern of an
    // in-place pass); any other overlap is refused
    if (bytes > 0 && d != s && d < s + uintptr_t(bytes) && s < d + uintptr_t(bytes)) return EFFT_ERR_OVERLAP;
    if (bytes == 0) return EFFT_OK;
    const int64_t n = bytes / 16;
    const int64_t per_block = int64_t(efft::BT) * efft::UNROLL;
    const int64_t blocks = (n + per_block - 1) / per_block;
    if (blocks > int64_t(0x7fffffff)) return EFFT_ERR_ARG;  // beyond one grid (> 128 TiB)
    hipLaunchKernelGGL(efft::stream_copy_kernel<efft::UNROLL>, dim3(unsigned(blocks)), dim3(efft::BT),
                       EFFT_COPY_LDS_KB * 1024,
                       static_cast<hipStream_t>(stream), static_cast<double2 *>(dst),
                       static_cast<const double2 *>(src), n);
    return hipGetLastError() == hipSuccess ? EFFT_OK : EFFT_ERR_HIP;
}
