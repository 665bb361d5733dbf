// efft_stream.hip -- the memory-bandwidth reference of the benchmark.
//
// The paper sets EFFT beside the STREAM benchmark to judge how well a
// bandwidth-bound transform uses the memory system (Section 5.4,
// Fig. "fig:parallel-perf").  The GPU counterpart is a plain streaming copy
// with the access style of the transform's passes: 16-byte loads and stores
// with the non-temporal hint, consecutive lanes on consecutive addresses,
// four independent loads in flight per thread.  With dst == src it rewrites
// the range in place, the pattern of an in-place pass.
#include <hip/hip_runtime.h>

#include "../../include/efft.h"
#include "efft_internal.hpp"

namespace efft {
namespace {

constexpr int BT = 256;
constexpr int UNROLL = 4;  // measured on gfx950: 8 and 16 are 5-10% slower

__global__ void __launch_bounds__(BT) stream_copy_kernel(double2 *dst, const double2 *src, int64_t n)
{
    const int64_t step = int64_t(gridDim.x) * BT * UNROLL;
    for (int64_t base = int64_t(blockIdx.x) * BT * UNROLL + threadIdx.x; base < n; base += step) {
        double2 v[UNROLL];
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
    int64_t blocks = (n + per_block - 1) / per_block;
    if (blocks > (int64_t(1) << 20)) blocks = int64_t(1) << 20;
    hipLaunchKernelGGL(efft::stream_copy_kernel, dim3(unsigned(blocks)), dim3(efft::BT), 0,
                       static_cast<hipStream_t>(stream), static_cast<double2 *>(dst),
                       static_cast<const double2 *>(src), n);
    return hipGetLastError() == hipSuccess ? EFFT_OK : EFFT_ERR_HIP;
}
