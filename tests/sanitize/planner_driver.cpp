// Exercises the host side of libefft (planner, argument checks, error paths)
// under AddressSanitizer and UndefinedBehaviorSanitizer, on a host without a
// GPU: efft_schedule (the planner's dry run, no device needed) for every
// q <= 36, element type, placement and digit-buffer size; plan creation with
// valid and invalid arguments (valid ones fail cleanly at the first device
// allocation); every exec entry point with NULL and stale handles; chosen
// decompositions; the bandwidth reference's argument checks.  Exits 0 when
// every call returned a status its contract allows.
#include <cstdio>
#include <cstdint>
#include <vector>

#include "efft.h"

static int failures = 0;
#define EXPECT(cond, ...)                        \
    do {                                         \
        if (!(cond)) {                           \
            std::fprintf(stderr, "FAIL: " __VA_ARGS__); \
            std::fprintf(stderr, "\n");          \
            ++failures;                          \
        }                                        \
    } while (0)

int main()
{
    // the planner's dry run at every size, with too small digit buffers too
    for (int q = -1; q <= 36; ++q) {
        const int64_t n = q < 0 ? 0 : (int64_t(1) << q);
        for (int dtype = 0; dtype <= 3; ++dtype) {
            for (int inplace = 0; inplace <= 1; ++inplace) {
                for (int maxd : {0, 1, 2, 8}) {
                    std::vector<int> d(size_t(maxd > 0 ? maxd : 1), -7);
                    int passes = -1;
                    const int m = efft_schedule(n, dtype, inplace, maxd ? d.data() : nullptr, maxd, &passes);
                    const bool valid = (dtype == EFFT_C64 || dtype == EFFT_C128) && q >= 0 && q <= EFFT_MAX_LOG2N;
                    if (!valid) {
                        EXPECT(m < 0, "schedule q=%d dtype=%d accepted", q, dtype);
                    } else if (m > 0) {
                        int sum = 0;
                        for (int i = 0; i < m; ++i) sum += d[size_t(i)];
                        EXPECT(sum == q && passes >= m, "schedule q=%d digits sum %d passes %d", q, sum, passes);
                    }
                }
            }
        }
    }
    // plan creation: invalid arguments, then valid ones (no device: the
    // first device allocation fails and the call returns NULL cleanly)
    const int64_t sizes[] = {0, 1, 2, 3, 12, 1000, 1024, (int64_t(1) << 20) + 1, int64_t(1) << 30, int64_t(1) << 35};
    for (int64_t n : sizes) {
        for (int dtype = 0; dtype <= 3; ++dtype) {
            for (int dir : {-2, -1, 0, 1}) {
                efft_plan_t *p = efft_plan(n, dtype, dir, 1);
                if (p) efft_destroy(p);
                const int e = efft_last_error();
                EXPECT(p != nullptr || e < 0, "plan n=%lld failed without a status", (long long)n);
                p = efft_plan_many(n, 3, dtype, dir, 0, 0.5);
                if (p) efft_destroy(p);
                p = efft_plan_real(n, dtype, dir, 1.0);
                if (p) efft_destroy(p);
            }
        }
    }
    const int dg[][4] = {{10, 10, 10, 0}, {4, 26, 0, 0}, {9, 8, 8, 9}, {11, 8, 11, 0}, {3, 3, 0, 0}};
    const int dn[] = {3, 2, 4, 3, 2};
    for (int i = 0; i < 5; ++i) {
        int q = 0;
        for (int j = 0; j < dn[i]; ++j) q += dg[i][j];
        efft_plan_t *p = efft_plan_digits(int64_t(1) << q, 1, EFFT_C128, EFFT_FORWARD, 1, 1.0, dg[i], dn[i]);
        if (p) efft_destroy(p);
        EXPECT(efft_last_error() <= 0, "plan_digits status");
    }
    EXPECT(efft_plan_digits(1024, 1, EFFT_C64, EFFT_FORWARD, 1, 1.0, nullptr, 2) == nullptr, "NULL digits");
    // exec entry points on NULL and foreign handles
    alignas(16) static char buf[4096];
    efft_plan_t *bogus = reinterpret_cast<efft_plan_t *>(buf);
    EXPECT(efft_exec(nullptr, buf, nullptr) == EFFT_ERR_NULLPTR, "exec NULL plan");
    EXPECT(efft_exec(bogus, buf, nullptr) == EFFT_ERR_BADPLAN, "exec foreign handle");
    EXPECT(efft_exec_oop(bogus, buf, buf + 1024, nullptr) == EFFT_ERR_BADPLAN, "oop foreign handle");
    EXPECT(efft_exec_scratch(bogus, buf, buf + 1024, nullptr) == EFFT_ERR_BADPLAN, "scratch foreign handle");
    EXPECT(efft_exec_noalloc(bogus, buf, nullptr) == EFFT_ERR_BADPLAN, "noalloc foreign handle");
    EXPECT(efft_exec_noalloc(nullptr, buf, nullptr) == EFFT_ERR_NULLPTR, "noalloc NULL plan");
    void *ev[2] = {nullptr, nullptr};
    EXPECT(efft_exec_events(bogus, buf, buf, nullptr, nullptr, ev, 2) == EFFT_ERR_BADPLAN, "events foreign handle");
    EXPECT(efft_destroy(nullptr) == EFFT_OK, "destroy NULL");
    EXPECT(efft_destroy(bogus) == EFFT_ERR_BADPLAN, "destroy foreign handle");
    EXPECT(efft_plan_passes(bogus) == -1 && efft_plan_bytes(bogus) == -1 && efft_scratch_bytes(bogus) == -1,
           "queries on a foreign handle");
    int opts[6] = {0};
    EXPECT(efft_pass_options(bogus, 0, 0, opts) < 0, "pass options foreign handle");
    for (int s = -20; s <= 2; ++s) EXPECT(efft_strerror(s) != nullptr, "strerror %d", s);
    // the bandwidth reference's host-side checks (nothing is launched)
    EXPECT(efft_stream_copy(nullptr, buf, 16, nullptr) == EFFT_ERR_NULLPTR, "copy NULL");
    EXPECT(efft_stream_copy(buf + 8, buf + 2048, 16, nullptr) == EFFT_ERR_ALIGN, "copy misaligned");
    EXPECT(efft_stream_copy(buf, buf + 16, 64, nullptr) == EFFT_ERR_OVERLAP, "copy overlap");
    EXPECT(efft_stream_copy(buf, buf + 2048, -16, nullptr) == EFFT_ERR_ARG, "copy negative");
    EXPECT(efft_stream_copy(buf, buf + 2048, 0, nullptr) == EFFT_OK, "copy empty");
    if (failures) {
        std::fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    std::printf("planner driver ok\n");
    return 0;
}
