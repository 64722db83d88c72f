// Error reporting for the C ABI: a thread-local message plus the return code.
#include <stdarg.h>
#include <stdio.h>

#include "common.h"

namespace mgs {

static thread_local char g_err[512] = "no error";

int set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#ifdef MGS_CHECK_BOUNDS
struct BoundsWord {
    int (*read)(uint32_t *);
    int (*clear)();
};
static BoundsWord g_bounds[32];
static int g_n_bounds = 0;
void register_bounds_word(int (*read)(uint32_t *), int (*clear)()) {
    if (g_n_bounds < 32) g_bounds[g_n_bounds++] = BoundsWord{read, clear};
}
#endif

}  // namespace mgs

extern "C" int mgs_bounds_checked(void) {
#ifdef MGS_CHECK_BOUNDS
    return 1;
#else
    return 0;
#endif
}

extern "C" int mgs_bounds_status(uint32_t *flags, int clear) {
    using namespace mgs;
    MGS_REQUIRE(flags != nullptr, "flags is NULL");
    *flags = 0;
#ifdef MGS_CHECK_BOUNDS
    if (hipDeviceSynchronize() != hipSuccess) return set_error(MGS_ERR_HIP, "hipDeviceSynchronize failed");
    for (int i = 0; i < g_n_bounds; ++i) {
        uint32_t v = 0;
        if (g_bounds[i].read(&v) != 0) return set_error(MGS_ERR_HIP, "reading a bounds word failed");
        *flags |= v;
        if (clear && g_bounds[i].clear() != 0) return set_error(MGS_ERR_HIP, "clearing a bounds word failed");
    }
#else
    (void)clear;
#endif
    return MGS_OK;
}

extern "C" int mgs_check_capacity(const uint32_t *n_pairs, uint64_t capacity, uint64_t *pairs, void *stream) {
    using namespace mgs;
    MGS_REQUIRE(n_pairs != nullptr, "n_pairs is NULL");
    uint32_t P = 0;
    const hipStream_t s = as_stream(stream);
    if (hipMemcpyAsync(&P, n_pairs, sizeof(P), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return set_error(MGS_ERR_HIP, "reading the pair count failed: %s", hipGetErrorString(hipGetLastError()));
    if (pairs) *pairs = P;
    if (uint64_t(P) > capacity)
        return set_error(MGS_ERR_CAPACITY, "%u tile/Gaussian pairs exceed the capacity of %llu", P,
                         (unsigned long long)capacity);
    return MGS_OK;
}

extern "C" const char *mgs_last_error(void) { return mgs::g_err; }
extern "C" const char *mgs_version(void) { return "mgs 0.1.0 gfx950"; }
