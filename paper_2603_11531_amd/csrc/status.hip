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

}  // namespace mgs

extern "C" const char *mgs_last_error(void) { return mgs::g_err; }
extern "C" const char *mgs_version(void) { return "mgs 0.1.0 gfx950"; }
