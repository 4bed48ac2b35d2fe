// Error reporting for the C ABI: a thread-local message plus status codes.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>

#include "epw_internal.h"

namespace epw {

static thread_local char g_msg[1024] = {0};

void clear_error() { g_msg[0] = 0; }

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

void hip_check(int err, const char* call, const char* file, int line) {
    if (err != (int)hipSuccess) throw HipFailure{err, call, file, line};
}

void launch_check(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw HipFailure{(int)e, what, __FILE__, __LINE__};
}

}  // namespace epw

extern "C" const char* epw_last_error(void) { return epw::g_msg; }

extern "C" int epw_version(void) { return 100; }
