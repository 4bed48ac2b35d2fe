// Internal declarations shared by the libepw translation units.
#pragma once

#include <cstddef>
#include <cstdint>

#include "epw.h"

namespace epw {

// ---- error reporting (thread-local message, see epw_last_error) ----
void clear_error();
int fail(int code, const char* fmt, ...);

// Thrown by host orchestration code on a HIP runtime failure; caught at the
// ABI boundary and turned into EPW_EHIP.
struct HipFailure {
    int code;
    const char* call;
    const char* file;
    int line;
};
void hip_check(int err, const char* call, const char* file, int line);
#define EPW_HIP(call) ::epw::hip_check((int)(call), #call, __FILE__, __LINE__)
// check the last kernel launch
void launch_check(const char* what);

// ---- stage timing (see epw_timing_enable) ----
// Usage: { StageTimer t(EPW_STAGE_FUSED, stream); launch...; }  records an
// event pair around the launches in scope when timing is enabled.
struct StageTimer {
    int stage;
    void* stream;
    void* ev0 = nullptr;
    StageTimer(int stage, void* stream);
    ~StageTimer();
};

// ---- caller-provided workspace, carved in 256-byte aligned pieces ----
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    bool dry = false;          // size query: count only
    void* take(size_t bytes) {
        used = (used + 255) & ~(size_t)255;
        void* p = dry ? nullptr : (void*)(base + used);
        used += bytes;
        return p;
    }
};

// Im Sigma (epw_imsigma) with its workspace in a fixed device buffer of cap
// bytes: checks the arguments, picks the largest q chunk that fits (or
// checks the given one) and only then calls base() for the buffer's device
// address (base sets *rc and returns nullptr on failure).
int imsigma_in_buffer(const char* fn, const epw_system* sys, const epw_points* pts, const epw_params* par,
                      double* imsig, size_t cap, void* (*base)(int* rc), void* stream);

// smallest power of two >= n (n >= 1)
inline int pow2_at_least(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

}  // namespace epw
