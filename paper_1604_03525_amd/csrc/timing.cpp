// Optional per-stage kernel timing with HIP events (diagnostics only).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "epw_internal.h"

namespace epw {
namespace {

std::mutex g_mu;
bool g_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_rec[EPW_NUM_STAGES];

void drop_all_locked() {
    for (auto& v : g_rec) {
        for (auto& e : v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        v.clear();
    }
}

}  // namespace

StageTimer::StageTimer(int s, void* st) : stage(s), stream(st) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, (hipStream_t)stream) != hipSuccess) {
        (void)hipEventDestroy(e);
        return;
    }
    ev0 = (void*)e;
}

StageTimer::~StageTimer() {
    if (!ev0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t e1;
    if (hipEventCreate(&e1) != hipSuccess || hipEventRecord(e1, (hipStream_t)stream) != hipSuccess) {
        (void)hipEventDestroy((hipEvent_t)ev0);
        return;
    }
    g_rec[stage].push_back({(hipEvent_t)ev0, e1});
}

}  // namespace epw

extern "C" int epw_timing_enable(int enable) {
    using namespace epw;
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    drop_all_locked();
    g_on = enable != 0;
    return EPW_OK;
}

extern "C" int epw_timing_read(int stage, double* total_ms, int64_t* launches) {
    using namespace epw;
    clear_error();
    if (stage < 0 || stage >= EPW_NUM_STAGES || !total_ms || !launches)
        return fail(EPW_EINVAL, "epw_timing_read: bad stage %d or NULL output", stage);
    std::vector<std::pair<hipEvent_t, hipEvent_t>> rec;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        rec.swap(g_rec[stage]);
    }
    double t = 0.0;
    int rc = EPW_OK;
    for (auto& e : rec) {
        float ms = 0.f;
        if (rc == EPW_OK) {
            hipError_t err = hipEventSynchronize(e.second);
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e.first, e.second);
            if (err != hipSuccess)
                rc = fail(EPW_EHIP, "epw_timing_read: %s", hipGetErrorString(err));
        }
        t += ms;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    *total_ms = t;
    *launches = (int64_t)rec.size();
    return rc;
}
