// epw_imsigma_noalloc: Im Sigma (Sec. 3 Eq. (8)) with its scratch in a
// library-owned device array instead of a caller workspace, for callers that
// cannot allocate device memory.
//
// `scratch` is a file-scope device array: every GPU the library runs this
// call on holds its own copy (EPW_NOALLOC_SCRATCH_BYTES) until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol): the device address of each GPU's copy
// is looked up once per device with hipGetSymbolAddress, with that device
// current, and kept; every use goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "epw_internal.h"

namespace epw {
namespace {

__device__ __align__(256) unsigned char scratch[EPW_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_addr[MAX_DEVICES] = {};

// Device address of the current device's scratch (looked up on first use).
void* scratch_base(int* rc) {
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *rc = fail(EPW_EHIP, "epw_imsigma_noalloc: hipGetDevice failed (%s)", hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= MAX_DEVICES) {
        *rc = fail(EPW_EHIP, "epw_imsigma_noalloc: device ordinal %d outside 0..%d", dev, MAX_DEVICES - 1);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void* p = nullptr;
        const hipError_t r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (r != hipSuccess || !p) {
            *rc = fail(EPW_EHIP, "epw_imsigma_noalloc: hipGetSymbolAddress of the scratch array failed on device %d "
                       "(%s)", dev, hipGetErrorString(r));
            return nullptr;
        }
        g_addr[dev] = p;
    }
    *rc = EPW_OK;
    return g_addr[dev];
}

}  // namespace
}  // namespace epw

extern "C" int epw_imsigma_noalloc(const epw_system* sys, const epw_points* pts, const epw_params* par,
                                   double* imsig, void* stream) {
    epw::clear_error();
    return epw::imsigma_in_buffer("epw_imsigma_noalloc", sys, pts, par, imsig, EPW_NOALLOC_SCRATCH_BYTES,
                                  &epw::scratch_base, stream);
}
