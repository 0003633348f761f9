// Device scratch of the allocation-free operator entry point
// (tm_mat_pc_noalloc): a file-scope device array that every GPU the library
// runs on holds, at its own address, until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol); it resolves the device address once per device and uses that.
#include <mutex>

#include "tm_fields.h"

namespace twm {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_done[kMaxDevices];
void *g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];
}  // namespace

hipError_t noalloc_scratch(int device, void **ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[device]) {
        // the caller has made `device` current
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_err[device] = e;
        g_ptr[device] = (e == hipSuccess) ? p : nullptr;
        g_done[device] = true;
    }
    *ptr = g_ptr[device];
    return g_err[device];
}

}  // namespace twm
