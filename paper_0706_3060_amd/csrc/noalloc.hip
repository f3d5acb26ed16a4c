// The device-resident scratch area of the allocation-free forward entry point
// (nbody_forces_noalloc): a file-scope device array that each GPU the library
// runs on holds until the process ends.  Host code never passes the array's
// name to a kernel or a copy (in host code it is a stand-in, not a device
// address); it asks for the device address once per device, with that device
// current, and uses that address from then on.
#include <mutex>

#include "noalloc.h"

namespace nbk {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_area(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace nbk
