// Static device workspace of the allocation-free batch launch
// (ea_sweep_batch_noalloc): the work-queue counter, the job descriptors and
// the unit list of one launch, at the fixed offsets of ea_internal.h.  Every
// device the library runs on holds its own copy until the process ends.
#include <mutex>

#include "ea_internal.h"

namespace ea {

// The array's name is only a host-side handle: host code uses the device
// address that hipGetSymbolAddress returns for the current device, never the
// name itself.
static __device__ __align__(256) uint8_t scratch[kNoallocBytes];

hipError_t noalloc_workspace(void **ptr)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

}  // namespace ea
