// Work memory of the allocation-free solve (spx_solve_noalloc): one fixed
// array per device, in the library's code object, so that the call needs no
// device allocation.  Host code never passes the array's name to a kernel
// (in host code it names a host-side stand-in): scratch_region() takes the
// device address once per device with hipGetSymbolAddress, with that device
// current, and every user works with that address.
#include "device.hpp"

#include <mutex>

namespace spx {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_region(void** ptr, size_t* bytes)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = kScratchBytes;
    return hipSuccess;
}

}  // namespace spx
