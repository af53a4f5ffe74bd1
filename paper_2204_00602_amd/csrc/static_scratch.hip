// The library's static device scratch area, for the entry points that must not
// allocate (slos_amplitudes_noalloc): callers under HIP graph capture, tight
// serving loops, or harnesses that forbid hipMalloc.
//
// `scratch` lives in the code object, so every GPU the library runs on holds
// its own copy from the first use until the process ends.  In host code its
// name is only a host-side stand-in; the device address of this GPU's copy
// comes from hipGetSymbolAddress, looked up once per device (with that device
// current) and kept.  Only that address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "slos_internal.h"

static __device__ __align__(256) unsigned char scratch[SLOS_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};
}  // namespace

int slos_static_scratch(void **ptr, int *device)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        g_addr[dev] = p;
    }
    *ptr = g_addr[dev];
    if (device) *device = dev;
    return 0;
}
