// Device memory of ftle_backward_noalloc: a fixed array in the library's code
// object instead of a workspace allocated at run time, for callers that cannot
// allocate (code under HIP graph capture, serving loops that forbid it).
//
// Each GPU the library runs on holds its own copy of the array (the runtime
// places it when it loads the code object on that device) until the process
// ends.  Host code never passes the array's name to a kernel: on the host the
// name is only a stand-in for the symbol.  The device address is looked up
// once per device, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ftle_internal.h"

static __device__ __align__(256) unsigned char scratch[ftle::kNoAllocScratchBytes];

namespace ftle {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void** ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes the device current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace ftle
