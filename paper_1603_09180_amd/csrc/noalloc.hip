// noalloc.hip -- the library's static device scratch array, used by the
// entry point that allocates nothing (thin_run_noalloc).
//
// The array lives in the code object: the HIP runtime gives every device the
// library runs on its own copy, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address of each device's copy is
// looked up once per device with hipGetSymbolAddress, with that device
// current, and kept.
#include "thin_internal.h"

#include <mutex>

namespace thin {

namespace {

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_addr[kMaxDevices];  // device address of each device's copy (null: not looked up)

}  // namespace

hipError_t noalloc_scratch(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_lock);
    if (!g_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return hipSuccess;
}

}  // namespace thin
