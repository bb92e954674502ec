// The library's static device scratch: the memory of the allocation-free
// entry point (tfft_exec_noalloc), which holds the report counters, the
// records and the multi-pass workspace of an execution there instead of in
// buffers the plan allocated.  Each device that loads the library holds one
// copy of the array, at its own address, until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tfft_internal.h"

namespace tfft {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on `device`, which must be the current device.
// Looked up once per device with hipGetSymbolAddress (in host code the
// array's name is only a host-side stand-in, never a device address) and
// kept; NULL if the lookup fails.
void *scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_addr[device] = ptr;
    }
    return g_addr[device];
}

}  // namespace tfft
