// noalloc.hip -- the fixed device workspace of pt_batch_loglik_noalloc.
//
// A file-scope device array, one copy per GPU the library runs on, held
// until the process ends.  Host code never uses the array's name as a
// device address: its address on each device is looked up once, with that
// device current, by noalloc_workspace(), and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace pt {

namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];
bool g_done[kMaxDevices];

}  // namespace

hipError_t noalloc_workspace(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if ((e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        (void)hipSetDevice(prev);
        if (e != hipSuccess) return e;
        g_ptr[device] = p;
        g_done[device] = true;
    }
    *out = g_ptr[device];
    return hipSuccess;
}

}  // namespace pt
