// hrms_noalloc.hip -- the device scratch of hrms_run_1d_noalloc.
//
// The entry point that allocates nothing keeps its plan tables (spectrum
// descriptors, tile queues, statistics segments) and its per-call scratch
// (queue counters, statistics partials, SNR constants) in one static device
// array per GPU instead of buffers of its own. Its host-side address is a
// stand-in, not a device address, so the device address of each GPU's copy is
// looked up once per device with hipGetSymbolAddress and only that address is
// handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hrms_internal.h"

namespace hrms {
namespace {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
hipError_t g_status[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int device, void** ptr)
{
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
        g_status[device] = e;
        g_ptr[device] = e == hipSuccess ? p : nullptr;
        g_done[device] = true;
    }
    *ptr = g_ptr[device];
    return g_status[device];
}

}  // namespace hrms
