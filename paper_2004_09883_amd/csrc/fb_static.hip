// fb_static.hip -- the staging buffer of the allocation-free host-buffer
// transform (fb_fft3d_exec_host_noalloc): a file-scope device array of
// FB_STATIC_SCRATCH_BYTES that every GPU the library runs on holds from the
// moment the code object is loaded until the process ends.
//
// In host code the array's name is only a stand-in for the symbol, not a
// device address: the address of each device's copy is looked up once per
// device with hipGetSymbolAddress (with that device current) and cached, and
// only that address is handed to copies and kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fb.h"
#include "fb_internal.hpp"

static __device__ __align__(256) unsigned char scratch[FB_STATIC_SCRATCH_BYTES];

namespace fb {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void **ptr)
{
    *ptr = nullptr;
    int dev = -1;
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

}  // namespace fb
