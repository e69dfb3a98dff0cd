// Fixed device workspace of sr_force_static: a file-scope device array, so a
// caller that cannot allocate (graph capture, a serving loop, a harness that
// forbids it) can still run the binning and the forward pair kernels.
//
// In host code the array's name is only a host-side stand-in: its device
// address comes from hipGetSymbolAddress, looked up once per device with
// that device current and kept here.  Every use on the host (kernel
// arguments, fills) goes through that pointer.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "sr_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[SR_STATIC_WORKSPACE_BYTES];

std::mutex g_mu;
std::vector<void *> g_ptr;  // device address of `scratch`, per device

}  // namespace

namespace sr {

hipError_t static_workspace(void **ptr, size_t *bytes)
{
    *ptr = nullptr;
    *bytes = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_mu);
    if ((int)g_ptr.size() <= dev) g_ptr.resize(dev + 1, nullptr);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    *bytes = SR_STATIC_WORKSPACE_BYTES;
    return hipSuccess;
}

}  // namespace sr
