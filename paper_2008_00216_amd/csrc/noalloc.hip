// A fixed device work area for the entry point that allocates nothing
// (sv_expect_noalloc): callers that cannot allocate device memory -- code
// under HIP graph capture, tight serving loops -- get their reduction
// partials, Pauli tables and results from this array instead of buffers the
// library allocates.
//
// The array is a file-scope __device__ object: every GPU that loads the
// library holds its own copy, at its own address, until the process ends.
// In host code its name is only a host-side stand-in, so the device address
// is looked up once per device with hipGetSymbolAddress and kept; kernels
// receive that address as an ordinary pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace svmi {

namespace {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t static_scratch(void** ptr) {
    *ptr = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}

}  // namespace svmi
