// noalloc.hip -- the library's static work space: device memory that comes
// with the loaded code object, for the one run call that must not allocate
// (stencil_run_noalloc).  Each device the library runs on holds its own copy
// of the array from the first such call until the process ends.
#include <mutex>

#include "internal.h"

namespace st {

namespace {

// Ping-pong buffer of stencil_run_noalloc: one grid's worth of cells.
static __device__ __align__(256) unsigned char scratch[kStaticWorkBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// The device address of `scratch` on the current device.  The array's name
// in host code is only a host-side handle, so the address is asked of the
// runtime once per device (with that device current) and kept.
hipError_t static_work(void** ptr, size_t* bytes) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    *bytes = kStaticWorkBytes;
    return hipSuccess;
}

}  // namespace st
