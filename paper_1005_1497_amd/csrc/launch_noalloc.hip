// The library's static device scratch, for the entry point that allocates
// nothing (conv_circular_noalloc): the four-step convolution's 2N scratch
// words live in a file-scope device array instead of a per-stream workspace.
//
// Each device that runs the library holds its own copy of `scratch` at its own
// address, from code-object load until the process ends.  Host code never
// uses the array's name as an address (on the host it is only a stand-in
// symbol): the device address is looked up once per device, with that device
// current, by hipGetSymbolAddress, and kept here.  Every call on a device
// shares that device's array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.hpp"

namespace nttmi {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {nullptr};   // device address of `scratch`, per device
}  // namespace

hipError_t noalloc_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace nttmi
