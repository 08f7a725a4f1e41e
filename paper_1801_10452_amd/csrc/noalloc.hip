// noalloc.hip -- the device scratch of the no-allocation batch entry point.
//
// raptor_trace_batch_noalloc keeps every device buffer of a launch that is neither an input nor
// an output (tile counter, statistics, job / grid / frequency / solid-angle tables, flux partial
// sums) in one file-scope array, so that the call itself allocates nothing.  Each GPU the
// library runs on holds its own copy of the array from the code object's load until the process
// ends.  Host code must not use the array's name as an address (that is a host-side stand-in):
// its device address is looked up here once per device and passed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mutex;
void* g_address[MAX_DEVICES] = {};

}  // namespace

hipError_t noalloc_scratch_address(int device, void** ptr)
{
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_address[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_address[device] = p;
    }
    *ptr = g_address[device];
    return hipSuccess;
}
