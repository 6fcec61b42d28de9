// Static device scratch of the allocation-free potential gradient
// (mwu_potential_backward_noalloc): the reduction records and chunk partials
// of its passes live in one file-scope device array per GPU instead of
// buffers the library allocates.  The array is held by each GPU the library
// runs on until the process ends; every call on that GPU shares it, so calls
// that overlap on one GPU race.  No kernel needs it cleared: every record and
// partial is written by its pass before the pass's finisher reads it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.h"

namespace mwu {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this GPU's copy of the array (the device must be
// current).  In host code the array's name is only a stand-in: kernels get
// the address hipGetSymbolAddress returns, looked up once per device.
void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) throw ApiError{MWU_ERR_INVALID_ARG, "device ordinal out of range"};
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) throw DeviceError(e, "hipGetSymbolAddress(scratch)");
        g_ptr[device] = p;
    }
    return g_ptr[device];
}

}  // namespace mwu
