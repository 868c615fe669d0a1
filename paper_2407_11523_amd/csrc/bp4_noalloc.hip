// bp4_decode_mixed_noalloc: the persistent mixed-code decode for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).  Its
// only scratch memory, the per-code shot-queue heads, lives in a file-scope device
// array instead of a caller workspace; the library calls no allocator for it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bp4.h"
#include "bp4_internal.h"

// Shot-queue heads of one mixed launch: one word per code (at most
// BP4_MAX_MIXED_CODES of the 64 are used).  Every GPU holds its own copy, at its own
// address, until the process ends; every call on that GPU shares it.
static_assert(BP4_MAX_MIXED_CODES <= 64, "queue heads exceed the static scratch array");
static __device__ __align__(256) unsigned int scratch[64];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned int *g_scratch[kMaxDevices] = {};   // device address of `scratch` per device

// The device address of this GPU's `scratch`, looked up once per device.  The array's
// name is only a host-side stand-in: kernels and fills get this address.
int scratch_of_current_device(unsigned int **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return bp4::report_error(BP4_EHIP, "decode_mixed_noalloc: hipGetDevice", e);
    if (dev < 0 || dev >= kMaxDevices) return bp4::report_error(BP4_EUNSUPPORTED, "decode_mixed_noalloc: device index above 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return bp4::report_error(BP4_EHIP, "decode_mixed_noalloc: hipGetSymbolAddress(scratch)", e);
        g_scratch[dev] = static_cast<unsigned int *>(ptr);
    }
    *out = g_scratch[dev];
    return BP4_OK;
}

}  // namespace

extern "C" int bp4_decode_mixed_noalloc(int32_t ncodes, const bp4_code_batch *codes, void *stream)
{
    if (ncodes < 1 || ncodes > BP4_MAX_MIXED_CODES)
        return bp4::report_error(BP4_EINVAL, "decode_mixed_noalloc: ncodes outside [1, BP4_MAX_MIXED_CODES = 16]");
    unsigned int *heads = nullptr;
    int rc = scratch_of_current_device(&heads);
    if (rc) return rc;
    return bp4::decode_mixed_with(ncodes, codes, heads, stream);
}
