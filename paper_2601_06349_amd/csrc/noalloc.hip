// Entry point that allocates nothing: utf16wf_validate_batch_noalloc, the
// batch validation of utf16wf_validate_batch with its device flag in a
// file-scope device array instead of a workspace the library allocates.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address comes from hipGetSymbolAddress, looked up once per device
// (with that device current) on the entry point's first call there, and only
// that address is ever passed to a kernel or a copy.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/utf16wf.h"
#include "internal.h"

namespace {

// 256 bytes per device, held until the process ends; the validation uses
// the first int32 (its flag), whatever the size of the batch.
constexpr int kScratchWords = 64;
static __device__ __align__(256) int32_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu[kMaxDevices];       // one validation at a time per device
int32_t *g_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

}  // namespace

extern "C" int utf16wf_validate_batch_noalloc(const uint16_t *in, const uint16_t *out, const int64_t *offsets,
                                              int64_t num_strings, int64_t buf_units, void *stream) {
    using namespace utf16wf;
    int rc = check_validate_batch_args(in, out, offsets, num_strings, buf_units);
    if (rc != UTF16WF_OK)
        return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return set_error(UTF16WF_EHIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(UTF16WF_EHIP, "device ordinal out of range");
    // the call is synchronous; holding the device's lock for its duration
    // keeps two validations in this process off the one flag
    std::lock_guard<std::mutex> lk(g_mu[dev]);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess || !p)
            return set_error(UTF16WF_EHIP, "hipGetSymbolAddress(scratch) failed");
        g_ptr[dev] = static_cast<int32_t *>(p);
    }
    return validate_batch_with(in, out, offsets, num_strings, buf_units, (hipStream_t)stream, g_ptr[dev]);
}
