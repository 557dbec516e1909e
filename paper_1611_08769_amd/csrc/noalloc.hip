// The encrypted FFT with its workspace in a fixed array of this library's
// device memory, for callers that cannot allocate device memory (code under
// stream capture, tight serving loops, harnesses that forbid it).
//
// The array `scratch` (SFFT_NOALLOC_WS_BYTES) is a file-scope __device__
// variable: every GPU the library runs on holds its own copy until the
// process ends.  In host code its name is only a stand-in, so the device
// address is taken once per device with hipGetSymbolAddress (with that device
// current, on the first call there) and kept; kernels get that address.
// Nothing in the workspace needs clearing: every slot and every transposed
// right operand is written before it is read.  All calls on one GPU share
// the array, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/sfft.h"
#include "plan_internal.hpp"

namespace {

static __device__ __align__(256) uint8_t scratch[SFFT_NOALLOC_WS_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

}  // namespace

extern "C" int sfft_execute_noalloc(const sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev,
                                    void* hip_stream)
{
    if (!plan) return sfft_fail(SFFT_EINVAL, "null plan");
    int64_t need = 0;
    int rc = sfft_plan_workspace_bytes(plan, &need);
    if (rc != SFFT_OK) return rc;
    if (need > (int64_t)SFFT_NOALLOC_WS_BYTES)
        return sfft_fail(SFFT_ENOMEM, "the plan's workspace (" + std::to_string(need) +
                                          " bytes) exceeds the fixed array of sfft_execute_noalloc (" +
                                          std::to_string((int64_t)SFFT_NOALLOC_WS_BYTES) + " bytes)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sfft_hip_fail(e, "current device");
    if (dev < 0 || dev >= kMaxDevices) return sfft_fail(SFFT_EUNSUPPORTED, "device index out of range");
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return sfft_hip_fail(e, "address of the fixed workspace");
            g_scratch_ptr[dev] = p;
        }
        ws = g_scratch_ptr[dev];
    }
    return sfft_execute(plan, ct_in_dev, ct_out_dev, ws, (int64_t)SFFT_NOALLOC_WS_BYTES, hip_stream);
}
