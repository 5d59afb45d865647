// The control step that allocates nothing: every buffer of the controller's workspace
// lives in a file-scope device array of MPPI_STATIC_SCRATCH_BYTES per GPU, held until the
// process ends.  Host code never passes the array's name to a kernel (in host code that
// name stands for a host-side symbol): the array's device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and that address is used.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mppi.h"
#include "policy_internal.h"

namespace {

constexpr size_t kScratchBytes = MPPI_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// the scratch array's address on the current device (looked up on first use)
hipError_t scratch_ptr(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" mppi_status mppi_step_static(mppi_ctx* ctx, const float* d_x0, float* d_nominal, float* d_u0_out,
                                        void* hip_stream)
{
    void* p = nullptr;
    if (scratch_ptr(&p) != hipSuccess) return mppi_host::step_in_region(ctx, nullptr, 0, d_x0, d_nominal, d_u0_out,
                                                                         (hipStream_t)hip_stream);
    return mppi_host::step_in_region(ctx, p, kScratchBytes, d_x0, d_nominal, d_u0_out, (hipStream_t)hip_stream);
}
