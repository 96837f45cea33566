// The staged pipeline on a library-owned, statically sized device scratch array, for callers
// that cannot allocate device memory (code under stream capture, serving loops, harnesses
// that forbid hipMalloc).
//
// The five stage kernels of grid_fd_grad_staged keep their intermediates (bias forces c, the
// factor L and 1/L_kk, dtau/du) in a per-knot workspace. Here that workspace is `scratch`, a
// file-scope device array of GRID_NOALLOC_SCRATCH_BYTES that lives as long as the process, one
// copy per device. Its device address is taken once per device with the device current
// (grid_noalloc_setup, called from grid_model_create) and passed to the kernels like the
// workspace pointer of the staged call; the array's own name is never used as an address on
// the host. Every stage writes what a later one reads, so nothing needs clearing between
// calls. Calls on one device share the array: calls that overlap in time on that device
// (different streams, or different host threads without ordering) race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "grid.h"
#include "grid_internal.h"

static __device__ __align__(256) float scratch[GRID_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float* g_ptr[kMaxDevices] = {};   // device address of `scratch` on each device, once known

}  // namespace

namespace grid_impl {

grid_status noalloc_setup(int device, std::string* err)
{
    if (device < 0 || device >= kMaxDevices) {
        *err = "device index out of range for the scratch array";
        return GRID_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device])
        return GRID_OK;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess)
        e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess)
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && !p)
        e = hipErrorInvalidSymbol;
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        *err = std::string("scratch array address: ") + hipGetErrorString(e);
        return GRID_EDEVICE;
    }
    g_ptr[device] = static_cast<float*>(p);
    return GRID_OK;
}

float* noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

}  // namespace grid_impl
