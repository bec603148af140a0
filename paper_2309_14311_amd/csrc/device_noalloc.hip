// device_noalloc.hip -- nasch_grid_step_device_noalloc: the device-buffer step
// of device_api.hip for callers that must not allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  Its only
// scratch, the per-block F(t) partials, lives in a file-scope device array
// instead of a stream-ordered allocation; the call itself allocates nothing.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress (with
// that device current) and kept, and only that address is handed to kernels.
// Every call on a device shares the device's array and leaves its contents
// behind; calls that overlap on one device race for it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "engine.hpp"
#include "nasch.h"

using namespace nasch;

namespace {
// One uint32 F(t) partial per block of 8 tiles (one per wave) of 1984 cells,
// for the longest ring (L = 2^31 - 1): about 0.5 MiB.
constexpr uint32_t kTileCells = 32u * (64u * kOneStepQ - 2u);
constexpr uint32_t kTilesPerBlock = kOneStepThreads / 64u;
constexpr uint32_t kScratchWords = (uint32_t)(((NASCH_MAX_L + kTileCells - 1u) / kTileCells +
                                               kTilesPerBlock - 1u) / kTilesPerBlock);
}  // namespace

// The scratch of every call on a device: the F(t) partials of the step's
// blocks, each written before the fold reads it.
static __device__ __align__(256) uint32_t scratch[kScratchWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
hipError_t scratch_on_current_device(uint32_t** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int nasch_grid_step_device_noalloc(const uint8_t* d_in, uint8_t* d_out, uint64_t L,
                                   uint32_t vmax, double p, uint64_t seed, uint32_t replica,
                                   uint64_t t, uint64_t* d_flux, void* stream) {
    RingDesc R;
    int rc = describe_device_ring(d_in, d_out, L, vmax, p, seed, replica, t, &R);
    if (rc) return rc;
    if (onestep_partials(R.ntiles) > kScratchWords) return NASCH_EINVAL;   // beyond the scratch
    uint32_t* partials = nullptr;
    hipError_t e = scratch_on_current_device(&partials);
    if (e == hipSuccess)
        e = launch_grid_onestep_direct(R, partials, (uint32_t)t,
                                       reinterpret_cast<unsigned long long*>(d_flux),
                                       (hipStream_t)stream);
    if (e != hipSuccess) {
        thread_last_hip_error() = (int)e;
        return NASCH_EDEVICE;
    }
    return NASCH_OK;
}

}  // extern "C"
