// device_api.hip -- one time step of a ring whose road lives in caller-owned
// device memory (nasch_grid_step_device, include/nasch.h): no handle, no state
// in the library.  A caller that keeps its roads in its own buffers (torch
// tensors, an arena of its own) steps them in place of nasch_init /
// nasch_step_n.  The step is the one-step kernel (grid_onestep.hip) launched
// on a ring described by value; F(t) is folded from per-block sums into the
// caller's uint64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "engine.hpp"
#include "nasch.h"

using namespace nasch;

namespace nasch {

// Validates the arguments of a device-buffer step and describes the ring.
int describe_device_ring(const uint8_t* d_in, const uint8_t* d_out, uint64_t L, uint32_t vmax,
                         double p, uint64_t seed, uint32_t replica, uint64_t t, RingDesc* R) {
    int rc = validate_params(L, 0, vmax, p);
    if (rc) return rc;
    if (!d_in || !d_out) return NASCH_EINVAL;
    const uintptr_t a = (uintptr_t)d_in, b = (uintptr_t)d_out;
    if (((a | b) & 15u) != 0u) return NASCH_EINVAL;   // 16-byte loads and stores
    if (a < b + L && b < a + L) return NASCH_EINVAL;  // the two roads overlap
    if (t >= 0xFFFFFFFFull) return NASCH_ERANGE;       // t + 1 must stay below 2^32
    RingDesc r{};
    r.buf[0] = const_cast<uint8_t*>(d_in);
    r.buf[1] = const_cast<uint8_t*>(d_out);
    r.L = (uint32_t)L;
    r.vmax = vmax;
    r.nw = plane_words(L);
    r.sp = slow_params(seed, replica, p);
    r.t_end = 0xFFFFFFFFu;
    r.warmup = ~0ull;
    onestep_geometry(r.L, kOneStepQ, &r.own, &r.halo, &r.ntiles);
    *R = r;
    return NASCH_OK;
}

}  // namespace nasch

namespace {

int device_error(hipError_t e) {
    thread_last_hip_error() = (int)e;
    return NASCH_EDEVICE;
}

}  // namespace

extern "C" {

int nasch_grid_step_device(const uint8_t* d_in, uint8_t* d_out, uint64_t L, uint32_t vmax,
                           double p, uint64_t seed, uint32_t replica, uint64_t t,
                           uint64_t* d_flux, void* stream) {
    RingDesc R;
    int rc = describe_device_ring(d_in, d_out, L, vmax, p, seed, replica, t, &R);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    uint32_t* partials = nullptr;
    const size_t words = onestep_partials(R.ntiles);
    hipError_t e = hipMallocAsync((void**)&partials, words * sizeof(uint32_t), s);
    if (e != hipSuccess) {
        thread_last_hip_error() = (int)e;
        return NASCH_ENOMEM;
    }
    e = launch_grid_onestep_direct(R, partials, (uint32_t)t,
                                   reinterpret_cast<unsigned long long*>(d_flux), s);
    const hipError_t ef = hipFreeAsync(partials, s);
    if (e != hipSuccess) return device_error(e);
    if (ef != hipSuccess) return device_error(ef);
    return NASCH_OK;
}

}  // extern "C"
