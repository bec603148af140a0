// valu_probe.hip -- throughput of the vector-ALU instructions the step kernels
// are made of, measured on the device, and the shader clock during the run.
//
// The step kernels do no floating point and no matrix work: their bound is the
// rate at which the SIMDs issue 32-bit integer instructions.  The nominal
// figure (256 CU x 4 SIMD x 16 lanes per cycle x 2.4 GHz) assumes one wave64
// instruction per SIMD every 4 cycles for every instruction; this probe
// measures what each instruction kind actually sustains.  Every lane runs
// kChains independent dependency chains of one instruction kind, enough waves
// run to fill every SIMD, and the launch is timed with HIP events.  One lane
// per block also reads the shader clock counter (s_memtime) and the constant
// 100 MHz counter (s_memrealtime) at its start and end, so the host can derive
// the clock the SIMDs actually ran at.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>

#include "nasch_probe.h"

namespace {

constexpr int kChains = 8;     // independent chains per lane
constexpr int kUnroll = 16;    // instructions per chain and loop iteration

template <int OP>
__device__ __forceinline__ uint32_t op(uint32_t a, uint32_t b, uint32_t c) {
    if constexpr (OP == NASCH_PROBE_BITOP3) {
        return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
    } else if constexpr (OP == NASCH_PROBE_ALIGNBIT) {
        return __builtin_amdgcn_alignbit(a, b, c);
    } else if constexpr (OP == NASCH_PROBE_BCNT) {
        return __builtin_popcount(a) + b;
    } else if constexpr (OP == NASCH_PROBE_MUL_LO) {
        return a * b;
    } else if constexpr (OP == NASCH_PROBE_MUL_HI) {
        return __umulhi(a, b);
    } else if constexpr (OP == NASCH_PROBE_DPP) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a, 0x130 /* wave_shl:1 */, 0xf, 0xf,
                                                     true);
    } else if constexpr (OP == NASCH_PROBE_ADD) {
        return a + b;
    } else if constexpr (OP == NASCH_PROBE_XOR) {
        return a ^ b;
    } else if constexpr (OP == NASCH_PROBE_SHIFT) {
        return a << c;
    } else if constexpr (OP == NASCH_PROBE_LSHL_OR) {
        return (a << 3) | b;
    } else if constexpr (OP == NASCH_PROBE_PERM) {
        return __builtin_amdgcn_perm(a, b, 0x05010400u);
    } else if constexpr (OP == NASCH_PROBE_MUL_U24) {
        return __umul24(a, b);
    } else if constexpr (OP == NASCH_PROBE_MIN) {
        return min(a, b);
    } else if constexpr (OP == NASCH_PROBE_SUB) {
        return a - b;
    } else if constexpr (OP == NASCH_PROBE_AND_OR) {
        return (a & b) | (c & ~b);   // v_and_or_b32 (c & ~b is loop-invariant)
    } else if constexpr (OP == NASCH_PROBE_CNDMASK) {
        return c > 7u ? a : b;   // v_cndmask_b32 on a loop-invariant condition
    } else if constexpr (OP == NASCH_PROBE_BFI) {
        // the chain value selects between b and c (written out: the compiler
        // turns the C form into v_bitop3_b32 here)
        uint32_t r;
        __asm__("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
        return r;
    } else if constexpr (OP == NASCH_PROBE_OR) {
        return a | b;
    } else if constexpr (OP == NASCH_PROBE_AND) {
        return a & b;
    } else if constexpr (OP == NASCH_PROBE_ADD3) {
        // written out: the compiler adds the loop-invariant b + c once
        uint32_t r;
        __asm__("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
        return r;
    } else {
        return a;
    }
}

template <int OP>
__global__ __launch_bounds__(256) void valu_probe_kernel(uint32_t* __restrict__ out,
                                                         uint64_t* __restrict__ clocks,
                                                         uint32_t iters, uint32_t seed) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a[kChains];
    uint64_t w[kChains];   // NASCH_PROBE_MAD_U64: 64-bit chains
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        a[j] = tid * 0x9E3779B9u + (uint32_t)j * 0x85EBCA6Bu + seed;
        w[j] = ((uint64_t)a[j] << 32) | (a[j] ^ 0x5bd1e995u);
    }
    // loop-invariant operands, opaque to the compiler
    uint32_t b = seed | 1u, c = (seed >> 3) & 31u;
    __asm__ volatile("" : "+v"(b), "+v"(c));
    uint64_t t0 = 0, r0 = 0;
    if (threadIdx.x == 0) {
        t0 = clock64();
        r0 = wall_clock64();
    }
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int j = 0; j < kChains; ++j) {
                if constexpr (OP == NASCH_PROBE_MAD_U64) {
                    // one v_mad_u64_u32: w = lo(w) * b + w, as in Philox's rounds
                    w[j] = (uint64_t)(uint32_t)w[j] * b + w[j];
                    __asm__ volatile("" : "+v"(w[j]));
                } else if constexpr (OP == NASCH_PROBE_ADD_U64) {
                    // one 64-bit add (v_lshl_add_u64 with no shift), as in address arithmetic
                    w[j] = w[j] + (((uint64_t)c << 32) | b);
                    __asm__ volatile("" : "+v"(w[j]));
                } else {
                    a[j] = op<OP>(a[j], b, c);
                    // keeps the compiler from folding a chain algebraically
                    // (a product of 16 factors b into one power); emits nothing
                    __asm__ volatile("" : "+v"(a[j]));
                }
            }
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc ^= a[j] ^ (uint32_t)w[j] ^ (uint32_t)(w[j] >> 32);
    out[tid] = acc;
    if (threadIdx.x == 0) {
        const uint64_t t1 = clock64(), r1 = wall_clock64();
        clocks[2 * blockIdx.x] = t1 - t0;
        clocks[2 * blockIdx.x + 1] = r1 - r0;
    }
}

template <int OP>
hipError_t launch(uint32_t blocks, uint32_t* out, uint64_t* clocks, uint32_t iters, uint32_t seed,
                  hipStream_t s) {
    (void)hipGetLastError();
    hipLaunchKernelGGL((valu_probe_kernel<OP>), dim3(blocks), dim3(256), 0, s, out, clocks, iters,
                       seed);
    return hipGetLastError();
}

hipError_t launch_op(uint32_t kind, uint32_t blocks, uint32_t* out, uint64_t* clocks,
                     uint32_t iters, uint32_t seed, hipStream_t s) {
    switch (kind) {
        case NASCH_PROBE_BITOP3: return launch<NASCH_PROBE_BITOP3>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_ALIGNBIT: return launch<NASCH_PROBE_ALIGNBIT>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_BCNT: return launch<NASCH_PROBE_BCNT>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_MUL_LO: return launch<NASCH_PROBE_MUL_LO>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_MUL_HI: return launch<NASCH_PROBE_MUL_HI>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_MAD_U64: return launch<NASCH_PROBE_MAD_U64>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_DPP: return launch<NASCH_PROBE_DPP>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_ADD: return launch<NASCH_PROBE_ADD>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_XOR: return launch<NASCH_PROBE_XOR>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_SHIFT: return launch<NASCH_PROBE_SHIFT>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_LSHL_OR: return launch<NASCH_PROBE_LSHL_OR>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_PERM: return launch<NASCH_PROBE_PERM>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_MUL_U24: return launch<NASCH_PROBE_MUL_U24>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_ADD_U64: return launch<NASCH_PROBE_ADD_U64>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_MIN: return launch<NASCH_PROBE_MIN>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_SUB: return launch<NASCH_PROBE_SUB>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_CNDMASK: return launch<NASCH_PROBE_CNDMASK>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_AND_OR: return launch<NASCH_PROBE_AND_OR>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_BFI: return launch<NASCH_PROBE_BFI>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_OR: return launch<NASCH_PROBE_OR>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_AND: return launch<NASCH_PROBE_AND>(blocks, out, clocks, iters, seed, s);
        case NASCH_PROBE_ADD3: return launch<NASCH_PROBE_ADD3>(blocks, out, clocks, iters, seed, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

extern "C" int nasch_probe_valu(uint32_t kind, uint32_t blocks, uint32_t iters,
                                nasch_probe_result* res) {
    if (!res || kind >= NASCH_PROBE_KINDS || blocks == 0 || iters == 0) return -1;
    *res = nasch_probe_result{};
    uint32_t* out = nullptr;
    uint64_t* clocks = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::size_t nclk = 2u * blocks;
    uint64_t* hclk = new (std::nothrow) uint64_t[nclk];
    hipError_t e = hclk ? hipSuccess : hipErrorOutOfMemory;
    if (e == hipSuccess) e = hipMalloc((void**)&out, (size_t)blocks * 256u * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&clocks, nclk * sizeof(uint64_t));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // one short untimed launch (code load, clocks up), then the timed one
    if (e == hipSuccess) e = launch_op(kind, blocks, out, clocks, iters / 8u + 1u, 1u, s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch_op(kind, blocks, out, clocks, iters, 7u, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess)
        e = hipMemcpy(hclk, clocks, nclk * sizeof(uint64_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess) {
        double cyc = 0, ref = 0;
        for (uint32_t b = 0; b < blocks; ++b) {
            cyc += (double)hclk[2 * b];
            ref += (double)hclk[2 * b + 1];
        }
        res->ms = ms;
        res->wave_instructions = (double)blocks * 4.0 * iters * kChains * kUnroll;
        res->lane_ops_per_s = res->wave_instructions * 64.0 / (ms * 1e-3);
        // s_memrealtime counts at a constant 100 MHz
        res->sclk_hz = ref > 0 ? cyc / ref * 100e6 : 0.0;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (out) (void)hipFree(out);
    if (clocks) (void)hipFree(clocks);
    delete[] hclk;
    return e == hipSuccess ? 0 : -(int)e;
}
