// agent.hip -- the agent representation ("Concepts Covered"; the Handout's starter
// code keeps two length-N vectors): int32 positions x[N] in road order and
// uint8 velocities v[N].  Car i's distance to the car in front is
// d = (x[i+1] - x[i]) mod L (d = L for a car alone); rules 1-4 follow.
//
// agent_kstep_kernel<C>: one wave per 64 C consecutive cars (C per lane, chosen
// on the host from the density), kept in registers for k steps.  Car i after
// s steps depends only on cars i .. i+s, so the last k cars of a wave are a
// halo: each wave writes back the first `own` cars and the waves overlap by
// the halo.  Launched with one step it is the one-step kernel.
// Rule 3 uses the same keyed draw as the grid kernels (R depends on the cell a
// car starts the step in), so both representations give identical results.
#include "launchers.hpp"

namespace nasch {

namespace {
// rules 1 and 2.  A real car always has d >= 1; the unsigned min leaves a car
// of a k-step halo that has caught up with its leader (d == 0, possible only
// for cars whose results are discarded) at its rule-1 speed instead of
// wrapping below zero.
__device__ __forceinline__ uint32_t accel_brake(uint32_t v, uint32_t d, uint32_t vmax) {
    return min(min(v + 1u, vmax), d - 1u);
}

constexpr uint32_t kBlockSlots = 256;   // rule-3 blocks tabulated per wave and step
constexpr uint32_t kTieCap = 256;       // tied cars queued per wave

// LDS scratch of one wave for rule 3.
struct AgentLds {
    uint2 blk[kBlockSlots];   // (lt, eq) masks of each tabulated block
    uint32_t tie_x[kTieCap];
    uint8_t tie_r[kTieCap];
    uint32_t n;               // tied cars of the step (0 between steps)
};

// Rule 3 for C consecutive cars per lane (keyed draw), shared by the wave.
// The wave's cars are cyclically sorted, so the 32-cell blocks they start in
// form one run from the block of lane 0's first car (mod the number of
// blocks): a car's slot in that run is its block minus lane 0's, and the run
// ends at the slot of lane 63's last car.  The lanes draw the first
// kBlockSlots blocks of the run together (one Philox call per lane and 64
// blocks), compare each block's 32 top nibbles with thr's at once, and keep
// two masks per block in LDS: cars below thr's nibble and cars tying with it.
// A car reads its two bits from its block's entry; a car past the table (a
// sparse road, or a wave whose cars go round a short ring) draws its own
// block.  The cars whose nibble ties with thr's are then queued in LDS (each
// lane reserving its slots with one LDS atomic add; the queue's order does not
// matter, a draw is keyed by the car's cell) and have their low 28 bits drawn
// 64 at a time.  `nv` holds each car's
// velocity after rules 1-2 and receives the result of rule 3.  All 64 lanes
// must be active; a car with nv == 0 never slows.
template <int C>
__device__ __forceinline__ void agent_rule3(uint32_t (&nv)[C], const uint32_t (&x)[C],
                                            uint32_t L, uint32_t t, const SlowParams& sp,
                                            AgentLds& lds, uint32_t lane) {
    const uint32_t nblk = (L + 31u) >> 5;
    const uint32_t b0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(x[0] >> 5));
    const uint32_t cap = min(kBlockSlots, nblk);
    uint32_t slot[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
        const uint32_t dlt = (x[q] >> 5) - b0;   // wraps above nblk when the block is below b0
        slot[q] = min(dlt, dlt + nblk);
    }
    const uint32_t n =
        min(cap, (uint32_t)__builtin_amdgcn_readlane((int)(slot[C - 1] + 1u), 63));
    const uint32_t th = sp.thr >> 28;
    for (uint32_t j = lane; j < n; j += 64u) {
        uint32_t blk = b0 + j;
        if (blk >= nblk) blk -= nblk;
        uint32_t lt, eq;
        block_lt_eq(slow_hi_planes(blk, t, sp), th, lt, eq);
        lds.blk[j] = make_uint2(lt, eq);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t lo_thr = sp.thr & 0x0FFFFFFFu;
    uint32_t tie = 0;
    // The table covers every car of the wave unless some car lies past it (a
    // sparse road, or a wave going round a short ring): the common case reads
    // it with no per-car test or clamp.  A slow car loses one unit of speed,
    // none below 0 (a saturating subtraction); a tie counts only for a moving car.
    uint32_t smax = slot[0];
#pragma unroll
    for (int q = 1; q < C; ++q) smax = max(smax, slot[q]);
    if (__builtin_amdgcn_ballot_w64(smax >= n) == 0u) {
#pragma unroll
        for (int q = 0; q < C; ++q) {
            const uint2 e = lds.blk[slot[q]];
            const uint32_t sh = x[q] & 31u;
            if (lo_thr != 0u) tie |= (__builtin_amdgcn_ubfe(e.y, sh, 1u) & min(nv[q], 1u)) << q;
            nv[q] = __builtin_elementwise_sub_sat(nv[q], __builtin_amdgcn_ubfe(e.x, sh, 1u));
        }
    } else {
#pragma unroll
        for (int q = 0; q < C; ++q) {
            uint2 e = lds.blk[min(slot[q], kBlockSlots - 1u)];
            if (slot[q] >= n) block_lt_eq(slow_hi_planes(x[q] >> 5, t, sp), th, e.x, e.y);
            const uint32_t sh = x[q] & 31u;
            if (lo_thr != 0u) tie |= (__builtin_amdgcn_ubfe(e.y, sh, 1u) & min(nv[q], 1u)) << q;
            nv[q] = __builtin_elementwise_sub_sat(nv[q], __builtin_amdgcn_ubfe(e.x, sh, 1u));
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lo_thr == 0u) return;   // a tie then never slows (the low bits cannot be below 0)
    const uint32_t cnt = __popc(tie);
    uint32_t base = 0u;
    if (cnt) base = atomicAdd(&lds.n, cnt);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t total = __builtin_amdgcn_readfirstlane(lds.n);
    if (total == 0u) return;
    const uint32_t nq = min(total, kTieCap);
    uint32_t idx = base;
#pragma unroll
    for (int q = 0; q < C; ++q) {
        if ((tie >> q) & 1u) {
            if (idx < kTieCap) lds.tie_x[idx] = x[q];
            ++idx;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t j = lane; j < nq; j += 64u)
        lds.tie_r[j] = slow_lo28(lds.tie_x[j], t, sp) < lo_thr ? 1 : 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    idx = base;
#pragma unroll
    for (int q = 0; q < C; ++q) {
        if ((tie >> q) & 1u) {
            const bool slow = idx < kTieCap ? lds.tie_r[idx] != 0 : slow_lo28(x[q], t, sp) < lo_thr;
            if (slow) --nv[q];
            ++idx;
        }
    }
    if (lane == 0u) lds.n = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
}  // namespace

// ---------------------------------------------------------------------------------
// Wave w holds cars [w own, w own + 64 CPL) and writes back the first own of
// them; F(t) of each wave and step goes to partials[s * ntiles + wave].  own is
// a multiple of 8 (agent_geometry), so for CPL = 4 and 8 a lane's x and v are
// aligned for vector loads and stores.  With `prev` (launches of one step
// each), the first wave of each of the first kFoldBlocks blocks first adds a
// chunk of the previous launch's partials, prev[0 .. ntiles), into its step's
// log entry: no fold launch between steps.  A block holds WAVES independent
// waves.
template <int CPL, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void agent_kstep_kernel(
    const AgentDesc* __restrict__ A, uint32_t own, uint32_t ntiles,
    uint32_t* __restrict__ partials, const uint32_t* __restrict__ prev, uint32_t k,
    const Clock* __restrict__ clk, uint32_t s_off, uint32_t launch_idx) {
    __shared__ AgentLds s_lds[WAVES];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t wave = blockIdx.x * WAVES + wib;
    if (prev && wib == 0u && blockIdx.x < kFoldBlocks && A->flux_log) {
        const unsigned long long f =
            chunk_sum(prev, ntiles, blockIdx.x, min(kFoldBlocks, gridDim.x), lane);
        const uint64_t t_prev = (uint64_t)clk->t + A->t + s_off - 1u;
        if (lane == 0u && f) atomicAdd(&A->flux_log[t_prev - A->log_t0], f);
    }
    if (wave >= ntiles) return;
    AgentLds& lds = s_lds[wib];
    if (lane == 0u) lds.n = 0u;
    const uint32_t N = A->N, L = A->L, vmax = A->vmax;
    const SlowParams sp = A->sp;
    const uint32_t t0 = clk->t + A->t + s_off;
    const uint32_t par = (clk->parity + A->parity + launch_idx) & 1u;
    const int32_t* __restrict__ xs = A->x[par];
    const uint8_t* __restrict__ vs = A->v[par];
    int32_t* __restrict__ xd = A->x[par ^ 1u];
    uint8_t* __restrict__ vd = A->v[par ^ 1u];

    const uint32_t c0 = wave * own;                  // first car of the wave
    const uint32_t own_len = min(own, N - c0);
    const uint32_t first = c0 + lane * CPL;          // first car of the lane (may exceed N)

    uint32_t x[CPL], v[CPL];
    if ((uint64_t)first + CPL <= N) {
        if constexpr (CPL == 8) {
            const u32x4 a = *gmem(reinterpret_cast<const u32x4*>(xs + first));
            const u32x4 b = *gmem(reinterpret_cast<const u32x4*>(xs + first + 4));
            x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
            x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
            typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
            const u32x2 vv = *gmem(reinterpret_cast<const u32x2*>(vs + first));
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v[q] = (vv.x >> (8 * q)) & 0xFFu;
                v[q + 4] = (vv.y >> (8 * q)) & 0xFFu;
            }
        } else if constexpr (CPL == 4) {
            const u32x4 a = *gmem(reinterpret_cast<const u32x4*>(xs + first));
            x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
            const uint32_t vv = *gmem(reinterpret_cast<const uint32_t*>(vs + first));
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = (vv >> (8 * q)) & 0xFFu;
        } else {
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                x[q] = (uint32_t)*gmem(xs + first + q);
                v[q] = *gmem(vs + first + q);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < (int)CPL; ++q) {
            const uint32_t idx = (uint32_t)(((uint64_t)first + q) % N);
            x[q] = (uint32_t)*gmem(xs + idx);
            v[q] = *gmem(vs + idx);
        }
    }

    uint32_t acc = 0u;
    const bool log = A->flux_log != nullptr;
    // shared stream: the number of the lane's first car at step t0, advanced
    // by a^N per step; car q adds a factor a, and a^-N when its index wraps.
    const uint32_t idx0 = (uint32_t)((uint64_t)first % N);
    uint32_t xs_first = 0u;
    if (A->rng)
        xs_first = mlcg_mul(mlcg_pow(A->mlcg_pow, (uint64_t)t0 * N + idx0 + 1u), A->mlcg_x0);
    // owned cars (F(t) counts them only), as masks
    uint32_t ownm[CPL];
#pragma unroll
    for (int q = 0; q < (int)CPL; ++q) ownm[q] = lane * CPL + q < own_len ? 0xFFFFFFFFu : 0u;
    for (uint32_t s = 0; s < k; ++s) {
        const uint32_t t = t0 + s;
        const uint32_t x_next_lane = from_next_lane(x[0]);
        uint32_t nv[CPL];
        if (N > 1) {
#pragma unroll
            for (int q = 0; q < (int)CPL; ++q) {
                // d = (x_next - x) mod L: the difference wraps above the sum
                // when the car ahead is past the end of the ring.  Lane 63's
                // last car reads 0 for the next lane's car: a halo car, whose
                // results are discarded.
                const uint32_t xn = (q + 1 < (int)CPL) ? x[(q + 1) % CPL] : x_next_lane;
                const uint32_t dd = xn - x[q];
                nv[q] = accel_brake(v[q], min(dd, dd + L), vmax);
            }
        } else {
#pragma unroll
            for (int q = 0; q < (int)CPL; ++q) nv[q] = accel_brake(v[q], L, vmax);
        }
        if (A->rng) {
            // rule 3 from the shared stream
            uint32_t r = xs_first;
            uint32_t idx = idx0;
#pragma unroll
            for (int q = 0; q < (int)CPL; ++q) {
                if (q > 0) {
                    r = mlcg_mul(r, kMlcgA);
                    if (++idx == N) {
                        idx = 0;
                        r = mlcg_mul(r, A->mlcg_inv_aN);
                    }
                }
                if (nv[q] > 0u && r < A->mlcg_thr) --nv[q];
            }
            xs_first = mlcg_mul(xs_first, A->mlcg_aN);
        } else if (sp.thr != 0u) {
            agent_rule3<(int)CPL>(nv, x, L, t, sp, lds, lane);   // rule 3
        }
        uint32_t fl = 0u;
#pragma unroll
        for (int q = 0; q < (int)CPL; ++q) {
            fl += nv[q] & ownm[q];
            const uint32_t xn = x[q] + nv[q];   // rule 4; x + v < 2L < 2^32
            x[q] = min(xn, xn - L);             // xn - L wraps above xn unless xn >= L
            v[q] = nv[q];
        }
        if (log) {
            const uint32_t total = wave_total(fl);
            if (lane == 0u) partials[(size_t)s * ntiles + wave] = total;
        }
        if ((uint64_t)t >= A->warmup) acc += fl;
    }
    if (A->flux_acc) {
        const uint32_t total = wave_total(acc);
        if (lane == 0u && total) atomicAdd(A->flux_acc, (unsigned long long)total);
    }

    // write back the owned cars
    if (lane * CPL + CPL <= own_len) {
        if constexpr (CPL == 8) {
            *gmem(reinterpret_cast<u32x4*>(xd + first)) = u32x4{x[0], x[1], x[2], x[3]};
            *gmem(reinterpret_cast<u32x4*>(xd + first + 4)) = u32x4{x[4], x[5], x[6], x[7]};
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lo |= v[q] << (8 * q);
                hi |= v[q + 4] << (8 * q);
            }
            typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
            *gmem(reinterpret_cast<u32x2*>(vd + first)) = u32x2{lo, hi};
        } else if constexpr (CPL == 4) {
            *gmem(reinterpret_cast<u32x4*>(xd + first)) = u32x4{x[0], x[1], x[2], x[3]};
            *gmem(reinterpret_cast<uint32_t*>(vd + first)) =
                v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24);
        } else {
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                *gmem(xd + first + q) = (int32_t)x[q];
                *gmem(vd + first + q) = (uint8_t)v[q];
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < (int)CPL; ++q) {
            if (lane * CPL + q < own_len) {
                *gmem(xd + first + q) = (int32_t)x[q];
                *gmem(vd + first + q) = (uint8_t)v[q];
            }
        }
    }
}

hipError_t launch_agent_kstep(const AgentDesc* a, uint32_t cpl, uint32_t own, uint32_t ntiles,
                              uint32_t* partials, const uint32_t* prev, uint32_t k,
                              const Clock* clk, uint32_t s_off, uint32_t launch_idx,
                              hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    if (prev && (k != 1u || s_off == 0u)) return hipErrorInvalidValue;
    // a launch of one step, bound by HBM, runs blocks of 8 waves; more steps
    // per launch, bound by the instruction count, blocks of 4 (each measured
    // about 2 % faster than the other way round)
    const bool one = k == 1u;
    const dim3 grid(one ? (ntiles + 7u) / 8u : (ntiles + 3u) / 4u);
#define NASCH_AGENT_CASE(C)                                                                   \
    case C:                                                                                   \
        if (one)                                                                              \
            NASCH_LAUNCH((agent_kstep_kernel<C, 8>), grid, dim3(512), 0, s, a, own, ntiles,   \
                         partials, prev, k, clk, s_off, launch_idx);                          \
        else                                                                                  \
            NASCH_LAUNCH((agent_kstep_kernel<C, 4>), grid, dim3(256), 0, s, a, own, ntiles,   \
                         partials, prev, k, clk, s_off, launch_idx);                          \
        break;
    switch (cpl) {
        NASCH_AGENT_CASE(4)
        NASCH_AGENT_CASE(5)
        NASCH_AGENT_CASE(6)
        NASCH_AGENT_CASE(7)
        NASCH_AGENT_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef NASCH_AGENT_CASE
    return hipGetLastError();
}

}  // namespace nasch
