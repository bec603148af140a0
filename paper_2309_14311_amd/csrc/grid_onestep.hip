// grid_onestep.hip -- the plain grid kernel: one step per launch, one byte per
// cell, a workgroup per tile of kOneStepTile cells staged through LDS with a
// vmax halo on each side (rules 1-4 of the Handout, applied car by car).
//
// Each thread owns 32 consecutive cells (one aligned rule-3 block, so one
// Philox call covers them).  It builds the occupancy mask of its cells and the
// 8 after them and decides rule 3 for all its cars at once: the block's top
// nibbles are compared with thr's, and the cars whose nibble ties are numbered
// across the wave and have their low 28 bits drawn 64 at a time, so no car
// loop ever runs a Philox call.  It then visits its cars through the mask (the
// distance to the car in front is a trailing-zero count) and scatters each car
// into a cleared LDS copy of the tile.  Cars up to vmax cells left of the tile can land inside
// it; lanes 0..vmax-1 recompute those.  The tile is then written back with
// 16-byte stores.  F(t) counts owned cars only.
//
// Open road: cells outside [0, L) load as empty, except cell L, which holds a
// stopped car when the step's gate keeps the exit closed; cars moving past
// L-1 are not written (they leave); the tile of cell 0 adds the entering car.
#include "launchers.hpp"

namespace nasch {

namespace {
constexpr uint32_t kThreads = 256;
constexpr uint32_t kHalo = 16;  // >= vmax, keeps the LDS copy 16-byte aligned
constexpr uint32_t kTile = kOneStepTile;
static_assert(kTile == kThreads * 32, "one 32-cell block per thread");

// bit 7 of each byte of w -> bits 0..3
__device__ __forceinline__ uint32_t byte_msbs(uint32_t w) {
    return (((w >> 7) & 0x01010101u) * 0x00204081u) >> 21 & 0xFu;
}

// Rules 1-3 for one car: v its velocity, d the distance to the car in front
// (capped at vmax + 1, which rule 2 cannot tell from farther), hi4 the top
// nibble of its R (the low bits are drawn only on a tie).
__device__ __forceinline__ uint32_t new_velocity(uint32_t v, uint32_t d, uint32_t vmax,
                                                 uint32_t hi4, uint32_t x, uint32_t t,
                                                 const SlowParams& sp) {
    uint32_t nv = min(v + 1u, vmax);       // rule 1
    if (nv >= d) nv = d - 1u;              // rule 2
    if (nv > 0 && sp.thr != 0 && slow_from_hi(hi4, x, t, sp)) --nv;   // rule 3
    return nv;
}

__device__ __forceinline__ uint32_t nibble(const Word4& w, uint32_t j) {
    return (((w.w0 >> j) & 1u) << 3) | (((w.w1 >> j) & 1u) << 2) | (((w.w2 >> j) & 1u) << 1) |
           ((w.w3 >> j) & 1u);
}

// LDS of one wave for the tied cars of its 64 words.
constexpr uint32_t kTieCap = 256;
struct TieLds {
    uint32_t code[kTieCap];   // lane << 5 | bit of each queued car
    uint32_t x0[64];          // first cell of each lane's word
    uint32_t slow[64];        // slow cars found by the draws, per lane
};

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The slow cars among `tie` (cars of cells x0 .. x0+31 whose top nibble of R
// equals thr's): decided by the low 28 bits of R.  Numbered with a wave prefix
// sum and drawn 64 at a time; cars beyond the queue's capacity are drawn by
// their own lane.  All 64 lanes of the wave must call it.
__device__ __forceinline__ uint32_t resolve_ties(uint32_t tie, uint32_t x0, uint32_t t,
                                                 const SlowParams& sp, TieLds& lds,
                                                 uint32_t lane) {
    const uint32_t lo_thr = sp.thr & 0x0FFFFFFFu;
    const uint32_t cnt = __popc(tie);
    const uint32_t incl = wave_scan_incl(cnt);
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    if (total == 0u) return 0u;
    const uint32_t nq = min(total, kTieCap);
    lds.x0[lane] = x0;
    lds.slow[lane] = 0u;
    uint32_t idx = incl - cnt, own = 0u;
    while (tie) {
        const uint32_t b = __builtin_ctz(tie);
        tie &= tie - 1u;
        if (idx < kTieCap) lds.code[idx] = (lane << 5) | b;
        else if (slow_lo28(x0 + b, t, sp) < lo_thr) own |= 1u << b;
        ++idx;
    }
    wave_sync_lds();
    for (uint32_t p = lane; p < nq; p += 64u) {
        const uint32_t c = lds.code[p];
        if (slow_lo28(lds.x0[c >> 5] + (c & 31u), t, sp) < lo_thr)
            atomicOr(&lds.slow[c >> 5], 1u << (c & 31u));
    }
    wave_sync_lds();
    return own | lds.slow[lane];
}
}  // namespace

// F(t) of the tile goes to partials[blockIdx.x] (summed by the fold kernel).
__global__ __launch_bounds__(kThreads) void grid_onestep_kernel(const RingDesc* __restrict__ ring,
                                                                uint32_t* __restrict__ partials,
                                                                const Clock* __restrict__ clk,
                                                                uint32_t s_off,
                                                                uint32_t launch_idx) {
    __shared__ __align__(16) uint8_t s_in[kTile + 2 * kHalo];
    __shared__ __align__(16) uint8_t s_out[kTile];
    __shared__ uint32_t s_flux[kThreads / 64];
    __shared__ TieLds s_tie[kThreads / 64];

    const RingDesc& R = *ring;
    const uint32_t L = R.L, vmax = R.vmax;
    const SlowParams sp = R.sp;
    const uint32_t t = clk->t + R.t + s_off;
    const uint32_t par = (clk->parity + R.parity + launch_idx) & 1u;
    const uint8_t* __restrict__ src = R.buf[par];
    uint8_t* __restrict__ dst = R.buf[par ^ 1u];

    const uint32_t start = blockIdx.x * kTile;
    const uint32_t len = min(kTile, L - start);
    const uint32_t tid = threadIdx.x;
    const bool open = R.open != 0;
    bool enter = false, exit_open = true;
    if (open && (start == 0 || (uint64_t)start + len + kHalo > L))   // uniform per block
        gate_draw(t, sp, R.thr_in, R.thr_out, enter, exit_open);

    // ---- load the tile and its halos (cells start-kHalo .. start+len+kHalo, mod L)
    if (start >= kHalo && (uint64_t)start + kTile + kHalo <= L) {
        const uint4* s4 = reinterpret_cast<const uint4*>(src + start - kHalo);
        uint4* d4 = reinterpret_cast<uint4*>(s_in);
        for (uint32_t i = tid; i < (kTile + 2 * kHalo) / 16; i += kThreads) d4[i] = s4[i];
    } else {
        for (uint32_t i = tid; i < kTile + 2 * kHalo; i += kThreads) {
            const int64_t c = (int64_t)i - kHalo;
            uint8_t val = (uint8_t)kEmpty;
            if (c < (int64_t)len + kHalo) {
                int64_t pos = (int64_t)start + c;
                if (open) {
                    if (pos >= 0 && pos < (int64_t)L) val = src[pos];
                    else if (pos == (int64_t)L && !exit_open) val = 0;   // closed exit
                } else {
                    pos %= (int64_t)L;
                    if (pos < 0) pos += L;
                    val = src[pos];
                }
            }
            s_in[i] = val;
        }
    }
    {
        uint4* o4 = reinterpret_cast<uint4*>(s_out);
        const uint4 e = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
        for (uint32_t i = tid; i < kTile / 16; i += kThreads) o4[i] = e;
    }
    __syncthreads();

    // ---- owned cars: occupancy of the thread's 32 cells and the 8 after them
    uint32_t flux = 0;
    const uint32_t c0 = tid * 32u;
    uint64_t occ = 0;
    uint32_t cars = 0;
    if (c0 < len) {
        const uint4* in4 = reinterpret_cast<const uint4*>(s_in + kHalo + c0);
        const uint4 a = in4[0], b = in4[1];
        const uint2 c = *reinterpret_cast<const uint2*>(s_in + kHalo + c0 + 32);
        const uint32_t w[10] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y};
#pragma unroll
        for (int d = 0; d < 10; ++d) occ |= (uint64_t)byte_msbs(~w[d]) << (4 * d);
        const uint32_t n = min(32u, len - c0);
        cars = (uint32_t)occ & (n >= 32u ? 0xFFFFFFFFu : ((1u << n) - 1u));
    }
    // ---- rule 3 for every car of the block (slow = R < thr); uniform branches
    uint32_t slow = 0u;
    if (sp.thr != 0) {
        uint32_t lt = 0u, eq = 0u;
        if (cars) block_lt_eq(slow_hi_planes((start + c0) >> 5, t, sp), sp.thr >> 28, lt, eq);
        slow = lt & cars;
        if ((sp.thr & 0x0FFFFFFFu) != 0u)
            slow |= resolve_ties(eq & cars, start + c0, t, sp, s_tie[tid >> 6], tid & 63u);
    }
    while (cars) {
        const uint32_t j = __builtin_ctz(cars);
        cars &= cars - 1u;
        const uint64_t ahead = occ >> (j + 1);
        const uint32_t d = ahead ? min((uint32_t)__builtin_ctzll(ahead) + 1u, vmax + 1u)
                                 : vmax + 1u;
        uint32_t v = min(s_in[kHalo + c0 + j] + 1u, vmax);   // rule 1
        if (v >= d) v = d - 1u;                                // rule 2
        if (v > 0 && ((slow >> j) & 1u)) --v;                  // rule 3
        if (c0 + j + v < len) s_out[c0 + j + v] = (uint8_t)v;  // rule 4
        flux += v;
    }
    // ---- the cars up to vmax cells left of the tile may land inside it: one lane each
    if (tid < vmax) {
        const int c = -1 - (int)tid;
        if (s_in[kHalo + c] != kEmpty) {
            uint32_t d = 1;
            while (d <= vmax && s_in[kHalo + c + d] == kEmpty) ++d;
            int64_t pos = ((int64_t)start + c) % (int64_t)L;
            if (pos < 0) pos += L;
            const uint32_t x = (uint32_t)pos;
            const Word4 hb = sp.thr != 0 ? slow_hi_planes(x >> 5, t, sp) : Word4{0, 0, 0, 0};
            const uint32_t v = new_velocity(s_in[kHalo + c], d, vmax, nibble(hb, x & 31u), x, t, sp);
            const int dstc = c + (int)v;
            if (dstc >= 0 && (uint32_t)dstc < len) s_out[dstc] = (uint8_t)v;
        }
    }
    // ---- open road: the entering car (no other car can land in cell 0)
    if (open && start == 0 && tid == 0 && enter && s_in[kHalo] == kEmpty) s_out[0] = 0;
    const uint32_t wsum = wave_total(flux);
    if ((tid & 63u) == 0) s_flux[tid >> 6] = wsum;
    __syncthreads();

    // ---- write back
    if (len == kTile) {
        const uint4* o4 = reinterpret_cast<const uint4*>(s_out);
        uint4* d4 = reinterpret_cast<uint4*>(dst + start);
        for (uint32_t i = tid; i < kTile / 16; i += kThreads) d4[i] = o4[i];
    } else {
        for (uint32_t i = tid; i < len; i += kThreads) dst[start + i] = s_out[i];
    }
    if (tid == 0) {
        uint32_t total = 0;
        for (uint32_t wv = 0; wv < kThreads / 64; ++wv) total += s_flux[wv];
        if (R.flux_log) partials[blockIdx.x] = total;
        if (R.flux_acc && (uint64_t)t >= R.warmup && total)
            atomicAdd(R.flux_acc, (unsigned long long)total);
    }
}

hipError_t launch_grid_onestep(const RingDesc* ring, uint32_t L, uint32_t* partials,
                               const Clock* clk, uint32_t s_off, uint32_t launch_idx,
                               hipStream_t s) {
    const uint32_t blocks = onestep_blocks(L);
    NASCH_LAUNCH(grid_onestep_kernel, dim3(blocks), dim3(kThreads), 0, s, ring, partials, clk,
                 s_off, launch_idx);
    return hipGetLastError();
}

}  // namespace nasch
