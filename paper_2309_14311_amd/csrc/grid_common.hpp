// grid_common.hpp -- device helpers shared by the grid kernels (the bit-sliced
// k-step kernel and the one-step kernel on the byte form): rule-3 draws of
// 32-cell words that are not one aligned block, the wave-wide refinement of
// tied draws, and loads and stores of the byte form.
#pragma once
#include "bitplanes.hpp"
#include "nasch_device.hpp"

namespace nasch {
namespace grid {

// mask of bits [a, b), 0 <= a <= b <= 32
__device__ __forceinline__ uint32_t bit_range(uint32_t a, uint32_t b) {
    const uint32_t hi = b >= 32 ? 0xFFFFFFFFu : ((1u << b) - 1u);
    const uint32_t lo = a >= 32 ? 0xFFFFFFFFu : ((1u << a) - 1u);
    return hi & ~lo;
}

// Top-nibble planes of R for the 32 consecutive ring cells x0, x0+1, ... (mod L)
// when they are not one aligned block: assembled from the blocks they touch.
__device__ __forceinline__ Word4 planes_unaligned(uint32_t x0, uint32_t t, uint32_t L,
                                              const SlowParams& sp) {
    Word4 r{0, 0, 0, 0};
    uint32_t pos = x0, i = 0;
    while (i < 32u) {
        const uint32_t off = pos & 31u;
        uint32_t run = min(32u - off, L - pos);
        run = min(run, 32u - i);
        const Word4 w = slow_hi_planes(pos >> 5, t, sp);
        const uint32_t m = run >= 32u ? 0xFFFFFFFFu : ((1u << run) - 1u);
        r.w0 |= ((w.w0 >> off) & m) << i;
        r.w1 |= ((w.w1 >> off) & m) << i;
        r.w2 |= ((w.w2 >> off) & m) << i;
        r.w3 |= ((w.w3 >> off) & m) << i;
        i += run;
        pos += run;
        if (pos >= L) pos = 0;
    }
    return r;
}

// Do the 32 ring cells x0, x0+1, ... (mod L) lie in at most two blocks: block
// x0 >> 5 from bit x0 & 31 up to its end or the ring's end, then the ring's
// next block from bit 0?  (Always on rings of 64 cells or more, except for a
// word that covers a short last block whole and runs on into block 0.)
__device__ __forceinline__ bool two_blocks(uint32_t x0, uint32_t L, uint32_t nw) {
    const uint32_t run0 = min(32u - (x0 & 31u), L - x0);
    if (run0 == 32u) return true;
    const uint32_t b1 = x0 + run0 >= L ? 0u : (x0 >> 5) + 1u;
    const uint32_t len1 = b1 + 1u == nw ? L - 32u * b1 : 32u;
    return 32u - run0 <= len1;
}

// planes_unaligned for cells that satisfy two_blocks, in straight-line code:
// two block draws joined by shifts.  An aligned word gets its block unchanged
// (the second draw is then unused).
__device__ __forceinline__ Word4 planes_two(uint32_t x0, uint32_t t, uint32_t L,
                                            const SlowParams& sp) {
    // The shift amounts below depend on x0 only; hoisted out of the step loop
    // they would hold ten more registers through the whole kernel (and cost
    // every wave occupancy).  An empty asm makes x0 opaque so they are
    // recomputed where they are used, in the few waves that take this path.
    __asm__ volatile("" : "+v"(x0));
    const uint32_t off = x0 & 31u;
    const uint32_t run0 = min(32u - off, L - x0);   // 1..32 cells from the first block
    const uint32_t b0 = x0 >> 5;
    const uint32_t b1 = x0 + run0 >= L ? 0u : b0 + 1u;
    const Word4 a = slow_hi_planes(b0, t, sp);
    const Word4 b = slow_hi_planes(b1, t, sp);
    const uint32_t m = 0xFFFFFFFFu >> (32u - run0);
    const uint32_t sh = run0 - 1u;   // b's bit 0 goes to bit run0 (nowhere when run0 = 32)
    Word4 r;
    r.w0 = ((a.w0 >> off) & m) | ((b.w0 << sh) << 1);
    r.w1 = ((a.w1 >> off) & m) | ((b.w1 << sh) << 1);
    r.w2 = ((a.w2 >> off) & m) | ((b.w2 << sh) << 1);
    r.w3 = ((a.w3 >> off) & m) | ((b.w3 << sh) << 1);
    return r;
}

// F(t) of a word from its thermometer planes T[1..VMAX] (T[m]: v >= m), by the
// binary digits of the speeds.  Bit i of v is the parity of the number of
// multiples m of 2^i with m <= v, that is the XOR of the planes T[m] with 2^i
// dividing m; so the sum of v over the word's cars is
// sum_i 2^i popc(XOR of those planes), at most four popcounts (4-cycle
// instructions) and a few three-input XORs (2-cycle) instead of VMAX popcounts.
// d[i] accumulates the popcount of digit i over the cars selected by `mask`.
template <int VMAX, int STEP>
__device__ __forceinline__ uint32_t speed_digit(const uint32_t* T) {
    uint32_t r = T[STEP];
    int m = 2 * STEP;
#pragma unroll
    for (; m + STEP <= VMAX; m += 2 * STEP) r = xor3(r, T[m], T[m + STEP]);
    if (m <= VMAX) r ^= T[m];
    return r;
}

template <int VMAX, bool MASKED>
__device__ __forceinline__ void add_speed_digits(const uint32_t* T, uint32_t mask,
                                                 uint32_t (&d)[4]) {
    const uint32_t k = MASKED ? mask : 0xFFFFFFFFu;
    if constexpr (VMAX >= 1) d[0] += __popc(speed_digit<VMAX, 1>(T) & k);
    if constexpr (VMAX >= 2) d[1] += __popc(speed_digit<VMAX, 2>(T) & k);
    if constexpr (VMAX >= 4) d[2] += __popc(speed_digit<VMAX, 4>(T) & k);
    if constexpr (VMAX >= 8) d[3] += __popc(speed_digit<VMAX, 8>(T) & k);
}

// The sum the digit counts stand for.
__device__ __forceinline__ uint32_t speed_sum(const uint32_t (&d)[4]) {
    return d[0] + 2u * d[1] + 4u * d[2] + 8u * d[3];
}

// How a wave draws the top-nibble planes (uniform over the wave, fixed for a
// launch): every word one aligned block (the interior of a ring); some words
// across two blocks (the tiles at the end of a ring whose length is not a
// multiple of 32); anything else (rings shorter than a segment).
enum : uint32_t { kDrawAligned = 0, kDrawTwo = 1, kDrawGeneric = 2 };

// Rule 3, first stage, for the moving cars of the lane's Q words (word q covers
// ring cells xw[q] .. xw[q]+31, mod L): S = cars whose top nibble of R is below
// thr's (slow), U = cars whose top nibble ties with thr's (decided by the low
// 28 bits).  The comparison is specialised on thr's top nibble, which is
// uniform over the wave.
template <int Q>
__device__ __forceinline__ void slow_hi(const uint32_t (&moving)[Q], const uint32_t (&xw)[Q],
                                        const bool (&aligned)[Q], uint32_t draw_mode,
                                        uint32_t t, uint32_t L, const SlowParams& sp,
                                        uint32_t (&S)[Q], uint32_t (&U)[Q]) {
    Word4 hp[Q];
    if (draw_mode == kDrawAligned) {
#pragma unroll
        for (int q = 0; q < Q; ++q) hp[q] = slow_hi_planes(xw[q] >> 5, t, sp);
    } else if (draw_mode == kDrawTwo) {
#pragma unroll
        for (int q = 0; q < Q; ++q) hp[q] = planes_two(xw[q], t, L, sp);
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            hp[q] = aligned[q] ? slow_hi_planes(xw[q] >> 5, t, sp)
                               : planes_unaligned(xw[q], t, L, sp);
    }
    uint32_t lt[Q], eq[Q];
#define NASCH_NIBBLE_CASE(TH)                                             \
    case TH:                                                              \
        for (int q = 0; q < Q; ++q) nibble_cmp<TH>(hp[q], lt[q], eq[q]); \
        break;
    switch (sp.thr >> 28) {
        NASCH_NIBBLE_CASE(0) NASCH_NIBBLE_CASE(1) NASCH_NIBBLE_CASE(2) NASCH_NIBBLE_CASE(3)
        NASCH_NIBBLE_CASE(4) NASCH_NIBBLE_CASE(5) NASCH_NIBBLE_CASE(6) NASCH_NIBBLE_CASE(7)
        NASCH_NIBBLE_CASE(8) NASCH_NIBBLE_CASE(9) NASCH_NIBBLE_CASE(10) NASCH_NIBBLE_CASE(11)
        NASCH_NIBBLE_CASE(12) NASCH_NIBBLE_CASE(13) NASCH_NIBBLE_CASE(14)
        default:
            for (int q = 0; q < Q; ++q) nibble_cmp<15>(hp[q], lt[q], eq[q]);
            break;
    }
#undef NASCH_NIBBLE_CASE
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        S[q] = moving[q] & lt[q];
        U[q] = moving[q] & eq[q];
    }
}

// Rule 3, second stage, shared by the whole wave.  Every lane with tied cars
// (bits of U) reserves consecutive slots of an LDS queue with one LDS atomic
// add and queues them there as (word, bit) codes, which are their segment
// cells; the wave then draws their low 28 bits 64 at a time, taking a car's
// ring cell from its segment cell (see XMode), and ORs each slow car into an
// LDS mask of its word.  Every lane then takes its words' masks (and clears
// them for the next step): one LDS read per word instead of a loop over the
// lane's tied cars.  The order of the lanes in the queue is arbitrary, and
// nothing depends on it: a car's draw is keyed by its cell.  (A wave prefix
// sum over DPP numbered the cars before; the atomic measured 11 % faster on
// the ensemble, the prefix sum's chain of dependent cross-lane steps being
// on every tie step's critical path.)  A word rarely holds more than two tied
// cars, so those two are queued without a loop.  When the wave has more tied
// cars than the queue holds (possible, never seen), cars numbered beyond its
// capacity are drawn by their own lane.
constexpr uint32_t kRefineCap = 256;

template <int Q>
struct RefineLds {
    uint32_t code[kRefineCap];   // (lane Q + q) << 5 | bit of each queued car
    uint32_t slow[64 * Q];       // slow cars found by the draws, per word
    uint32_t n;                  // tied cars of the step (0 between steps)
};

// The ring cell of segment cell j is seg0 + j reduced by XMode (uniform over the
// wave): kXNone on an open road (seg0 is the road cell of segment cell 0, taken
// modulo 2^32, and queued cars lie on the road), kXSub on a ring at least as
// long as the segment (seg0 < L, so one subtraction), kXMod on a shorter ring.
enum : uint32_t { kXNone = 0, kXSub = 1, kXMod = 2 };

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int Q>
__device__ __forceinline__ void slow_lo_wave(uint32_t (&S)[Q], const uint32_t (&U)[Q],
                                             const uint32_t (&xw)[Q], uint32_t L, uint32_t seg0,
                                             uint32_t x_mode, uint32_t t, const SlowParams& sp,
                                             RefineLds<Q>& lds, uint32_t lane) {
    const uint32_t lo_thr = sp.thr & 0x0FFFFFFFu;
    uint32_t cnt = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) cnt += __popc(U[q]);
    // each lane with tied cars reserves its queue slots with one LDS atomic
    uint32_t idx = 0u;
    if (cnt) idx = atomicAdd(&lds.n, cnt);
    wave_sync_lds();
    const uint32_t total = __builtin_amdgcn_readfirstlane(lds.n);
    if (total == 0u) return;
    const uint32_t nq = min(total, kRefineCap);
    if (total <= kRefineCap) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const uint32_t u = U[q];
            const uint32_t wcode = (lane * Q + q) << 5;
            const uint32_t u1 = u & (u - 1u);
            if (u) lds.code[idx] = wcode | __builtin_ctz(u);
            if (u1) lds.code[idx + 1u] = wcode | __builtin_ctz(u1);
            uint32_t r = u1 & (u1 - 1u);
            for (uint32_t j = idx + 2u; r; ++j) {
                lds.code[j] = wcode | __builtin_ctz(r);
                r &= r - 1u;
            }
            idx += __popc(u);
        }
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            uint32_t u = U[q];
            const uint32_t wcode = (lane * Q + q) << 5;
            while (u) {
                const uint32_t b = __builtin_ctz(u);
                u &= u - 1u;
                if (idx < kRefineCap) {
                    lds.code[idx] = wcode | b;
                } else {
                    uint32_t x = xw[q] + b;
                    if (x >= L) x %= L;
                    if (slow_lo28(x, t, sp) < lo_thr) S[q] |= 1u << b;
                }
                ++idx;
            }
        }
    }
    wave_sync_lds();
    for (uint32_t p = lane; p < nq; p += 64u) {
        const uint32_t c = lds.code[p];   // the car's segment cell
        uint32_t x = seg0 + c;
        if (x_mode == kXSub) {
            x = min(x, x - L);   // x - L wraps above x unless x >= L
        } else if (x_mode == kXMod) {
            x %= L;
        }
        if (slow_lo28(x, t, sp) < lo_thr) atomicOr(&lds.slow[c >> 5], 1u << (c & 31u));
    }
    wave_sync_lds();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        S[q] |= lds.slow[lane * Q + q];
        lds.slow[lane * Q + q] = 0u;
    }
    if (lane == 0u) lds.n = 0u;
    // the queue is rewritten at the next step only after every lane has read it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The bit planes of the 32 consecutive ring cells x0, x0+1, ... (mod L) when
// they are not one aligned word of the stored planes (a word across the end
// of the ring, or a ring shorter than a segment): assembled run by run.
template <int VMAX>
__device__ __forceinline__ void gather_ring(const uint32_t* __restrict__ src, uint32_t nw, uint32_t L,
                                         uint32_t x0, uint32_t (&T)[VMAX + 1]) {
#pragma unroll
    for (int m = 0; m <= VMAX; ++m) T[m] = 0u;
    uint32_t pos = x0, i = 0;
    while (i < 32u) {
        const uint32_t off = pos & 31u;
        uint32_t run = min(32u - off, L - pos);
        run = min(run, 32u - i);
        const uint32_t mask = run >= 32u ? 0xFFFFFFFFu : ((1u << run) - 1u);
        const uint32_t w = pos >> 5;
#pragma unroll
        for (int m = 0; m <= VMAX; ++m) T[m] |= ((*gmem(src + (size_t)m * nw + w) >> off) & mask) << i;
        i += run;
        pos += run;
        if (pos >= L) pos = 0;
    }
}

// ---- the byte form (the one-step kernel): the road is read and written as one
// byte per cell and converted to and from bit planes in registers.

// The 32 bytes of an aligned 32-cell word (16-byte loads).
__device__ __forceinline__ void load_bytes32(const uint8_t* __restrict__ p, uint32_t (&d)[8]) {
    const u32x4 a = *gmem(reinterpret_cast<const u32x4*>(p));
    const u32x4 b = *gmem(reinterpret_cast<const u32x4*>(p + 16));
    d[0] = a.x; d[1] = a.y; d[2] = a.z; d[3] = a.w;
    d[4] = b.x; d[5] = b.y; d[6] = b.z; d[7] = b.w;
}

// The bytes of the 32 consecutive ring cells x0, x0+1, ... (mod L), x0 < L,
// one at a time (a word across the end of the ring, or a short ring).
__device__ __forceinline__ void gather_bytes_ring(const uint8_t* __restrict__ src, uint32_t L,
                                                  uint32_t x0, uint32_t (&d)[8]) {
    uint32_t pos = x0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        uint32_t w = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            w |= (uint32_t)*gmem(src + pos) << (8 * b);
            pos = pos + 1u == L ? 0u : pos + 1u;
        }
        d[i] = w;
    }
}

// Open road: the bytes of cells p0 .. p0+31 (p0 < L, a multiple of 32); cells
// at or past L read as empty.
__device__ __forceinline__ void load_bytes_open(const uint8_t* __restrict__ src, uint32_t L,
                                                uint32_t p0, uint32_t (&d)[8]) {
    if (p0 + 32u <= L) {
        load_bytes32(src + p0, d);
        return;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        uint32_t w = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t c = p0 + 4u * i + b;
            w |= (uint32_t)(c < L ? *gmem(src + c) : (uint8_t)kEmpty) << (8 * b);
        }
        d[i] = w;
    }
}

// Write the owned cells (bits of own) of the word of road cells c0 .. c0+31;
// a wholly owned word lies inside the road and is written with 16-byte stores.
__device__ __forceinline__ void store_bytes(uint8_t* __restrict__ dst, uint32_t c0, uint32_t own,
                                            const uint32_t (&d)[8]) {
    if (own == 0xFFFFFFFFu) {
        *gmem(reinterpret_cast<u32x4*>(dst + c0)) = u32x4{d[0], d[1], d[2], d[3]};
        *gmem(reinterpret_cast<u32x4*>(dst + c0 + 16)) = u32x4{d[4], d[5], d[6], d[7]};
        return;
    }
#pragma unroll
    for (int i = 0; i < 32; ++i)
        if ((own >> i) & 1u) *gmem(dst + c0 + i) = (uint8_t)(d[i >> 2] >> (8 * (i & 3)));
}

}  // namespace grid
}  // namespace nasch
