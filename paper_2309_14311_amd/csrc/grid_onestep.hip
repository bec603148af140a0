// grid_onestep.hip -- the one-step grid kernel: one step of rules 1-4 per
// launch on the road's byte form (one byte per cell, 0xFF empty, else v).
//
// Without temporal blocking every step reads and writes each cell's byte once,
// so the kernel is bound by HBM (2 B per cell-update) and everything else has
// to fit under that: the work per 32-cell word is the byte <-> bit-plane
// conversion in registers (bitplanes.hpp), the bit-sliced step itself (the
// same rules as the k-step kernel, see grid_kstep.hip) and one Philox call for
// the top nibble of R of the word's 32 cars.
//
// Layout.  A block of four waves handles one tile: a segment of 256 Q
// consecutive 32-cell words, lane l of wave w holding words (64 w + l) Q ..
// +Q-1.  Segment word 0 and the last word are a one-word halo: the first only
// supplies the cars that drive into the tile (at most vmax <= 8 cells), the
// last only the occupancy that the tile's front cars see.  The tile owns the
// 32 (256 Q - 2) cells in between, so the halo re-reads 2 words of every 256 Q.
// Inside a wave neighbouring words come through DPP lane shifts; the waves of a
// block swap their edge words through LDS (two barriers per step).
//
// Segment cell i is ring cell (own_start - 32 + i) mod L.  A tile whose
// segment lies inside [0, L) is the common case and takes aligned 16-byte
// loads and stores with no reduction mod L; the first tile, a last tile that
// runs past the end of the ring and every ring shorter than a segment read the
// segment cell by cell where it crosses the end (the periodic images of a
// short ring are exact by periodicity) and draw rule 3 across block edges.
// The branch is uniform over the block.
//
// Tiles map to blocks so that the blocks dispatched to one XCD (blocks are
// handed to the 8 XCDs in turn) take consecutive tiles, whose shared halo words
// then meet in the same L2.
#include "grid_common.hpp"
#include "launchers.hpp"

namespace nasch {

using namespace grid;

namespace {

constexpr uint32_t kOsWaves = kOneStepThreads / 64u;

// Item of block b when n blocks are dealt to the 8 XCDs in turn: XCD x gets the
// x-th contiguous run of items (runs of ceil(n/8) items first, then floor(n/8)).
__device__ __forceinline__ uint32_t xcd_item(uint32_t b, uint32_t n) {
    const uint32_t xcd = b & 7u, idx = b >> 3;
    const uint32_t per = n >> 3, rem = n & 7u;
    return xcd < rem ? xcd * (per + 1u) + idx : rem * (per + 1u) + (xcd - rem) * per + idx;
}

template <int Q>
struct OneStepLds {
    RefineLds<Q> ref[kOsWaves];   // tied draws, per wave
    uint32_t occ[kOsWaves];       // occupancy of each wave's first word
    uint32_t eq[kOsWaves][8];     // cars with v3 == j (j = 1..8) of each wave's last word
    uint32_t flux[kOsWaves];
};

}  // namespace

// Step t of tile `tile` of ring R, from R.buf[par] to R.buf[par ^ 1].  The
// block's F(t) goes to *partial (if not null) and, from the warm-up on, into
// R.flux_acc.
template <int VMAX, int Q>
__device__ __forceinline__ void onestep_tile(const RingDesc& R, uint32_t tile, uint32_t t,
                                             uint32_t par, uint32_t* __restrict__ partial,
                                             OneStepLds<Q>& lds) {
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t L = R.L;
    const SlowParams sp = R.sp;
    const uint8_t* __restrict__ src = R.buf[par];
    uint8_t* __restrict__ dst = R.buf[par ^ 1u];
    const uint32_t own_start = tile * R.own;
    const uint32_t own_len = min(R.own, L - own_start);
    const uint32_t s0 = (own_start + L - (32u % L)) % L;   // ring cell of segment cell 0
    // the segment lies inside [0, L): aligned words, no reduction mod L
    const bool inside = own_start >= 32u && own_start - 32u + 32u * kOneStepThreads * Q <= L;
    const bool run = t < R.t_end;   // no step at or past t_end (the state is copied)

    uint32_t T[Q][VMAX + 1];
    uint32_t xw[Q];     // ring cell of each word's first cell
    bool aligned[Q];    // the word is one aligned 32-cell block of the ring
    uint32_t own[Q];    // owned cells of each word
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint32_t j = (wv * 64u + lane) * Q + q;
        uint32_t x0 = s0 + 32u * j;   // s0 < 2^31, 32 j < 2^15: no overflow
        uint32_t d[8];
        if (inside) {
            aligned[q] = true;
            load_bytes32(src + x0, d);
        } else {
            x0 %= L;
            aligned[q] = (x0 & 31u) == 0u && x0 + 32u <= L;
            if (aligned[q]) load_bytes32(src + x0, d);
            else gather_bytes_ring(src, L, x0, d);
        }
        xw[q] = x0;
        bytes_to_thermo<VMAX>(d, T[q]);
        const uint32_t lo = max(32u, 32u * j), hi = min(32u + own_len, 32u * j + 32u);
        own[q] = lo < hi ? bit_range(lo - 32u * j, hi - 32u * j) : 0u;
    }
    RefineLds<Q>& rl = lds.ref[wv];
#pragma unroll
    for (int q = 0; q < Q; ++q) rl.slow[lane * Q + q] = 0u;
    if (lane == 0u) lds.occ[wv] = T[0][0];
    __syncthreads();

    uint32_t fl = 0u;
    if constexpr (VMAX > 0) {
        if (run) {
            // occupancy of the word after the lane's last one
            const uint32_t occ_wave = lds.occ[wv + 1u < kOsWaves ? wv + 1u : wv];
            uint32_t occ_next = from_next_lane(T[0][0]);
            if (lane == 63u) occ_next = wv + 1u < kOsWaves ? occ_wave : 0u;
            uint32_t T2[Q][VMAX + 2];
            uint32_t S[Q], U[Q], moving[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const uint32_t occ = T[q][0];
                const uint32_t nxt = (q + 1 < Q) ? T[(q + 1) % Q][0] : occ_next;
                uint32_t A = 0u;
#pragma unroll
                for (int g = 1; g <= VMAX; ++g) {
                    A |= __builtin_amdgcn_alignbit(nxt, occ, g);   // car in cell i+g
                    T2[q][g] = T[q][g - 1] & ~A;                    // rules 1 and 2
                }
                T2[q][VMAX + 1] = 0u;
                moving[q] = T2[q][1];
                S[q] = 0u;
                U[q] = 0u;
            }
            // rule 3: the top nibble of R of 32 cars per Philox call, then the
            // wave's tied cars
            if (sp.thr != 0u) {
                const uint32_t draw_mode = inside ? kDrawAligned : kDrawGeneric;
                slow_hi<Q>(moving, xw, aligned, draw_mode, t, L, sp, S, U);
            }
            if ((sp.thr & 0x0FFFFFFFu) != 0u) {
                uint32_t seg0 = s0 + 2048u * Q * wv;   // ring cell of the wave's first cell
                if (!inside) seg0 %= L;
                slow_lo_wave<Q>(S, U, xw, L, seg0, inside ? kXNone : kXMod, t, sp, rl, lane);
            }
            uint32_t Eq[Q][VMAX + 1];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                uint32_t T3[VMAX + 2];
                T3[0] = T[q][0];
#pragma unroll
                for (int m = 1; m <= VMAX; ++m)
                    T3[m] = (T2[q][m] & ~S[q]) | (T2[q][m + 1] & S[q]);
                T3[VMAX + 1] = 0u;
#pragma unroll
                for (int m = 1; m <= VMAX; ++m) fl += __popc(T3[m] & own[q]);
#pragma unroll
                for (int j = 0; j <= VMAX; ++j) Eq[q][j] = T3[j] & ~T3[j + 1];
            }
            if (lane == 63u) {
#pragma unroll
                for (int j = 1; j <= VMAX; ++j) lds.eq[wv][j - 1] = Eq[Q - 1][j];
            }
            __syncthreads();
            // rule 4: cars with v3 == j move j cells right
            uint32_t prevEq[VMAX + 1];
#pragma unroll
            for (int j = 1; j <= VMAX; ++j) {
                const uint32_t from_wave = wv > 0u ? lds.eq[wv - 1u][j - 1] : 0u;
                prevEq[j] = from_prev_lane(Eq[Q - 1][j]);
                if (lane == 0u) prevEq[j] = from_wave;
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                uint32_t accm = 0u;
#pragma unroll
                for (int j = VMAX; j >= 1; --j) {
                    const uint32_t prv = (q > 0) ? Eq[(q + Q - 1) % Q][j] : prevEq[j];
                    accm |= __builtin_amdgcn_alignbit(Eq[q][j], prv, 32 - j);
                    T[q][j] = accm;
                }
                T[q][0] = accm | Eq[q][0];
            }
        }
    }

    // F(t) of the tile: one partial per block, folded per ring by the fold kernel
    const uint32_t wtot = wave_total(fl);
    if (lane == 0u) lds.flux[wv] = wtot;
    __syncthreads();
    if (threadIdx.x == 0u) {
        uint32_t total = 0u;
#pragma unroll
        for (uint32_t w = 0; w < kOsWaves; ++w) total += lds.flux[w];
        if (partial) *partial = total;
        if (R.flux_acc && run && (uint64_t)t >= R.warmup && total)
            atomicAdd(R.flux_acc, (unsigned long long)total);
    }

    // store the owned cells (they lie in [0, L) and start on a word boundary)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (own[q] == 0u) continue;
        uint32_t d[8];
        thermo_to_bytes<VMAX>(T[q], d);
        store_bytes(dst, xw[q], own[q], d);
    }
}

// One step of every item (ring, tile) of a launch sequence: step and buffer
// parity from the device clock, F(t) partials per item for the fold kernel.
template <int VMAX, int Q>
__global__ __launch_bounds__(kOneStepThreads) void grid_onestep_kernel(
    const RingDesc* __restrict__ rings, const TileItem* __restrict__ items, uint32_t n_items,
    uint32_t* __restrict__ partials, const Clock* __restrict__ clk, uint32_t s_off,
    uint32_t launch_idx) {
    __shared__ OneStepLds<Q> lds;
    const uint32_t item = xcd_item(blockIdx.x, n_items);
    const TileItem it = items[item];
    const RingDesc& R = rings[it.ring];
    const uint32_t t = clk->t + R.t + s_off;
    const uint32_t par = (clk->parity + R.parity + launch_idx) & 1u;
    onestep_tile<VMAX, Q>(R, it.tile, t, par, R.flux_log ? partials + item : nullptr, lds);
}

// One step t of every tile of one ring described by value (buf[0] is read,
// buf[1] written): the launch of the stateless device-buffer entry points.
// partials[tile] receives each tile's F(t).
template <int VMAX, int Q>
__global__ __launch_bounds__(kOneStepThreads) void grid_onestep_direct_kernel(
    const RingDesc R, uint32_t ntiles, uint32_t* __restrict__ partials, uint32_t t) {
    __shared__ OneStepLds<Q> lds;
    const uint32_t tile = xcd_item(blockIdx.x, ntiles);
    onestep_tile<VMAX, Q>(R, tile, t, 0u, partials + tile, lds);
}

// *out = the sum of n uint32 partials (one block).
__global__ __launch_bounds__(256) void sum_partials_kernel(const uint32_t* __restrict__ partials,
                                                           uint32_t n,
                                                           unsigned long long* __restrict__ out) {
    __shared__ unsigned long long s[4];
    unsigned long long acc = 0;
    for (uint32_t i = threadIdx.x; i < n; i += 256u) acc += partials[i];
    // F(t) can pass 2^32 (up to 2^31 cars of v <= 8), so a lane's sum (below
    // 2^27) is added across the wave as its low 16 bits and the rest separately
    const uint32_t lo = wave_total((uint32_t)(acc & 0xFFFFu));
    const uint32_t hi = wave_total((uint32_t)(acc >> 16));
    if ((threadIdx.x & 63u) == 0u)
        s[threadIdx.x >> 6] = (unsigned long long)lo + ((unsigned long long)hi << 16);
    __syncthreads();
    if (threadIdx.x == 0u) *out = s[0] + s[1] + s[2] + s[3];
}

namespace {
template <int Q>
hipError_t launch_os_q(uint32_t vmax, dim3 grid, hipStream_t s, const RingDesc* rings,
                       const TileItem* items, uint32_t n_items, uint32_t* partials,
                       const Clock* clk, uint32_t s_off, uint32_t launch_idx) {
#define NASCH_ONESTEP_CASE(V)                                                                   \
    case V:                                                                                     \
        NASCH_LAUNCH((grid_onestep_kernel<V, Q>), grid, dim3(kOneStepThreads), 0, s, rings,     \
                     items, n_items, partials, clk, s_off, launch_idx);                         \
        break;
    switch (vmax) {
        NASCH_ONESTEP_CASE(0)
        NASCH_ONESTEP_CASE(1)
        NASCH_ONESTEP_CASE(2)
        NASCH_ONESTEP_CASE(3)
        NASCH_ONESTEP_CASE(4)
        NASCH_ONESTEP_CASE(5)
        NASCH_ONESTEP_CASE(6)
        NASCH_ONESTEP_CASE(7)
        NASCH_ONESTEP_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef NASCH_ONESTEP_CASE
    return hipGetLastError();
}
}  // namespace

hipError_t launch_grid_onestep_direct(const RingDesc& R, uint32_t ntiles, uint32_t* partials,
                                      uint32_t t, unsigned long long* flux, hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    const dim3 grid(ntiles);
#define NASCH_ONESTEP_DIRECT_CASE(V)                                                            \
    case V:                                                                                     \
        NASCH_LAUNCH((grid_onestep_direct_kernel<V, kOneStepQ>), grid, dim3(kOneStepThreads),   \
                     0, s, R, ntiles, partials, t);                                             \
        break;
    switch (R.vmax) {
        NASCH_ONESTEP_DIRECT_CASE(0)
        NASCH_ONESTEP_DIRECT_CASE(1)
        NASCH_ONESTEP_DIRECT_CASE(2)
        NASCH_ONESTEP_DIRECT_CASE(3)
        NASCH_ONESTEP_DIRECT_CASE(4)
        NASCH_ONESTEP_DIRECT_CASE(5)
        NASCH_ONESTEP_DIRECT_CASE(6)
        NASCH_ONESTEP_DIRECT_CASE(7)
        NASCH_ONESTEP_DIRECT_CASE(8)
        default:
            return hipErrorInvalidValue;
    }
#undef NASCH_ONESTEP_DIRECT_CASE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !flux) return e;
    NASCH_LAUNCH(sum_partials_kernel, dim3(1), dim3(256), 0, s, partials, ntiles, flux);
    return hipGetLastError();
}

hipError_t launch_grid_onestep(uint32_t vmax, uint32_t q, const RingDesc* rings,
                               const TileItem* items, uint32_t n_items, uint32_t* partials,
                               const Clock* clk, uint32_t s_off, uint32_t launch_idx,
                               hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    const dim3 grid(n_items);
    switch (q) {
        case 1: return launch_os_q<1>(vmax, grid, s, rings, items, n_items, partials, clk, s_off, launch_idx);
        case 2: return launch_os_q<2>(vmax, grid, s, rings, items, n_items, partials, clk, s_off, launch_idx);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nasch
