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
// Tiles.  A wave handles a tile as a segment of 64 Q consecutive 32-cell
// words, lane l holding words l Q .. l Q + Q - 1.  Segment word 0 and the last
// word are a one-word halo: the first only supplies the cars that drive into
// the tile (at most vmax <= 8 cells), the last only the occupancy that the
// tile's front cars see; the tile owns the 32 (64 Q - 2) cells in between.
// Neighbouring words come through DPP lane shifts, so the waves never wait
// for each other.
//
// Memory accesses.  A tile inside the ring is 2 KiB of contiguous bytes; the
// wave reads it with two loads of 16 bytes per lane (each 1 KiB contiguous, the
// fastest form measured here) and regroups the bytes into the lanes' 32-byte
// words through 2 KiB of LDS per wave, and writes a whole tile back the same way
// (its halo words' chunks masked off) with non-temporal stores (1 % faster
// than plain ones here).  Loading each lane's own 32 bytes directly (two
// 16-byte loads 32 bytes apart) measured 4 % slower.
//
// Streaming.  One tile per wave and one launch over all tiles: on this GPU a
// launch whose waves each move one tile and exit streams faster (5.8 TB/s for
// the bare copy of this access pattern) than persistent waves that loop over
// tiles (5.0 - 5.3 TB/s, with or without prefetching the next tile), and two
// tiles per wave measured slower too.  The 8 waves of a block take 8
// consecutive tiles and add their F(t) into one partial (blocks of 1, 2, 4
// and 16 waves measured 9, 4, 2 and 1 % slower); blocks dealt to one XCD (the
// 8 XCDs take blocks in turn) take consecutive tiles.
//
// F(t).  Each block stores its sum as one partial; the first waves of the
// first 64 blocks of the next launch add the partials up in 64 chunks, each
// into the log entry with one atomic add (a launch of their own after the
// last step).  Consecutive launches alternate between two sets of partials.
// A fold kernel of its own after every step measured about 1 % slower (381.4
// against 378.2 - 378.7 ms for 1000 steps of the 2^30-cell ring).
//
// Segment cell i is ring cell (own_start - 32 + i) mod L.  A tile whose
// segment lies inside [0, L) is the common case and takes aligned 16-byte
// loads and stores with no reduction mod L; the first tile, a last tile that
// runs past the end of the ring and every ring shorter than a segment read the
// segment cell by cell where it crosses the end (the periodic images of a
// short ring are exact by periodicity) and draw rule 3 across block edges.
// The branch is uniform over the wave.
//
// Open road (OPEN = true).  Segment cell i is road cell own_start - 32 + i;
// cells before 0 and from L on load as empty, and words stay aligned to the
// road's 32-cell blocks.  Tiles inside the road run the ring code.  A segment
// that holds cell L puts a stopped car there when the step's gate keeps the
// exit closed (the tile before a last tile of fewer than 8 cells holds it
// too), and the first tile adds the entering car (v = 0) to cell 0 after rule
// 4 if the gate lets one in and the cell was empty at the start of the step.
// The tile code is compiled once per kind of tile (inside, ring edge, open
// road edge): with the open road's branches in the interior tiles' code those
// ran 2 % slower.
#include "grid_common.hpp"
#include "launchers.hpp"

namespace nasch {

using namespace grid;

namespace {

constexpr uint32_t kOsWaves = kOneStepThreads / 64u;   // independent waves per block


// Item of block b when n blocks are dealt to the 8 XCDs in turn: XCD x gets the
// x-th contiguous run of items (runs of ceil(n/8) items first, then floor(n/8)).
__device__ __forceinline__ uint32_t xcd_item(uint32_t b, uint32_t n) {
    const uint32_t xcd = b & 7u, idx = b >> 3;
    const uint32_t per = n >> 3, rem = n & 7u;
    return xcd < rem ? xcd * (per + 1u) + idx : rem * (per + 1u) + (xcd - rem) * per + idx;
}

// Where a tile's segment lies on the ring.
struct OsTile {
    uint32_t own_start, own_len;
    uint32_t s0;       // ring cell of segment cell 0
    bool inside;       // the segment lies inside [0, L): aligned, no reduction mod L
};

template <int Q>
__device__ __forceinline__ OsTile os_tile(const RingDesc& R, uint32_t tile) {
    OsTile g;
    const uint32_t L = R.L;
    g.own_start = tile * R.own;
    g.own_len = min(R.own, L - g.own_start);
    g.s0 = (g.own_start + L - (32u % L)) % L;
    g.inside = g.own_start >= 32u && g.own_start - 32u + 32u * 64u * Q <= L;
    return g;
}

// The tile code is compiled once per kind of tile, so that the interior
// tiles' code holds no branch of the edge tiles': a tile whose segment lies
// inside [0, L), a ring's other tiles, and an open road's other tiles.
enum : int { kTileInside = 0, kTileRingEdge = 1, kTileOpenEdge = 2 };

// Ring cell of the first cell of segment word j (< 64 Q).
template <int MODE>
__device__ __forceinline__ uint32_t os_word_cell(const OsTile& g, uint32_t j, uint32_t L) {
    const uint32_t x0 = g.s0 + 32u * j;   // s0 < 2^31, 32 j < 2^14: no overflow
    return MODE == kTileInside ? x0 : x0 % L;
}

// Open road: road cell of the first cell of segment word j (negative before
// the road's start).
__device__ __forceinline__ int64_t os_road_cell(const OsTile& g, uint32_t j) {
    return (int64_t)g.own_start - 32 + 32 * (int64_t)j;
}

// The bytes of the lane's Q words of a tile of kind MODE.
template <int Q, int MODE>
__device__ __forceinline__ void os_load(const RingDesc& R, const uint8_t* __restrict__ src,
                                        uint32_t tile, uint32_t lane, uint32_t (&d)[Q][8],
                                        uint32_t* stage) {
    const OsTile g = os_tile<Q>(R, tile);
    if (MODE == kTileInside && Q == 1) {
        // two contiguous 1 KiB loads (16 bytes per lane), regrouped into the
        // lanes' 32-byte words through LDS
        const uint8_t* base = src + g.s0;
        const u32x4 a = *gmem(reinterpret_cast<const u32x4*>(base + 16u * lane));
        const u32x4 b = *gmem(reinterpret_cast<const u32x4*>(base + 1024u + 16u * lane));
        *reinterpret_cast<u32x4*>(stage + 4u * lane) = a;
        *reinterpret_cast<u32x4*>(stage + 256u + 4u * lane) = b;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const u32x4 c = *reinterpret_cast<const u32x4*>(stage + 8u * lane);
        const u32x4 e = *reinterpret_cast<const u32x4*>(stage + 8u * lane + 4u);
        d[0][0] = c.x; d[0][1] = c.y; d[0][2] = c.z; d[0][3] = c.w;
        d[0][4] = e.x; d[0][5] = e.y; d[0][6] = e.z; d[0][7] = e.w;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        return;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if constexpr (MODE == kTileOpenEdge) {
            const int64_t p0 = os_road_cell(g, lane * Q + q);
            if (p0 >= 0 && p0 < (int64_t)R.L) {
                load_bytes_open(src, R.L, (uint32_t)p0, d[q]);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) d[q][i] = 0xFFFFFFFFu;   // off the road: empty
            }
        } else {
            const uint32_t x0 = os_word_cell<MODE>(g, lane * Q + q, R.L);
            if (MODE == kTileInside || ((x0 & 31u) == 0u && x0 + 32u <= R.L))
                load_bytes32(src + x0, d[q]);
            else
                gather_bytes_ring(src, R.L, x0, d[q]);
        }
    }
}

// Step t of one tile of kind MODE from the bytes d of the lane's words:
// writes the owned cells to dst and returns the lane's share of F(t) (owned
// cars only).
template <int VMAX, int Q, int MODE>
__device__ __forceinline__ uint32_t os_step(const RingDesc& R, uint8_t* __restrict__ dst,
                                            uint32_t tile, uint32_t t, bool run, uint32_t lane,
                                            const uint32_t (&d)[Q][8], RefineLds<Q>& rl,
                                            uint32_t* stage) {
    const uint32_t L = R.L;
    const SlowParams sp = R.sp;
    constexpr bool OPEN = MODE == kTileOpenEdge;
    constexpr bool inside = MODE == kTileInside;
    const OsTile g = os_tile<Q>(R, tile);
    uint32_t T[Q][VMAX + 1];
    uint32_t xw[Q];     // ring cell of each word's first cell
    bool aligned[Q];    // the word is one aligned 32-cell block of the ring
    uint32_t own[Q];    // owned cells of each word
    uint32_t obst[Q];   // open road: cell L
    uint32_t inj[Q];    // open road: cell 0
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint32_t j = lane * Q + q;
        if constexpr (OPEN) {
            // words before cell 0 hold no car; their draws are never used
            const int64_t p0 = os_road_cell(g, j);
            xw[q] = p0 < 0 ? 0u : (uint32_t)p0;
            aligned[q] = true;
            obst[q] = (p0 <= (int64_t)L && (int64_t)L < p0 + 32) ? 1u << (uint32_t)(L - p0) : 0u;
            inj[q] = p0 == 0 ? 1u : 0u;
        } else {
            xw[q] = os_word_cell<MODE>(g, j, L);
            aligned[q] = inside || ((xw[q] & 31u) == 0u && xw[q] + 32u <= L);
            obst[q] = inj[q] = 0u;
        }
        bytes_to_thermo<VMAX>(d[q], T[q]);
        const uint32_t lo = max(32u, 32u * j), hi = min(32u + g.own_len, 32u * j + 32u);
        own[q] = lo < hi ? bit_range(lo - 32u * j, hi - 32u * j) : 0u;
    }
    bool enter = false;
    uint32_t empty0[Q];   // open road: cell 0, if it is empty at the start of the step
    if (OPEN && run) {
        bool exit_open;
        gate_draw(t, sp, R.thr_in, R.thr_out, enter, exit_open);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (!exit_open) T[q][0] |= obst[q];   // stopped car in cell L, v = 0
            empty0[q] = inj[q] & ~T[q][0];
        }
    }

    uint32_t fl = 0u;
    if constexpr (VMAX > 0) {
        if (run) {
            uint32_t dig[4] = {0u, 0u, 0u, 0u};   // F(t) as binary digit counts
            // occupancy of the word after the lane's last one (lane 63's is the
            // halo word's, whose own results are not kept)
            const uint32_t occ_next = from_next_lane(T[0][0]);
            uint32_t T2[Q][VMAX + 2];
            uint32_t S[Q], U[Q], moving[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const uint32_t occ = T[q][0];
                const uint32_t nxt = (q + 1 < Q) ? T[(q + 1) % Q][0] : occ_next;
                uint32_t A = 0u;
#pragma unroll
                for (int gg = 1; gg <= VMAX; ++gg) {
                    A |= __builtin_amdgcn_alignbit(nxt, occ, gg);   // car in cell i+gg
                    T2[q][gg] = T[q][gg - 1] & ~A;                   // rules 1 and 2
                }
                T2[q][VMAX + 1] = 0u;
                moving[q] = T2[q][1];
                S[q] = 0u;
                U[q] = 0u;
            }
            // rule 3: the top nibble of R of 32 cars per Philox call, then the
            // wave's tied cars
            if (sp.thr != 0u) {
                slow_hi<Q>(moving, xw, aligned,
                           (OPEN || inside) ? kDrawAligned : kDrawGeneric, t, L, sp, S, U);
            }
            // a queued car's ring cell: segment cell + s0 (an open road's
            // segment cell 0 is road cell own_start - 32, taken modulo 2^32)
            if ((sp.thr & 0x0FFFFFFFu) != 0u)
                slow_lo_wave<Q>(S, U, xw, L, OPEN ? g.own_start - 32u : g.s0,
                                (OPEN || inside) ? kXNone : kXMod, t, sp, rl, lane);
            uint32_t Eq[Q][VMAX + 1];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                uint32_t T3[VMAX + 2];
                T3[0] = T[q][0];
#pragma unroll
                for (int m = 1; m <= VMAX; ++m)
                    T3[m] = select_bits(S[q], T2[q][m + 1], T2[q][m]);
                T3[VMAX + 1] = 0u;
                add_speed_digits<VMAX, true>(T3, own[q], dig);
#pragma unroll
                for (int j = 1; j <= VMAX; ++j) Eq[q][j] = T3[j] & ~T3[j + 1];
                Eq[q][0] = T3[1];   // the moving cars; the stopped ones are T3[0] & ~T3[1]
            }
            // rule 4: cars with v3 == j move j cells right (lane 0's incoming
            // cars are unknown: its word is the halo)
            uint32_t prevEq[VMAX + 1];
#pragma unroll
            for (int j = 1; j <= VMAX; ++j) prevEq[j] = from_prev_lane(Eq[Q - 1][j]);
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                uint32_t accm = 0u;
#pragma unroll
                for (int j = VMAX; j >= 1; --j) {
                    const uint32_t prv = (q > 0) ? Eq[(q + Q - 1) % Q][j] : prevEq[j];
                    accm |= __builtin_amdgcn_alignbit(Eq[q][j], prv, 32 - j);
                    T[q][j] = accm;
                }
                // occupancy: the moved cars and the stopped ones, accm | (T3[0] & ~T3[1])
                T[q][0] = __builtin_amdgcn_bitop3_b32(T[q][0], Eq[q][0], accm, 0xBA);
            }
            fl = speed_sum(dig);
        }
    }
    if (OPEN && run && enter) {
#pragma unroll
        for (int q = 0; q < Q; ++q) T[q][0] |= empty0[q];   // entering car in cell 0, v = 0
    }

    // store the owned cells (they lie in [0, L) and start on a word boundary)
    if (Q == 1 && inside && g.own_len == 32u * (64u * Q - 2u)) {
        // a whole tile: regroup through LDS into two contiguous 1 KiB stores,
        // without the halo words (chunks 0, 1 and 126, 127)
        uint32_t dd[8];
        thermo_to_bytes<VMAX>(T[0], dd);
        *reinterpret_cast<u32x4*>(stage + 8u * lane) = u32x4{dd[0], dd[1], dd[2], dd[3]};
        *reinterpret_cast<u32x4*>(stage + 8u * lane + 4u) = u32x4{dd[4], dd[5], dd[6], dd[7]};
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const u32x4 a = *reinterpret_cast<const u32x4*>(stage + 4u * lane);
        const u32x4 b = *reinterpret_cast<const u32x4*>(stage + 256u + 4u * lane);
        uint8_t* base = dst + g.s0;
        if (lane >= 2u) __builtin_nontemporal_store(a, reinterpret_cast<u32x4*>(base + 16u * lane));
        if (lane < 62u) __builtin_nontemporal_store(b, reinterpret_cast<u32x4*>(base + 1024u + 16u * lane));
        return fl;
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (own[q] == 0u) continue;
        uint32_t dd[8];
        thermo_to_bytes<VMAX>(T[q], dd);
        store_bytes(dst, xw[q], own[q], dd);
    }
    return fl;
}

// Step t of tile 8 b + wave of ring R (b: the block's tile group), from
// R.buf[par] to R.buf[par ^ 1].  The block's F(t) goes to *partial (if not
// null), to *whole (if not null: a launch of one block, whose F(t) is the
// ring's) and, from the warm-up on, is added into R.flux_acc.
template <int VMAX, int Q, bool OPEN>
__device__ __forceinline__ void os_block(const RingDesc& R, uint32_t b, uint32_t t, uint32_t par,
                                         uint32_t* __restrict__ partial,
                                         unsigned long long* __restrict__ whole,
                                         RefineLds<Q>* ref, uint32_t* s_flux, uint32_t* s_stage) {
    const uint32_t wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t tile = b * kOsWaves + wib;
    const bool run = t < R.t_end;   // no step at or past t_end (the state is copied)
    uint32_t fl = 0u;
    if (tile < R.ntiles) {
        RefineLds<Q>& rl = ref[wib];
#pragma unroll
        for (int q = 0; q < Q; ++q) rl.slow[lane * Q + q] = 0u;
        if (lane == 0u) rl.n = 0u;
        uint32_t d[Q][8];
        uint32_t* stage = s_stage + 512u * wib;
        // the code of the tile's kind (wave-uniform): an open road's tiles
        // inside [0, L) run the ring's code
        uint8_t* __restrict__ dst = R.buf[par ^ 1u];
        if (os_tile<Q>(R, tile).inside) {
            os_load<Q, kTileInside>(R, R.buf[par], tile, lane, d, stage);
            fl = os_step<VMAX, Q, kTileInside>(R, dst, tile, t, run, lane, d, rl, stage);
        } else if constexpr (OPEN) {
            os_load<Q, kTileOpenEdge>(R, R.buf[par], tile, lane, d, stage);
            fl = os_step<VMAX, Q, kTileOpenEdge>(R, dst, tile, t, run, lane, d, rl, stage);
        } else {
            os_load<Q, kTileRingEdge>(R, R.buf[par], tile, lane, d, stage);
            fl = os_step<VMAX, Q, kTileRingEdge>(R, dst, tile, t, run, lane, d, rl, stage);
        }
    }
    const uint32_t wtot = wave_total(fl);
    if (lane == 0u) s_flux[wib] = wtot;
    __syncthreads();
    if (threadIdx.x == 0u) {
        uint32_t total = 0u;
#pragma unroll
        for (uint32_t w = 0; w < kOsWaves; ++w) total += s_flux[w];
        if (partial) *partial = total;
        if (whole) *whole = total;
        if (R.flux_acc && run && (uint64_t)t >= R.warmup && total)
            atomicAdd(R.flux_acc, (unsigned long long)total);
    }
}

}  // namespace

// One step of a ring (RingDesc at `ring`, step and buffer parity from the
// device clock).  With a flux log and more than one block, every block stores
// its F(t) in partial set launch_idx of `scratch` (sets of gridDim.x words),
// and (fold_prev) the first wave of each of the first 64 blocks first adds a
// chunk of the previous launch's set into its log entry.
template <int VMAX, int Q, bool OPEN>
__global__ __launch_bounds__(kOneStepThreads) void grid_onestep_kernel(
    const RingDesc* __restrict__ ring, uint32_t* __restrict__ scratch,
    const Clock* __restrict__ clk, uint32_t s_off, uint32_t launch_idx, uint32_t fold_prev) {
    __shared__ RefineLds<Q> s_ref[kOsWaves];
    __shared__ uint32_t s_flux[kOsWaves];
    __shared__ uint32_t s_stage[kOsWaves * 512];
    const RingDesc& R = *ring;
    const uint32_t t = clk->t + R.t + s_off;
    const uint32_t nb = gridDim.x;
    const uint32_t m = min(kFoldBlocks, nb);
    if (fold_prev && blockIdx.x < m && threadIdx.x < 64u) {
        const unsigned long long f = chunk_sum(scratch + (size_t)((launch_idx + 1u) & 1u) * nb,
                                               nb, blockIdx.x, m, threadIdx.x);
        if (threadIdx.x == 0u && f) atomicAdd(&R.flux_log[(uint64_t)t - 1u - R.log_t0], f);
    }
    const uint32_t b = xcd_item(blockIdx.x, nb);
    const uint32_t par = (clk->parity + R.parity + launch_idx) & 1u;
    // one block (a ring of at most 8 tiles) writes F(t) itself
    const bool one = nb == 1u && R.flux_log;
    os_block<VMAX, Q, OPEN>(
        R, b, t, par,
        R.flux_log && !one ? scratch + (size_t)(launch_idx & 1u) * nb + blockIdx.x : nullptr,
        one ? R.flux_log + ((uint64_t)t - R.log_t0) : nullptr, s_ref, s_flux, s_stage);
}

// One step t of a ring described by value (buf[0] is read, buf[1] written):
// the launch of the stateless device-buffer entry points.  With flux and more
// than one block, *flux is cleared here and the fold adds the partials to it.
template <int VMAX, int Q>
__global__ __launch_bounds__(kOneStepThreads) void grid_onestep_direct_kernel(
    const RingDesc R, uint32_t* __restrict__ partials, uint32_t t,
    unsigned long long* __restrict__ flux) {
    __shared__ RefineLds<Q> s_ref[kOsWaves];
    __shared__ uint32_t s_flux[kOsWaves];
    __shared__ uint32_t s_stage[kOsWaves * 512];
    const uint32_t b = xcd_item(blockIdx.x, gridDim.x);
    // one block writes F(t) itself
    const bool one = gridDim.x == 1u;
    if (flux && !one && blockIdx.x == 0u && threadIdx.x == 0u) *flux = 0ull;
    os_block<VMAX, Q, false>(R, b, t, 0u, flux && !one ? partials + blockIdx.x : nullptr,
                             one ? flux : nullptr, s_ref, s_flux, s_stage);
}

// Adds a launch's n partials into *out, or into the ring's flux log at step
// s_off of the run (when ring is given): block c adds chunk c of gridDim.x.
__global__ __launch_bounds__(64) void fold_partials_kernel(const uint32_t* __restrict__ partials,
                                                           uint32_t n,
                                                           unsigned long long* __restrict__ out,
                                                           const RingDesc* __restrict__ ring,
                                                           const Clock* __restrict__ clk,
                                                           uint32_t s_off) {
    const unsigned long long f = chunk_sum(partials, n, blockIdx.x, gridDim.x, threadIdx.x);
    if (threadIdx.x != 0u || !f) return;
    if (ring) {
        const uint64_t t = (uint64_t)clk->t + ring->t + s_off;
        out = ring->flux_log + (t - ring->log_t0);
    }
    atomicAdd(out, f);
}

namespace {

// Blocks of a one-step launch: one tile per wave.
uint32_t os_blocks(uint32_t ntiles) { return std::max(1u, (ntiles + kOsWaves - 1u) / kOsWaves); }

// KERNEL<vmax, TARGS...> for the launch's vmax; TARGS is a parenthesised list.
#define NASCH_OS_UNPAREN(...) __VA_ARGS__
#define NASCH_OS_VMAX_SWITCH(KERNEL, TARGS, ...)                                               \
    switch (vmax) {                                                                            \
        case 0: NASCH_LAUNCH((KERNEL<0, NASCH_OS_UNPAREN TARGS>), __VA_ARGS__); break;          \
        case 1: NASCH_LAUNCH((KERNEL<1, NASCH_OS_UNPAREN TARGS>), __VA_ARGS__); break;          \
        case 2: NASCH_LAUNCH((KERNEL<2, NASCH_OS_UNPAREN TARGS>), __VA_ARGS__); break;          \
        case 3: NASCH_LAUNCH((KERNEL<3, NASCH_OS_UNPAREN TARGS>), __VA_ARGS__); break;          \
        case 4: NASCH_LAUNCH((KERNEL<4, NASCH_OS_UNPAREN TARGS>), __VA_ARGS__); break;          \
        case 5: NASCH_LAUNCH((KERNEL<5, NASCH_OS_UNPAREN TARGS>), __VA_ARGS__); break;          \
        case 6: NASCH_LAUNCH((KERNEL<6, NASCH_OS_UNPAREN TARGS>), __VA_ARGS__); break;          \
        case 7: NASCH_LAUNCH((KERNEL<7, NASCH_OS_UNPAREN TARGS>), __VA_ARGS__); break;          \
        case 8: NASCH_LAUNCH((KERNEL<8, NASCH_OS_UNPAREN TARGS>), __VA_ARGS__); break;          \
        default: return hipErrorInvalidValue;                                                  \
    }

hipError_t fold(const uint32_t* partials, uint32_t n, unsigned long long* out,
                const RingDesc* ring, const Clock* clk, uint32_t s_off, hipStream_t s) {
    NASCH_LAUNCH(fold_partials_kernel, dim3(std::min(kFoldBlocks, n)), dim3(64), 0, s, partials,
                 n, out, ring, clk, s_off);
    return hipGetLastError();
}

}  // namespace

uint32_t onestep_partials(uint32_t ntiles) { return os_blocks(ntiles); }

hipError_t launch_grid_onestep(uint32_t vmax, bool open, uint32_t ntiles, const RingDesc* ring,
                               uint32_t* scratch, bool log, const Clock* clk, uint32_t s_off,
                               uint32_t launch_idx, bool first, bool last, hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    const uint32_t nb = os_blocks(ntiles);
    const bool fold_log = log && nb > 1u;   // one block writes F(t) itself
    const uint32_t fold_prev = (fold_log && !first) ? 1u : 0u;
    if (open) {
        NASCH_OS_VMAX_SWITCH(grid_onestep_kernel, (kOneStepQ, true), dim3(nb),
                             dim3(kOneStepThreads), 0, s, ring, scratch, clk, s_off, launch_idx,
                             fold_prev)
    } else {
        NASCH_OS_VMAX_SWITCH(grid_onestep_kernel, (kOneStepQ, false), dim3(nb),
                             dim3(kOneStepThreads), 0, s, ring, scratch, clk, s_off, launch_idx,
                             fold_prev)
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !fold_log || !last) return e;
    return fold(scratch + (size_t)(launch_idx & 1u) * nb, nb, nullptr, ring, clk, s_off, s);
}

hipError_t launch_grid_onestep_direct(const RingDesc& R, uint32_t* scratch, uint32_t t,
                                      unsigned long long* flux, hipStream_t s) {
    if (R.ntiles == 0) return hipSuccess;
    const uint32_t vmax = R.vmax;
    const uint32_t nb = os_blocks(R.ntiles);
    NASCH_OS_VMAX_SWITCH(grid_onestep_direct_kernel, (kOneStepQ), dim3(nb),
                         dim3(kOneStepThreads), 0, s, R, scratch, t, flux)
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !flux || nb == 1u) return e;   // one block wrote F(t) itself
    return fold(scratch, nb, flux, nullptr, nullptr, 0u, s);
}

#undef NASCH_OS_VMAX_SWITCH
#undef NASCH_OS_UNPAREN

}  // namespace nasch
