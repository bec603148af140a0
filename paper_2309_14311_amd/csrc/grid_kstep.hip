// grid_kstep.hip -- temporal-blocked grid kernel: k steps of rules 1-4 per launch,
// with the road held bit-sliced in registers.
//
// Layout.  Each wave owns one segment of 64 lanes x Q words x 32 cells.  A lane
// holds Q consecutive 32-cell words; word q of lane l covers segment cells
// [32 (l Q + q), +32).  A word is stored as VMAX + 1 bit planes:
//   T[0]    occupancy (bit i set iff a car is in cell i),
//   T[m]    the car in cell i has v >= m   (m = 1..VMAX, a thermometer code).
// In this form the four rules become a few bitwise operations per 32 cells:
//   rule 1   v1 >= m  <=>  T[m-1]                (m <= vmax; T[0] for m = 1)
//   rule 2   gap >= m <=>  cells i+1..i+m empty  (OR of shifted occupancies)
//            v2 >= m  <=>  T[m-1] & (gap >= m)
//   rule 3   a slow-down mask S (moving cars with R < thr) shifts the
//            thermometer down by one: v3 >= m <=> S ? v2 >= m+1 : v2 >= m
//   rule 4   the cars with v3 == j are shifted j cells to the right, and the
//            new thermometer is the suffix-OR of the shifted classes.
// The road is stored in HBM in the same planes (RingDesc), so a launch loads
// and stores VMAX + 1 words per 32 cells and converts nothing (the one-step
// kernel, grid_onestep.hip, works on the byte form instead).
// Neighbouring words come from the same lane or, at lane edges, from lane +-1
// by cross-lane shuffles.  The segment is the tile's owned cells plus a halo
// of H >= k*vmax cells on each side (read modulo L, so short rings repeat
// periodically); after k steps only the owned cells are exact, and only they
// are written back and counted in F(t).  Segments never talk to each other:
// one launch reads one ping-pong buffer and writes the other.
//
// Rule 3 draws.  The top 4 bits of R for a 32-cell block are the four words of
// one Philox call, bit-sliced already, so one call serves 32 cells; a lane
// compares them with the top nibble of thr bit-sliced as well.  Only cars whose
// top nibble ties (1 in 16) need the per-cell low 28 bits.
//
// Open road (OPEN = true).  Segment cell j is road cell own_start - H + j,
// which may lie before 0 or past L-1; such cells load as empty and words stay
// aligned to the road's 32-cell blocks.  A segment that reaches past L-1
// clears those cells at the start of every step (cars there have left) and,
// when the step's gate keeps the exit closed, puts a stopped car in cell L,
// which rules 1-2 then see like any car.  A segment that contains cell 0 adds
// the entering car (v = 0) after rule 4 if the gate lets one in and the cell
// was empty at the start of the step.  Both branches are uniform over the wave
// and cost nothing in the other segments.
#include "grid_common.hpp"
#include "launchers.hpp"

namespace nasch {

using namespace grid;

// One wave advances one tile item by up to k steps.  F(t) of a ring with a
// flux log goes to partials[s * n_items + item] (summed per ring and step by
// the fold kernel); flux_acc gets one atomic per wave.
template <int VMAX, int Q, bool OPEN>
__device__ __forceinline__ void kstep_tile(const RingDesc& R, const TileItem it, uint32_t item,
                                           uint32_t n_items, uint32_t* __restrict__ partials,
                                           uint32_t lane, uint32_t k,
                                           const Clock* __restrict__ clk, uint32_t s_off,
                                           uint32_t launch_idx, RefineLds<Q>& rl) {
    const uint32_t L = R.L;
    const SlowParams sp = R.sp;
    const uint32_t t0 = clk->t + R.t + s_off;
    uint32_t nsteps = k;
    if (R.t_end != 0xFFFFFFFFu) nsteps = R.t_end > t0 ? min(k, R.t_end - t0) : 0u;
    const uint32_t par = (clk->parity + R.parity + launch_idx) & 1u;
    const uint32_t nw = R.nw;
    const uint32_t* __restrict__ src = R.pl[par];
    uint32_t* __restrict__ dst = R.pl[par ^ 1u];

    const uint32_t own_start = it.tile * R.own;
    const uint32_t own_len = min(R.own, L - own_start);
    const uint32_t H = R.halo;
    const uint32_t seg_len = own_len + 2u * H;
    const uint32_t s0 = (own_start + L - (H % L)) % L;  // ring cell of segment cell 0
    const bool short_ring = L < kstep_segment(Q);        // the segment wraps the ring
    const int64_t base = (int64_t)own_start - (int64_t)H;  // open road: cell of segment cell 0
    // open road: does the segment hold cell 0 / cells at or past L (wave-uniform)
    const bool edge_l = OPEN && base <= 0;
    const bool edge_r = OPEN && base + (int64_t)seg_len > (int64_t)L;

    uint32_t T[Q][VMAX + 1];
    uint32_t xw[Q];       // ring cell of each word's first cell
    bool aligned[Q];      // word is one aligned rule-3 block
    uint32_t own[Q];      // owned cells of each word
    uint32_t keep[Q];     // open road: cells before L
    uint32_t obst[Q];     // open road: cell L
    uint32_t inj[Q];      // open road: cell 0

    // ---- load the segment's words as bit planes (from the planes in HBM, or
    // from the byte form converted in registers)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint32_t j0 = 32u * (lane * Q + q);
        const int64_t p0 = base + j0;   // open road: cell of the word's first cell
        uint32_t x0;
        if constexpr (OPEN) {
            // words before cell 0 hold no car; their draws are never used
            x0 = p0 < 0 ? 0u : (uint32_t)p0;
            aligned[q] = true;
            keep[q] = p0 >= (int64_t)L ? 0u
                      : (p0 + 32 <= (int64_t)L ? 0xFFFFFFFFu : (1u << (uint32_t)(L - p0)) - 1u);
            obst[q] = (p0 <= (int64_t)L && (int64_t)L < p0 + 32) ? 1u << (uint32_t)(L - p0) : 0u;
            inj[q] = p0 == 0 ? 1u : 0u;
        } else {
            // s0 < L < 2^31 and j0 < the segment length: at most one
            // subtraction unless the ring is shorter than the segment (a
            // wave-uniform branch)
            x0 = s0 + j0;
            if (short_ring) {
                x0 %= L;
            } else {
                x0 = min(x0, x0 - L);   // x0 - L wraps above x0 unless x0 >= L
            }
            aligned[q] = ((x0 & 31u) == 0u) && (x0 + 32u <= L);
            keep[q] = obst[q] = inj[q] = 0u;
        }
        xw[q] = x0;
        const uint32_t lo = max(H, j0), hi = min(H + own_len, j0 + 32u);
        own[q] = lo < hi ? bit_range(lo - j0, hi - j0) : 0u;

        // segment cells past seg_len stay empty; so do road cells outside
        // [0, L) on an open road
        const uint32_t valid = j0 + 32u <= seg_len ? 0xFFFFFFFFu
                               : (j0 < seg_len ? (1u << (seg_len - j0)) - 1u : 0u);
        if constexpr (OPEN) {
            if (p0 >= 0 && p0 < (int64_t)L) {
                const uint32_t v = valid & keep[q];
                const uint32_t w = (uint32_t)p0 >> 5;
#pragma unroll
                for (int m = 0; m <= VMAX; ++m) T[q][m] = *gmem(src + (size_t)m * nw + w) & v;
            } else {
#pragma unroll
                for (int m = 0; m <= VMAX; ++m) T[q][m] = 0u;
            }
        } else if (aligned[q]) {
            const uint32_t w = x0 >> 5;
#pragma unroll
            for (int m = 0; m <= VMAX; ++m) T[q][m] = *gmem(src + (size_t)m * nw + w) & valid;
        } else {
            gather_ring<VMAX>(src, nw, L, x0, T[q]);
#pragma unroll
            for (int m = 0; m <= VMAX; ++m) T[q][m] &= valid;
        }
    }

    // rule-3 tables of this wave
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        rl.slow[lane * Q + q] = 0u;
    }
    if (lane == 0u) rl.n = 0u;
    wave_sync_lds();
    uint32_t draw_mode = kDrawAligned;   // open roads: every word is aligned
    if constexpr (!OPEN) {
        bool all_aligned = true;
#pragma unroll
        for (int q = 0; q < Q; ++q) all_aligned = all_aligned && aligned[q];
        if (__builtin_amdgcn_ballot_w64(!all_aligned) != 0u) {
            // only waves at the end of a ring (or on a short one) get here
            bool all_two = true;
#pragma unroll
            for (int q = 0; q < Q; ++q) all_two = all_two && two_blocks(xw[q], L, nw);
            draw_mode = (L >= 64u && __builtin_amdgcn_ballot_w64(!all_two) == 0u) ? kDrawTwo
                                                                                 : kDrawGeneric;
        }
    }

    // segment cell -> ring cell for the tied cars' draws
    const uint32_t seg0 = OPEN ? (uint32_t)base : s0;
    const uint32_t x_mode = OPEN ? kXNone : (short_ring ? kXMod : kXSub);

    // ---- k steps
    uint32_t acc = 0u;
    // F(t) as binary digit counts (add_speed_digits), summed over the steps
    // that count: every step with a flux log, else the steps past the warm-up
    uint32_t dig[4] = {0u, 0u, 0u, 0u};
    uint32_t sum_prev = 0u;   // flux log: speed_sum(dig) after the previous step
    const bool log = R.flux_log != nullptr;
    // steps of this launch before the warm-up ends (their flux is not summed)
    // (compared as integers: min<uint64_t> here compiled to double-precision instructions)
    const uint64_t to_warm = R.warmup > (uint64_t)t0 ? R.warmup - t0 : 0u;
    const uint32_t s_warm = to_warm < nsteps ? (uint32_t)to_warm : nsteps;
    for (uint32_t s = 0; s < nsteps; ++s) {
        const uint32_t t = t0 + s;
        const bool need_fl = log || s >= s_warm;   // uniform over the wave
        bool enter = false;
        uint32_t empty0[Q];   // open road: cell 0, if it is empty at the start of the step
        if constexpr (OPEN) {
            if (edge_l || edge_r) {
                bool exit_open;
                gate_draw(t, sp, R.thr_in, R.thr_out, enter, exit_open);
                if (edge_r) {
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
#pragma unroll
                        for (int m = 0; m <= VMAX; ++m) T[q][m] &= keep[q];
                        if (!exit_open) T[q][0] |= obst[q];   // stopped car, v = 0
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) empty0[q] = inj[q] & ~T[q][0];
        }
        if constexpr (VMAX > 0) {
            const uint32_t occ_next = from_next_lane(T[0][0]);
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
            if (sp.thr != 0u) slow_hi<Q>(moving, xw, aligned, draw_mode, t, L, sp, S, U);  // rule 3
            if ((sp.thr & 0x0FFFFFFFu) != 0u)
                slow_lo_wave<Q>(S, U, xw, L, seg0, x_mode, t, sp, rl, lane);
            uint32_t Eq[Q][VMAX + 1];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                uint32_t T3[VMAX + 2];
                T3[0] = T[q][0];
#pragma unroll
                for (int m = 1; m <= VMAX; ++m)
                    T3[m] = select_bits(S[q], T2[q][m + 1], T2[q][m]);
                T3[VMAX + 1] = 0u;
                // (skipped in a warm-up step of a ring without a flux log)
                if (need_fl) add_speed_digits<VMAX, true>(T3, own[q], dig);
#pragma unroll
                for (int j = 1; j <= VMAX; ++j) Eq[q][j] = T3[j] & ~T3[j + 1];
                Eq[q][0] = T3[1];   // the moving cars; the stopped ones are T3[0] & ~T3[1]
            }
            // rule 4: cars with v3 == j move j cells right
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
        }
        if constexpr (OPEN) {
            if (edge_l && enter) {
#pragma unroll
                for (int q = 0; q < Q; ++q) T[q][0] |= empty0[q];   // entering car, v = 0
            }
        }
        if (log) {
            const uint32_t sum = speed_sum(dig);
            const uint32_t fl = sum - sum_prev;   // this lane's share of F(t)
            sum_prev = sum;
            const uint32_t total = wave_total(fl);
            if (lane == 0u) partials[(size_t)s * n_items + item] = total;
            acc += s >= s_warm ? fl : 0u;
        }
    }
    if (!log) acc = speed_sum(dig);   // only the steps past the warm-up were added
    if (R.flux_acc) {
        const uint32_t total = wave_total(acc);
        if (lane == 0u && total) atomicAdd(R.flux_acc, (unsigned long long)total);
    }

    // ---- store the owned cells (whole words: tiles start on word boundaries;
    // the road's last plane word keeps zeros past cell L-1, and its last byte
    // word is written cell by cell up to L-1)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        if (own[q] == 0u) continue;
        const uint32_t j0 = 32u * (lane * Q + q);
        const uint32_t w = (own_start + (j0 - H)) >> 5;
#pragma unroll
        for (int m = 0; m <= VMAX; ++m) *gmem(dst + (size_t)m * nw + w) = T[q][m] & own[q];
    }
}

// Blocks of one wave: a wave's slot frees as soon as its tile is done, which
// matters where the tiles' work differs (an ensemble's rings differ in vmax,
// p and density).  Blocks of 2, 4 and 8 waves measured 0.5, 2 and 3.5 % slower
// on the ensemble (the same on one large ring).
//
// All items of a launch share vmax (and the boundary): one specialisation.
template <int VMAX, int Q, bool OPEN>
__global__ __launch_bounds__(64) void grid_kstep_kernel(const RingDesc* __restrict__ rings,
                                                        const TileItem* __restrict__ items,
                                                        uint32_t n_items, uint32_t* partials,
                                                        uint32_t k, const Clock* __restrict__ clk,
                                                        uint32_t s_off, uint32_t launch_idx) {
    __shared__ RefineLds<Q> s_ref;
    const uint32_t wave = blockIdx.x;
    if (wave >= n_items) return;
    const TileItem it = items[wave];
    kstep_tile<VMAX, Q, OPEN>(rings[it.ring], it, wave, n_items, partials, threadIdx.x, k, clk,
                              s_off, launch_idx, s_ref);
}

// Items of different vmax in one launch: the branch on the ring's vmax is
// uniform over the wave.  OPEN: every ring of the launch is an open road.
template <int Q, bool OPEN>
__global__ __launch_bounds__(64) void grid_kstep_mixed_kernel(const RingDesc* __restrict__ rings,
                                                              const TileItem* __restrict__ items,
                                                              uint32_t n_items, uint32_t* partials,
                                                              uint32_t k,
                                                              const Clock* __restrict__ clk,
                                                              uint32_t s_off,
                                                              uint32_t launch_idx) {
    __shared__ RefineLds<Q> s_ref;
    const uint32_t wave = blockIdx.x;
    if (wave >= n_items) return;
    const TileItem it = items[wave];
    const RingDesc& R = rings[it.ring];
    const uint32_t lane = threadIdx.x;
    RefineLds<Q>& rl = s_ref;
    switch (R.vmax) {
        case 0: kstep_tile<0, Q, OPEN>(R, it, wave, n_items, partials, lane, k, clk, s_off, launch_idx, rl); break;
        case 1: kstep_tile<1, Q, OPEN>(R, it, wave, n_items, partials, lane, k, clk, s_off, launch_idx, rl); break;
        case 2: kstep_tile<2, Q, OPEN>(R, it, wave, n_items, partials, lane, k, clk, s_off, launch_idx, rl); break;
        case 3: kstep_tile<3, Q, OPEN>(R, it, wave, n_items, partials, lane, k, clk, s_off, launch_idx, rl); break;
        case 4: kstep_tile<4, Q, OPEN>(R, it, wave, n_items, partials, lane, k, clk, s_off, launch_idx, rl); break;
        case 5: kstep_tile<5, Q, OPEN>(R, it, wave, n_items, partials, lane, k, clk, s_off, launch_idx, rl); break;
        case 6: kstep_tile<6, Q, OPEN>(R, it, wave, n_items, partials, lane, k, clk, s_off, launch_idx, rl); break;
        case 7: kstep_tile<7, Q, OPEN>(R, it, wave, n_items, partials, lane, k, clk, s_off, launch_idx, rl); break;
        case 8: kstep_tile<8, Q, OPEN>(R, it, wave, n_items, partials, lane, k, clk, s_off, launch_idx, rl); break;
        default: break;
    }
}

namespace {
template <int Q>
hipError_t launch_q(uint32_t vmax, bool open, dim3 grid, hipStream_t s, const RingDesc* rings,
                    const TileItem* items, uint32_t n_items, uint32_t* partials, uint32_t k,
                    const Clock* clk, uint32_t s_off, uint32_t launch_idx) {
#define NASCH_KSTEP_CASE(V)                                                                      \
    case V:                                                                                      \
        if (open)                                                                                \
            NASCH_LAUNCH((grid_kstep_kernel<V, Q, true>), grid, dim3(64), 0, s, rings,          \
                         items, n_items, partials, k, clk, s_off, launch_idx);                   \
        else                                                                                     \
            NASCH_LAUNCH((grid_kstep_kernel<V, Q, false>), grid, dim3(64), 0, s, rings,         \
                         items, n_items, partials, k, clk, s_off, launch_idx);                   \
        break;
    switch (vmax) {
        NASCH_KSTEP_CASE(0)
        NASCH_KSTEP_CASE(1)
        NASCH_KSTEP_CASE(2)
        NASCH_KSTEP_CASE(3)
        NASCH_KSTEP_CASE(4)
        NASCH_KSTEP_CASE(5)
        NASCH_KSTEP_CASE(6)
        NASCH_KSTEP_CASE(7)
        NASCH_KSTEP_CASE(8)
        case kMixedVmax:
            if (open)
                NASCH_LAUNCH((grid_kstep_mixed_kernel<Q, true>), grid, dim3(64), 0, s, rings,
                             items, n_items, partials, k, clk, s_off, launch_idx);
            else
                NASCH_LAUNCH((grid_kstep_mixed_kernel<Q, false>), grid, dim3(64), 0, s, rings,
                             items, n_items, partials, k, clk, s_off, launch_idx);
            break;
        default:
            return hipErrorInvalidValue;
    }
#undef NASCH_KSTEP_CASE
    return hipGetLastError();
}
}  // namespace

hipError_t launch_grid_kstep(uint32_t vmax, bool open, uint32_t q, const RingDesc* rings,
                             const TileItem* items, uint32_t n_items, uint32_t* partials,
                             uint32_t k, const Clock* clk, uint32_t s_off, uint32_t launch_idx,
                             hipStream_t s) {
    if (n_items == 0) return hipSuccess;
    const dim3 grid(n_items);
    switch (q) {
        case 1: return launch_q<1>(vmax, open, grid, s, rings, items, n_items, partials, k, clk, s_off, launch_idx);
        case 2: return launch_q<2>(vmax, open, grid, s, rings, items, n_items, partials, k, clk, s_off, launch_idx);
        case 3: return launch_q<3>(vmax, open, grid, s, rings, items, n_items, partials, k, clk, s_off, launch_idx);
        case 4: return launch_q<4>(vmax, open, grid, s, rings, items, n_items, partials, k, clk, s_off, launch_idx);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nasch
