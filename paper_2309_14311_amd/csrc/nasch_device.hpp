// nasch_device.hpp -- device-side building blocks shared by the libnasch kernels:
// Philox4x32-10, the rule-3 draw, the Feistel placement, and the descriptor
// structs the runtime hands to the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nasch {

constexpr uint32_t kEmpty = 0xFFu;
// Counter word 3 of Philox separates the independent streams.
constexpr uint32_t kTagSlowHi = 1u;  // rule 3: top 4 bits of R, one block per 32 cells
constexpr uint32_t kTagSlowLo = 2u;  // rule 3: low 28 bits of R, one block per cell
constexpr uint32_t kTagPlace = 3u;   // initial placement (Feistel round function)
constexpr uint32_t kTagVel0 = 4u;    // initial velocities
constexpr uint32_t kTagGate = 5u;    // open road: entry and exit gates, one block per step

struct Word4 {
    uint32_t w0, w1, w2, w3;
};

// The roads, planes and agent vectors live in device (global) memory, but a
// pointer read out of a descriptor struct is generic to the compiler, which
// then emits flat loads and stores; those also count against the LDS wait
// counter, so every wait for an LDS access would wait for them too.  Accesses
// through gmem() are global ones.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}
// 16-byte vector of the global accesses (a built-in vector type: HIP's uint4
// class has no address-space-qualified copies)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// a ^ b ^ c in one gfx950 three-input bitwise instruction (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two 32x32->64
// multiplies by the Philox constants, key bumped by the Weyl constants between
// rounds.  With a wave-uniform key and counter words 1-3 uniform, the compiler
// keeps the key schedule and the first multiply of round 0 in scalar registers.
__device__ __forceinline__ Word4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        // With counter words 1-3 uniform (every call site), some operands of
        // rounds 0-2 are uniform too; grouping those with plain XORs lets the
        // scalar unit combine them, where a three-input vector XOR would need
        // a move for its second scalar operand: round 0's n0 is uniform
        // outright; in round 1, c1 (a product of uniform words) and hi(m0)
        // (c0 is round 0's uniform n0) are; in round 2, c3 is (round 1's
        // lo(m0)).
        const uint32_t h0 = (uint32_t)(m0 >> 32), h1 = (uint32_t)(m1 >> 32);
        const uint32_t n0 = r == 0 ? (h1 ^ c1) ^ k0
                          : r == 1 ? h1 ^ (c1 ^ k0)
                                   : xor3(h1, c1, k0);
        const uint32_t n2 = r == 1 ? (h0 ^ k1) ^ c3
                          : r == 2 ? h0 ^ (c3 ^ k1)
                                   : xor3(h0, c3, k1);
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Word4{c0, c1, c2, c3};
}

// Per-simulation constants of rule 3.
struct SlowParams {
    uint32_t k0, k1;     // Philox key: seed low / high word
    uint32_t replica;    // counter word 2
    uint32_t thr;        // floor(p * 2^32); 0 disables rule 3 draws entirely
};

// The four top-bit planes of R for the aligned block of 32 cells [32*blk, 32*blk+32):
// bit j of word i is bit (31 - i) of R for cell 32*blk + j.
__device__ __forceinline__ Word4 slow_hi_planes(uint32_t blk, uint32_t t, const SlowParams& sp) {
    return philox(blk, t, sp.replica, kTagSlowHi, sp.k0, sp.k1);
}

// Low 28 bits of R for cell x.
__device__ __forceinline__ uint32_t slow_lo28(uint32_t x, uint32_t t, const SlowParams& sp) {
    return philox(x, t, sp.replica, kTagSlowLo, sp.k0, sp.k1).w0 >> 4;
}

// The bit-sliced nibble (w0 w1 w2 w3), w0 most significant, compared with the
// constant TH: lt = nibble < TH, eq = nibble == TH.  With TH known the chain
// folds into a few three-input bitwise operations.
template <int TH>
__device__ __forceinline__ void nibble_cmp(const Word4& w, uint32_t& lt, uint32_t& eq) {
    const uint32_t P[4] = {w.w0, w.w1, w.w2, w.w3};
    uint32_t l = 0u, e = 0xFFFFFFFFu;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if ((TH >> (3 - b)) & 1) {
            l |= e & ~P[b];
            e &= P[b];
        } else {
            e &= ~P[b];
        }
    }
    lt = l;
    eq = e;
}

// The same comparison of one block with thr's top nibble `th` (uniform over
// the wave): lt = cars whose nibble is below th, eq = cars whose nibble ties.
__device__ __forceinline__ void block_lt_eq(const Word4& w, uint32_t th, uint32_t& lt,
                                            uint32_t& eq) {
    switch (th) {
        case 0: nibble_cmp<0>(w, lt, eq); break;
        case 1: nibble_cmp<1>(w, lt, eq); break;
        case 2: nibble_cmp<2>(w, lt, eq); break;
        case 3: nibble_cmp<3>(w, lt, eq); break;
        case 4: nibble_cmp<4>(w, lt, eq); break;
        case 5: nibble_cmp<5>(w, lt, eq); break;
        case 6: nibble_cmp<6>(w, lt, eq); break;
        case 7: nibble_cmp<7>(w, lt, eq); break;
        case 8: nibble_cmp<8>(w, lt, eq); break;
        case 9: nibble_cmp<9>(w, lt, eq); break;
        case 10: nibble_cmp<10>(w, lt, eq); break;
        case 11: nibble_cmp<11>(w, lt, eq); break;
        case 12: nibble_cmp<12>(w, lt, eq); break;
        case 13: nibble_cmp<13>(w, lt, eq); break;
        case 14: nibble_cmp<14>(w, lt, eq); break;
        default: nibble_cmp<15>(w, lt, eq); break;
    }
}


// Open road: the gate draw of step t.  A car enters empty cell 0 iff word 0 is
// below thr_in = floor(alpha 2^32); the exit is open iff word 1 is below
// thr_out = floor(beta 2^32) (both thresholds in [0, 2^32]).
__device__ __forceinline__ void gate_draw(uint32_t t, const SlowParams& sp, uint64_t thr_in,
                                          uint64_t thr_out, bool& enter, bool& exit_open) {
    const Word4 g = philox(0u, t, sp.replica, kTagGate, sp.k0, sp.k1);
    enter = (uint64_t)g.w0 < thr_in;
    exit_open = (uint64_t)g.w1 < thr_out;
}

// ---- initial placement --------------------------------------------------------
// b = ceil(log2 L) rounded up to even, at least 2.
__host__ __device__ inline uint32_t feistel_bits(uint64_t L) {
    uint32_t b = 0;
    while ((1ull << b) < L) ++b;
    b += b & 1u;
    return b < 2 ? 2 : b;
}

// Round function j of the placement permutation: F_j(r), r < 2^half.
__device__ __forceinline__ uint32_t feistel_round(uint32_t r, uint32_t j, uint32_t mask,
                                                  const SlowParams& sp) {
    return philox(r, j, sp.replica, kTagPlace, sp.k0, sp.k1).w0 & mask;
}

// Inverse of the 4-round Feistel permutation on b bits: forward round j maps
// (l, r) to (r, l ^ F_j(r)); undo rounds 3..0.
__device__ __forceinline__ uint32_t feistel_inv(uint32_t y, uint32_t half, uint32_t mask,
                                                const SlowParams& sp) {
    uint32_t l = (y >> half) & mask, r = y & mask;
#pragma unroll
    for (int j = 3; j >= 0; --j) {
        const uint32_t f = feistel_round(l, (uint32_t)j, mask, sp);
        const uint32_t pr = l;
        l = r ^ f;
        r = pr;
    }
    return (l << half) | r;
}

// Forward 4-round Feistel permutation on b bits: round j maps (l, r) to
// (r, l ^ F_j(r)), with F_j(r) = round(r, j) (feistel_round, or a table of its
// values: a round sees only 2^half inputs).
template <class Round>
__device__ __forceinline__ uint32_t feistel_fwd_by(uint32_t i, uint32_t half, uint32_t mask,
                                                   const Round& round) {
    uint32_t l = (i >> half) & mask, r = i & mask;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t f = round(r, (uint32_t)j);
        const uint32_t nl = r;
        r = l ^ f;
        l = nl;
    }
    return (l << half) | r;
}

struct PhiloxRound {
    SlowParams sp;
    uint32_t mask;
    __device__ uint32_t operator()(uint32_t r, uint32_t j) const {
        return feistel_round(r, j, mask, sp);
    }
};

__device__ __forceinline__ uint32_t feistel_fwd(uint32_t i, uint32_t half, uint32_t mask,
                                                const SlowParams& sp) {
    return feistel_fwd_by(i, half, mask, PhiloxRound{sp, mask});
}

// Cell of car i: the Feistel permutation cycle-walked until it lands in [0, L).
__device__ __forceinline__ uint32_t placement(uint32_t i, uint32_t L, uint32_t b,
                                              const SlowParams& sp) {
    const uint32_t half = b >> 1;
    const uint32_t mask = (half >= 32) ? 0xFFFFFFFFu : ((1u << half) - 1u);
    uint32_t y = feistel_fwd(i, half, mask, sp);
    while (y >= L) y = feistel_fwd(y, half, mask, sp);
    return y;
}

// Index of the car that starts in cell y (cycle-walking the inverse until it
// lands in [0, L)); the cell is occupied iff the index is below N.
__device__ __forceinline__ uint32_t placement_preimage(uint32_t y, uint32_t L, uint32_t b,
                                                       const SlowParams& sp) {
    const uint32_t half = b >> 1;
    const uint32_t mask = (half >= 32) ? 0xFFFFFFFFu : ((1u << half) - 1u);
    uint32_t z = feistel_inv(y, half, mask, sp);
    while (z >= L) z = feistel_inv(z, half, mask, sp);
    return z;
}

__device__ __forceinline__ uint32_t initial_velocity(uint32_t x, uint32_t vmax, const SlowParams& sp) {
    const uint32_t w = philox(x, 0u, sp.replica, kTagVel0, sp.k0, sp.k1).w0;
    return (uint32_t)(((uint64_t)w * (uint64_t)(vmax + 1u)) >> 32);
}

// ---- descriptors --------------------------------------------------------------
// One ring as the grid kernels see it.  Tiles own `own` cells each (the last
// one the remainder); a tile's segment is its owned cells plus `halo` cells on
// each side, read modulo L.  With `open` set the road is not a ring: cells
// outside [0, L) are empty, a car enters cell 0 and the exit at cell L opens
// by the gate draw of each step (see gate_draw).
//
// The road is kept in one of two forms: bytes (buf, one per cell: 0xFF or v),
// read by the one-step kernel, the snapshots and the initial placement; or bit
// planes (pl), read and written by the temporal-blocked kernel.  Plane m
// (m = 0..vmax) holds nw = ceil(L / 32) words at pl[b] + m * nw: plane 0 is the
// occupancy (bit i of word w for cell 32 w + i), plane m >= 1 the cars with
// v >= m.  Bits past cell L-1 are zero.
struct RingDesc {
    uint8_t* buf[2];         // ping-pong grids, L bytes each
    uint32_t* pl[2];         // ping-pong bit planes, (vmax + 1) * nw words each
    unsigned long long* flux_log;  // F(t) at flux_log[t - log_t0] (may be null)
    unsigned long long* flux_acc;  // += F(t) for t >= warmup (may be null)
    uint64_t log_t0;
    uint64_t warmup;
    uint32_t t;              // step of the state in buf[parity] when the launch sequence starts
    uint32_t parity;
    uint32_t L, vmax;
    uint32_t own, halo;      // geometry for the current (k, q)
    uint32_t ntiles;
    uint32_t t_end;          // no step t >= t_end is run (serving); 0xFFFFFFFF = none
    uint32_t first_item;     // index of the ring's first item in the launch
    uint32_t open;           // 1: open road (entry at cell 0, exit after cell L-1)
    uint32_t nw;             // words per bit plane, ceil(L / 32)
    uint32_t pad;
    SlowParams sp;
    uint64_t thr_in, thr_out;  // open road: gate thresholds floor(alpha 2^32), floor(beta 2^32)
};

// One conversion between the byte and bit-plane forms of a road (see
// RingDesc); ConvChunk names kConvChunk consecutive words of one job.
struct ConvJob {
    uint8_t* bytes;
    uint32_t* planes;
    uint32_t L, nw, vmax, pad;
};
struct ConvChunk {
    uint32_t job;
    uint32_t first;
};
constexpr uint32_t kConvChunk = 256;

// Words of the bit planes of a road of L cells.
__host__ __device__ inline uint32_t plane_words(uint64_t L) { return (uint32_t)((L + 31) / 32); }

// Initial placement of one ring: cars [0, N) scattered into g (already EMPTY).
struct InitRing {
    uint8_t* g;
    uint32_t L, N, vmax, init_v;
    uint32_t b;              // Feistel width
    uint32_t pad;
    SlowParams sp;
    uint32_t* tab;           // the placement's round-function table (init_tab_words(b)
                             // words, filled by launch_init_tables), or null: computed
};
// Words of a ring's placement table: 4 rounds x 2^(b/2) inputs.
__host__ __device__ inline uint64_t init_tab_words(uint32_t b) { return 4ull << (b >> 1); }
// kInitChunk consecutive cars of one ring.
struct InitChunk {
    uint32_t ring;
    uint32_t first;
};
constexpr uint32_t kInitChunk = 4096;

struct TileItem {
    uint32_t ring;   // index into the RingDesc table
    uint32_t tile;   // tile index within the ring
};

// Step counter and buffer parity shared by every ring of a launch sequence.  It
// lives in device memory so that a captured launch sequence can be replayed:
// launch i of a sequence runs steps clock.t + ring.t + s_off ... and reads
// buf[(clock.parity + ring.parity + i) & 1].  A one-thread kernel advances it
// after the sequence.
struct Clock {
    uint32_t t;
    uint32_t parity;
};

// ---- the shared-stream generator ------------------------------------------------
// minstd_rand: x <- 48271 x mod (2^31 - 1).  Car i at step t takes output number
// t N + i + 1 of one stream, x_n = a^n x_0 mod m.
constexpr uint32_t kMlcgA = 48271u;
constexpr uint32_t kMlcgM = 0x7FFFFFFFu;

// a * b mod (2^31 - 1) for a, b < 2^31, by folding (2^31 = 1 mod m).
__host__ __device__ inline uint32_t mlcg_mul(uint32_t a, uint32_t b) {
    const uint64_t z = (uint64_t)a * b;
    uint32_t r = (uint32_t)(z & kMlcgM) + (uint32_t)(z >> 31);
    r = (r & kMlcgM) + (r >> 31);
    return r >= kMlcgM ? r - kMlcgM : r;
}

// a^n mod m from pow_tab[16 j + d] = a^(d 16^j) mod m.
__device__ __forceinline__ uint32_t mlcg_pow(const uint32_t* __restrict__ pow_tab, uint64_t n) {
    uint32_t r = 1u;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t d = (uint32_t)(n >> (4 * j)) & 15u;
        if (d) r = mlcg_mul(r, pow_tab[16 * j + d]);
    }
    return r;
}

// One ring in the agent representation.
struct AgentDesc {
    int32_t* x[2];           // ping-pong positions, road order
    uint8_t* v[2];           // ping-pong velocities
    unsigned long long* flux_log;
    unsigned long long* flux_acc;
    uint64_t log_t0;
    uint64_t warmup;
    uint32_t t, parity;
    uint32_t N, L, vmax;
    uint32_t rng;            // 0: keyed Philox draw; 1: shared minstd stream
    SlowParams sp;
    // shared stream (rng == 1)
    const uint32_t* mlcg_pow;   // 256-entry jump table
    uint32_t mlcg_x0;           // stream state before the first draw
    uint32_t mlcg_thr;          // slow iff x < ceil(p m)
    uint32_t mlcg_aN;           // a^N mod m: one step of every car
    uint32_t mlcg_inv_aN;       // its inverse mod m
};

// ---- cross-lane helpers (gfx9 DPP) ----------------------------------------------
// Lane i receives lane i+1's value; lane 63 receives 0 (bound_ctrl writes 0
// where the source lane does not exist, so no old value has to be set up).
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}
// Lane i receives lane i-1's value; lane 0 receives 0.
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}
// Inclusive prefix sum over the lanes of a wave (all lanes active): DPP row
// shifts 1, 2, 4, 8 scan each row of 16 lanes, then the row broadcasts of
// lanes 15 and 31 carry the row totals into the rows above.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111 /* row_shr:1 */, 0xf, 0xf, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112 /* row_shr:2 */, 0xf, 0xf, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114 /* row_shr:4 */, 0xf, 0xf, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118 /* row_shr:8 */, 0xf, 0xf, true);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142 /* row_bcast:15 */, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143 /* row_bcast:31 */, 0xc, 0xf, false);
    return v;
}

// Maximum over the 64 lanes of a wave (all lanes active), returned to every lane.
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111 /* row_shr:1 */, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112 /* row_shr:2 */, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114 /* row_shr:4 */, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118 /* row_shr:8 */, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142 /* row_bcast:15 */, 0xa, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143 /* row_bcast:31 */, 0xc, 0xf, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Sum over the 64 lanes of a wave (all lanes active), returned to every lane:
// an inclusive DPP scan (row shifts 1, 2, 4, 8, then the row broadcasts of
// lanes 15 and 31) leaves the total in lane 63.
__device__ __forceinline__ uint32_t wave_total(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111 /* row_shr:1 */, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112 /* row_shr:2 */, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114 /* row_shr:4 */, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118 /* row_shr:8 */, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142 /* row_bcast:15 */, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143 /* row_bcast:31 */, 0xc, 0xf, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

}  // namespace nasch
