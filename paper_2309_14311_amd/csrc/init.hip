// init.hip -- initial state, representation changes and small utility kernels.
#include "bitplanes.hpp"
#include "launchers.hpp"

namespace nasch {

// Initial grid of one ring: EMPTY everywhere, then car i < N at its placement.
// Scatter form: each car's Feistel value is cycle-walked until it lands in
// [0, L).  A car needs two walks on average but up to about seven in a wave of
// 64, so a lane whose car has landed takes the next car of the wave's range
// instead of idling: the wave's work is the sum of the walks, not 64 times
// their maximum.
//
// A Feistel round sees only 2^(b/2) inputs, so when the ring has a table of
// its round functions (InitRing::tab, filled by init_table_kernel) a walk is
// four table reads instead of four Philox calls: the block copies a table of
// at most kInitLdsTab words into LDS, a larger one is read from global memory
// (L2).  Without a table the rounds are computed.
constexpr uint32_t kInitLdsTab = 4096;   // 4 rounds x 1024 inputs: b <= 20, L <= 2^20

// Table reads of the round function (an LDS or a global table).
struct LdsRound {
    const uint32_t* t;
    uint32_t half;
    __device__ uint32_t operator()(uint32_t r, uint32_t j) const { return t[(j << half) | r]; }
};
struct GlobalRound {
    const uint32_t* t;
    uint32_t half;
    __device__ uint32_t operator()(uint32_t r, uint32_t j) const {
        return *gmem(t + ((j << half) | r));
    }
};

template <class Round>
__device__ __forceinline__ void scatter_range(const InitRing& R, uint32_t begin, uint32_t end,
                                              uint32_t lane, uint32_t half, uint32_t mask,
                                              const Round& round) {
    uint32_t y = begin + lane;      // the lane's car, then its walk
    bool active = y < end;
    uint32_t next = begin + 64u;    // first car not yet taken (uniform)
    while (__builtin_amdgcn_ballot_w64(active) != 0u) {
        y = feistel_fwd_by(y, half, mask, round);
        const bool done = active && y < R.L;
        if (done) R.g[y] = (uint8_t)(R.init_v ? initial_velocity(y, R.vmax, R.sp) : 0u);
        const bool take = done || !active;
        const uint64_t m = __builtin_amdgcn_ballot_w64(take);
        const uint32_t rank =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (take) {
            y = next + rank;
            active = y < end;
        }
        next += (uint32_t)__popcll(m);
    }
}

__global__ __launch_bounds__(256) void init_scatter_kernel(const InitRing* __restrict__ rings,
                                                           const InitChunk* __restrict__ chunks,
                                                           InitRing single) {
    __shared__ uint32_t s_tab[kInitLdsTab];
    const InitChunk c = chunks ? chunks[blockIdx.x] : InitChunk{0u, blockIdx.x * kInitChunk};
    const InitRing R = chunks ? rings[c.ring] : single;
    const uint32_t half = R.b >> 1;
    const uint32_t mask = (half >= 32) ? 0xFFFFFFFFu : ((1u << half) - 1u);
    const uint64_t ntab = init_tab_words(R.b);
    const bool lds_tab = R.tab && ntab <= kInitLdsTab;   // uniform over the block
    if (lds_tab) {
        for (uint32_t e = threadIdx.x; e < (uint32_t)ntab; e += 256u) s_tab[e] = *gmem(R.tab + e);
        __syncthreads();
    }
    constexpr uint32_t kPerWave = kInitChunk / 4;   // 256 threads: four waves
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t begin =
        c.first + kPerWave * (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t end = min(begin + kPerWave, R.N);
    if (begin >= end) return;   // uniform over the wave
    if (lds_tab) scatter_range(R, begin, end, lane, half, mask, LdsRound{s_tab, half});
    else if (R.tab) scatter_range(R, begin, end, lane, half, mask, GlobalRound{R.tab, half});
    else scatter_range(R, begin, end, lane, half, mask, PhiloxRound{R.sp, mask});
}

// Round-function tables: entry e = j 2^half + r of a ring's table is F_j(r).
__global__ __launch_bounds__(256) void init_table_kernel(const InitRing* __restrict__ rings,
                                                         const InitChunk* __restrict__ chunks,
                                                         InitRing single) {
    const InitChunk c = chunks ? chunks[blockIdx.x] : InitChunk{0u, blockIdx.x * 256u};
    const InitRing R = chunks ? rings[c.ring] : single;
    const uint32_t half = R.b >> 1;
    const uint32_t mask = (half >= 32) ? 0xFFFFFFFFu : ((1u << half) - 1u);
    const uint32_t e = c.first + threadIdx.x;
    if (!R.tab || (uint64_t)e >= init_tab_words(R.b)) return;
    *gmem(R.tab + e) = feistel_round(e & mask, e >> half, mask, R.sp);
}

hipError_t launch_init_scatter(const InitRing* rings, const InitChunk* chunks, uint32_t n_chunks,
                               hipStream_t s) {
    if (n_chunks == 0) return hipSuccess;
    NASCH_LAUNCH(init_scatter_kernel, dim3(n_chunks), dim3(256), 0, s, rings, chunks, InitRing{});
    return hipGetLastError();
}

hipError_t launch_init_tables(const InitRing* rings, const InitChunk* chunks, uint32_t n_chunks,
                              hipStream_t s) {
    if (n_chunks == 0) return hipSuccess;
    NASCH_LAUNCH(init_table_kernel, dim3(n_chunks), dim3(256), 0, s, rings, chunks, InitRing{});
    return hipGetLastError();
}

hipError_t launch_init_grid(uint8_t* g, uint32_t L, uint32_t N, uint32_t vmax, uint32_t init_v,
                            SlowParams sp, hipStream_t s, uint32_t* tab) {
    hipError_t e = launch_fill_u8(g, L, (uint8_t)kEmpty, s);
    if (e != hipSuccess || N == 0) return e;
    InitRing r{g, L, N, vmax, init_v, feistel_bits(L), 0u, sp, tab};
    if (tab) {
        const uint64_t n = init_tab_words(r.b);
        NASCH_LAUNCH(init_table_kernel, dim3((uint32_t)((n + 255u) / 256u)), dim3(256), 0, s,
                     nullptr, nullptr, r);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const uint32_t chunks = (N + kInitChunk - 1) / kInitChunk;
    NASCH_LAUNCH(init_scatter_kernel, dim3(chunks), dim3(256), 0, s, nullptr, nullptr, r);
    return hipGetLastError();
}

// ---- bytes <-> bit planes ------------------------------------------------------
// One thread per 32-cell word, a block per kConvChunk words of one job.
// The bytes of a word and their code planes are exchanged with the transposes
// of bitplanes.hpp; vmax is a run-time value here.
namespace {
// (P3 P2 P1 P0) >= m, bit-sliced over 32 cells, for 1 <= m <= 15
__device__ __forceinline__ uint32_t ge_value(const uint32_t (&P)[4], uint32_t m) {
    uint32_t gt = 0u, eq = 0xFFFFFFFFu;
    for (int b = 3; b >= 0; --b) {
        if ((m >> b) & 1u) {
            eq &= P[b];
        } else {
            gt |= eq & P[b];
            eq &= ~P[b];
        }
    }
    return gt | eq;
}
__device__ __forceinline__ bool conv_job(const ConvJob* jobs, const ConvChunk* chunks,
                                         const ConvJob& single, ConvJob& J, uint32_t& w) {
    const ConvChunk c = chunks ? chunks[blockIdx.x] : ConvChunk{0u, blockIdx.x * kConvChunk};
    J = chunks ? jobs[c.job] : single;
    w = c.first + threadIdx.x;
    return w < J.nw;
}
}  // namespace

__global__ __launch_bounds__(kConvChunk) void bytes_to_planes_kernel(const ConvJob* jobs,
                                                                     const ConvChunk* chunks,
                                                                     ConvJob single) {
    ConvJob J;
    uint32_t w;
    if (!conv_job(jobs, chunks, single, J, w)) return;
    const uint64_t c0 = (uint64_t)w * 32u;
    uint32_t by[8];
    if (c0 + 32u <= J.L) {   // J.bytes is 16-byte aligned (every caller's buffers are)
        const uint4* p = reinterpret_cast<const uint4*>(J.bytes + c0);
        const uint4 a = p[0], b = p[1];
        by[0] = a.x; by[1] = a.y; by[2] = a.z; by[3] = a.w;
        by[4] = b.x; by[5] = b.y; by[6] = b.z; by[7] = b.w;
    } else {
        for (int d = 0; d < 8; ++d) {
            uint32_t y = 0;
            for (int e = 0; e < 4; ++e) {
                const uint64_t c = c0 + 4u * d + e;
                const uint32_t val = c < J.L ? J.bytes[c] : kEmpty;   // past the road: empty
                y |= val << (8 * e);
            }
            by[d] = y;
        }
    }
    uint32_t P[4];   // v, bit by bit (code 15 where empty)
    bytes_to_code_planes(by, P);
    const uint32_t occ = code_occupied(P);
    J.planes[w] = occ;
    for (uint32_t m = 1; m <= J.vmax; ++m) J.planes[(uint64_t)m * J.nw + w] = occ & ge_value(P, m);
}

__global__ __launch_bounds__(kConvChunk) void planes_to_bytes_kernel(const ConvJob* jobs,
                                                                     const ConvChunk* chunks,
                                                                     ConvJob single) {
    ConvJob J;
    uint32_t w;
    if (!conv_job(jobs, chunks, single, J, w)) return;
    uint32_t T[9];
    for (uint32_t m = 0; m <= 8; ++m) T[m] = m <= J.vmax ? J.planes[(uint64_t)m * J.nw + w] : 0u;
    // thermometer (T[m]: v >= m) -> binary digits of v
    uint32_t B0 = 0u;
    for (uint32_t m = 1; m <= 8; ++m) B0 ^= T[m];
    const uint32_t B1 = (T[2] & ~T[4]) | (T[6] & ~T[8]);
    const uint32_t B2 = T[4] & ~T[8];
    const uint32_t B3 = T[8];
    const uint32_t E = ~T[0];
    // an empty cell gets code 15, which becomes 0xFF
    const uint32_t N[4] = {B0 | E, B1 | E, B2 | E, B3 | E};
    uint32_t by[8];
    code_planes_to_bytes(N, by);
    const uint64_t c0 = (uint64_t)w * 32u;
    if (c0 + 32u <= J.L) {
        uint4* p = reinterpret_cast<uint4*>(J.bytes + c0);
        p[0] = make_uint4(by[0], by[1], by[2], by[3]);
        p[1] = make_uint4(by[4], by[5], by[6], by[7]);
    } else {
        for (uint32_t i = 0; i < 32u && c0 + i < J.L; ++i)
            J.bytes[c0 + i] = (uint8_t)(by[i >> 2] >> (8 * (i & 3)));
    }
}

hipError_t launch_bytes_to_planes(const ConvJob* jobs, const ConvChunk* chunks, uint32_t n_chunks,
                                  hipStream_t s) {
    if (n_chunks == 0) return hipSuccess;
    NASCH_LAUNCH(bytes_to_planes_kernel, dim3(n_chunks), dim3(kConvChunk), 0, s, jobs, chunks,
                 ConvJob{});
    return hipGetLastError();
}

hipError_t launch_planes_to_bytes(const ConvJob* jobs, const ConvChunk* chunks, uint32_t n_chunks,
                                  hipStream_t s) {
    if (n_chunks == 0) return hipSuccess;
    NASCH_LAUNCH(planes_to_bytes_kernel, dim3(n_chunks), dim3(kConvChunk), 0, s, jobs, chunks,
                 ConvJob{});
    return hipGetLastError();
}

hipError_t launch_bytes_to_planes_one(const ConvJob& job, hipStream_t s) {
    const uint32_t blocks = (job.nw + kConvChunk - 1) / kConvChunk;
    if (blocks == 0) return hipSuccess;
    NASCH_LAUNCH(bytes_to_planes_kernel, dim3(blocks), dim3(kConvChunk), 0, s, nullptr, nullptr,
                 job);
    return hipGetLastError();
}

hipError_t launch_planes_to_bytes_one(const ConvJob& job, hipStream_t s) {
    const uint32_t blocks = (job.nw + kConvChunk - 1) / kConvChunk;
    if (blocks == 0) return hipSuccess;
    NASCH_LAUNCH(planes_to_bytes_kernel, dim3(blocks), dim3(kConvChunk), 0, s, nullptr, nullptr,
                 job);
    return hipGetLastError();
}

// ---- grid -> agent compaction ---------------------------------------------------
// One workgroup of 256 threads per chunk; thread i scans a contiguous run of
// kCompactChunk / 256 cells so that the writes come out in ascending order.
constexpr uint32_t kRun = kCompactChunk / 256;

__global__ __launch_bounds__(256) void count_chunks_kernel(const uint8_t* __restrict__ g,
                                                           uint32_t L,
                                                           uint32_t* __restrict__ counts) {
    __shared__ uint32_t partial[256];
    const uint64_t begin = (uint64_t)blockIdx.x * kCompactChunk + (uint64_t)threadIdx.x * kRun;
    uint32_t c = 0;
    for (uint32_t i = 0; i < kRun; ++i) {
        const uint64_t y = begin + i;
        if (y < L && g[y] != kEmpty) ++c;
    }
    partial[threadIdx.x] = c;
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) partial[threadIdx.x] += partial[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = partial[0];
}

__global__ __launch_bounds__(256) void compact_chunks_kernel(const uint8_t* __restrict__ g,
                                                             uint32_t L,
                                                             const uint32_t* __restrict__ offsets,
                                                             int32_t* __restrict__ x,
                                                             uint8_t* __restrict__ v) {
    __shared__ uint32_t scan[256];
    const uint64_t begin = (uint64_t)blockIdx.x * kCompactChunk + (uint64_t)threadIdx.x * kRun;
    uint32_t c = 0;
    for (uint32_t i = 0; i < kRun; ++i) {
        const uint64_t y = begin + i;
        if (y < L && g[y] != kEmpty) ++c;
    }
    scan[threadIdx.x] = c;
    __syncthreads();
    // inclusive Hillis-Steele scan over the 256 thread counts
    for (uint32_t off = 1; off < 256; off <<= 1) {
        const uint32_t add = threadIdx.x >= off ? scan[threadIdx.x - off] : 0u;
        __syncthreads();
        scan[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t out = offsets[blockIdx.x] + scan[threadIdx.x] - c;
    for (uint32_t i = 0; i < kRun; ++i) {
        const uint64_t y = begin + i;
        if (y < L) {
            const uint8_t cell = g[y];
            if (cell != kEmpty) {
                x[out] = (int32_t)y;
                v[out] = cell;
                ++out;
            }
        }
    }
}

hipError_t launch_count_chunks(const uint8_t* g, uint32_t L, uint32_t* counts, hipStream_t s) {
    const uint32_t chunks = (uint32_t)(((uint64_t)L + kCompactChunk - 1) / kCompactChunk);
    NASCH_LAUNCH(count_chunks_kernel, dim3(chunks), dim3(256), 0, s, g, L, counts);
    return hipGetLastError();
}

hipError_t launch_compact_chunks(const uint8_t* g, uint32_t L, const uint32_t* offsets,
                                 int32_t* x, uint8_t* v, hipStream_t s) {
    const uint32_t chunks = (uint32_t)(((uint64_t)L + kCompactChunk - 1) / kCompactChunk);
    NASCH_LAUNCH(compact_chunks_kernel, dim3(chunks), dim3(256), 0, s, g, L, offsets, x, v);
    return hipGetLastError();
}

// ---- agent -> grid ----------------------------------------------------------------
__global__ __launch_bounds__(256) void fill_u8_kernel(uint8_t* __restrict__ p, uint64_t n,
                                                      uint8_t value) {
    const uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16u;
    if (i + 16 <= n) {
        const uint32_t w = 0x01010101u * value;
        *reinterpret_cast<uint4*>(p + i) = make_uint4(w, w, w, w);
    } else {
        for (uint64_t j = i; j < n; ++j) p[j] = value;
    }
}

hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t value, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint64_t threads = (n + 15) / 16;
    NASCH_LAUNCH(fill_u8_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s,
                       p, n, value);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_u64_kernel(unsigned long long* __restrict__ p,
                                                       uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    NASCH_LAUNCH(fill_u64_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void scatter_agents_kernel(const int32_t* __restrict__ x,
                                                             const uint8_t* __restrict__ v,
                                                             uint32_t N, uint8_t* __restrict__ g,
                                                             uint32_t L) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        const uint32_t pos = (uint32_t)x[i];
        if (pos < L) g[pos] = v[i];
    }
}

hipError_t launch_agent_to_grid(const int32_t* x, const uint8_t* v, uint32_t N, uint8_t* g,
                                uint32_t L, hipStream_t s) {
    hipError_t e = launch_fill_u8(g, L, (uint8_t)kEmpty, s);
    if (e != hipSuccess || N == 0) return e;
    NASCH_LAUNCH(scatter_agents_kernel, dim3((N + 255) / 256), dim3(256), 0, s, x, v, N, g,
                       L);
    return hipGetLastError();
}

// ---- flux folding -------------------------------------------------------------
// The kernels leave F(t) per item and step in partials[s * n_items + item]; the
// fold adds them up.  Block (r, s, c) sums chunk c (kFoldChunk items) of ring
// log_rings[r] for step s and adds it to the ring's (zero-initialised) log
// entry: a handful of atomics per step instead of one per item.  Chunks of
// 1024 items (4 per thread) keep a step's fold short: with 4096 it took 9 us of
// the agent one-step's 127 us on the 2^28 ring.
constexpr uint32_t kFoldChunk = 1024;

__device__ __forceinline__ unsigned long long block_sum(const uint32_t* p, uint32_t n) {
    __shared__ unsigned long long part[4];
    unsigned long long v = 0;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
    // 64-bit wave sum from two 32-bit wave totals of the halves of v
    const uint32_t lo = wave_total((uint32_t)(v & 0xFFFFFFFFull));
    const uint32_t hi = wave_total((uint32_t)(v >> 32));
    const unsigned long long w = ((unsigned long long)hi << 32) + lo;
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = w;
    __syncthreads();
    unsigned long long total = 0;
    if (threadIdx.x == 0)
        for (uint32_t i = 0; i < blockDim.x / 64; ++i) total += part[i];
    return total;
}

__global__ __launch_bounds__(256) void fold_ring_flux_kernel(const RingDesc* __restrict__ rings,
                                                             const uint32_t* __restrict__ log_rings,
                                                             const uint32_t* __restrict__ partials,
                                                             uint32_t n_items, uint32_t k,
                                                             const Clock* __restrict__ clk,
                                                             uint32_t s_off) {
    const RingDesc& R = rings[log_rings[blockIdx.x]];
    const uint32_t s = blockIdx.y;
    const uint32_t first = blockIdx.z * kFoldChunk;
    const uint32_t t = clk->t + R.t + s_off + s;
    if (s >= k || first >= R.ntiles || (R.t_end != 0xFFFFFFFFu && t >= R.t_end)) return;
    const uint32_t n = min(kFoldChunk, R.ntiles - first);
    const unsigned long long total =
        block_sum(partials + (size_t)s * n_items + R.first_item + first, n);
    if (threadIdx.x == 0 && total) atomicAdd(&R.flux_log[(uint64_t)t - R.log_t0], total);
}

hipError_t launch_fold_ring_flux(const RingDesc* rings, const uint32_t* log_rings, uint32_t n_log,
                                 uint32_t max_tiles, const uint32_t* partials, uint32_t n_items,
                                 uint32_t k, const Clock* clk, uint32_t s_off, hipStream_t s) {
    if (n_log == 0 || k == 0 || max_tiles == 0) return hipSuccess;
    const uint32_t chunks = (max_tiles + kFoldChunk - 1) / kFoldChunk;
    NASCH_LAUNCH(fold_ring_flux_kernel, dim3(n_log, k, chunks), dim3(256), 0, s, rings, log_rings,
                 partials, n_items, k, clk, s_off);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void fold_agent_flux_kernel(const AgentDesc* __restrict__ A,
                                                              const uint32_t* __restrict__ partials,
                                                              uint32_t n_items, uint32_t k,
                                                              const Clock* __restrict__ clk,
                                                              uint32_t s_off) {
    const uint32_t s = blockIdx.x;
    const uint32_t first = blockIdx.y * kFoldChunk;
    const uint32_t t = clk->t + A->t + s_off + s;
    const uint32_t n = min(kFoldChunk, n_items - first);
    const unsigned long long total = block_sum(partials + (size_t)s * n_items + first, n);
    if (threadIdx.x == 0 && A->flux_log && total)
        atomicAdd(&A->flux_log[(uint64_t)t - A->log_t0], total);
}

hipError_t launch_fold_agent_flux(const AgentDesc* a, const uint32_t* partials, uint32_t n_items,
                                  uint32_t k, const Clock* clk, uint32_t s_off, hipStream_t s) {
    if (k == 0 || n_items == 0) return hipSuccess;
    const uint32_t chunks = (n_items + kFoldChunk - 1) / kFoldChunk;
    NASCH_LAUNCH(fold_agent_flux_kernel, dim3(k, chunks), dim3(256), 0, s, a, partials, n_items, k,
                 clk, s_off);
    return hipGetLastError();
}

__global__ void clock_advance_kernel(Clock* clk, uint32_t T, uint32_t nlaunch) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        clk->t += T;
        clk->parity ^= (nlaunch & 1u);
    }
}

hipError_t launch_clock_advance(Clock* clk, uint32_t T, uint32_t nlaunch, hipStream_t s) {
    NASCH_LAUNCH(clock_advance_kernel, dim3(1), dim3(64), 0, s, clk, T, nlaunch);
    return hipGetLastError();
}

}  // namespace nasch
