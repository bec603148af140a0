// init.hip -- initial state, representation changes and small utility kernels.
#include "launchers.hpp"

namespace nasch {

// One thread per 4 cells; a cell holds a car iff the cycle-walked inverse
// Feistel permutation maps it below N.
__global__ __launch_bounds__(256) void init_grid_kernel(uint8_t* __restrict__ g, uint32_t L,
                                                        uint32_t N, uint32_t vmax,
                                                        uint32_t init_v, SlowParams sp,
                                                        uint32_t b) {
    const uint64_t base = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4u;
    if (base >= L) return;
    uint32_t word = 0;
    const uint32_t n = (uint32_t)min((uint64_t)4, (uint64_t)L - base);
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t y = (uint32_t)base + i;
        uint32_t cell = kEmpty;
        if (N > 0 && placement_preimage(y, L, b, sp) < N)
            cell = init_v ? initial_velocity(y, vmax, sp) : 0u;
        word |= cell << (8 * i);
    }
    if (n == 4) {
        *reinterpret_cast<uint32_t*>(g + base) = word;
    } else {
        for (uint32_t i = 0; i < n; ++i) g[base + i] = (uint8_t)(word >> (8 * i));
    }
}

hipError_t launch_init_grid(uint8_t* g, uint32_t L, uint32_t N, uint32_t vmax, uint32_t init_v,
                            SlowParams sp, hipStream_t s) {
    const uint64_t threads = ((uint64_t)L + 3) / 4;
    const uint32_t blocks = (uint32_t)((threads + 255) / 256);
    NASCH_LAUNCH(init_grid_kernel, dim3(blocks), dim3(256), 0, s, g, L, N, vmax, init_v,
                       sp, feistel_bits(L));
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
