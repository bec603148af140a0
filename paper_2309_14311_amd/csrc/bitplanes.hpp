// bitplanes.hpp -- conversion between the byte form of the road (one byte per
// cell: 0xFF empty, else the car's v <= 8) and the bit planes of the bit-sliced
// kernels, 32 cells at a time, by 8x8 bit-matrix transposes.
//
// A 32-cell word is eight 32-bit values d[0..7]: cell 4i + b is byte b of d[i].
// Its eight bit planes P[0..7] hold, in bit c, bit k of cell c's byte.  Each
// 8-cell block (two of the d) is an 8x8 bit matrix whose transpose puts the
// cells' bit k in its byte k; the planes are then the blocks' bytes side by
// side.  The thermometer planes the kernels use (T[0] occupancy, T[m] v >= m)
// follow from the planes of bits 0..3 (v) and bit 7 (empty).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nasch {

// 8x8 bit-matrix transpose of the 64-bit block (hi:lo): bit 8r + c and bit
// 8c + r trade places.  Three delta swaps exchange the bits one, two and four
// places off the diagonal (2x2, then 4x4 sub-blocks).
__host__ __device__ inline void transpose8x8(uint32_t& lo, uint32_t& hi) {
    uint32_t t;
    t = (lo ^ (lo >> 7)) & 0x00AA00AAu;
    lo ^= t ^ (t << 7);
    t = (hi ^ (hi >> 7)) & 0x00AA00AAu;
    hi ^= t ^ (t << 7);
    t = (lo ^ (lo >> 14)) & 0x0000CCCCu;
    lo ^= t ^ (t << 14);
    t = (hi ^ (hi >> 14)) & 0x0000CCCCu;
    hi ^= t ^ (t << 14);
    // the last swap crosses the halves: (hi:lo) >> 28 against (hi:lo)
    t = (lo ^ ((lo >> 28) | (hi << 4))) & 0xF0F0F0F0u;
    lo ^= t;
    hi ^= t >> 4;
}

// byte j of x, moved to byte position `to`
__host__ __device__ inline uint32_t byte_at(uint32_t x, int j, int to) {
    return ((x >> (8 * j)) & 0xFFu) << (8 * to);
}

// The eight bit planes of a 32-cell word of bytes.
__host__ __device__ inline void bytes_to_bitplanes(const uint32_t (&d)[8], uint32_t (&P)[8]) {
    uint32_t lo[4], hi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        lo[j] = d[2 * j];
        hi[j] = d[2 * j + 1];
        transpose8x8(lo[j], hi[j]);   // byte k: bit k of cells 8j .. 8j+7
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        P[k] = byte_at(lo[0], k, 0) | byte_at(lo[1], k, 1) | byte_at(lo[2], k, 2) |
               byte_at(lo[3], k, 3);
        P[k + 4] = byte_at(hi[0], k, 0) | byte_at(hi[1], k, 1) | byte_at(hi[2], k, 2) |
                   byte_at(hi[3], k, 3);
    }
}

// The 32 bytes of a word from its eight bit planes (the inverse).
__host__ __device__ inline void bitplanes_to_bytes(const uint32_t (&P)[8], uint32_t (&d)[8]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint32_t lo = byte_at(P[0], j, 0) | byte_at(P[1], j, 1) | byte_at(P[2], j, 2) |
                      byte_at(P[3], j, 3);
        uint32_t hi = byte_at(P[4], j, 0) | byte_at(P[5], j, 1) | byte_at(P[6], j, 2) |
                      byte_at(P[7], j, 3);
        transpose8x8(lo, hi);
        d[2 * j] = lo;
        d[2 * j + 1] = hi;
    }
}

// (b3 b2 b1 b0) >= M, bit-sliced over 32 cells, for a constant 1 <= M <= 15.
template <int M>
__host__ __device__ inline uint32_t bits_ge(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3) {
    const uint32_t b[4] = {b0, b1, b2, b3};
    uint32_t gt = 0u, eq = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 3; i >= 0; --i) {
        if ((M >> i) & 1) {
            eq &= b[i];
        } else {
            gt |= eq & b[i];
            eq &= ~b[i];
        }
    }
    return gt | eq;
}

template <int VMAX, int M>
struct ThermoFill {
    __host__ __device__ static void run(uint32_t occ, uint32_t b0, uint32_t b1, uint32_t b2,
                                        uint32_t b3, uint32_t (&T)[VMAX + 1]) {
        if constexpr (M <= VMAX) {
            T[M] = occ & bits_ge<M>(b0, b1, b2, b3);
            ThermoFill<VMAX, M + 1>::run(occ, b0, b1, b2, b3, T);
        }
    }
};

// Thermometer planes of a word of bytes (0xFF or v <= VMAX): T[0] occupancy,
// T[m] the cells whose car has v >= m.
template <int VMAX>
__host__ __device__ inline void bytes_to_thermo(const uint32_t (&d)[8], uint32_t (&T)[VMAX + 1]) {
    uint32_t P[8];
    bytes_to_bitplanes(d, P);
    const uint32_t occ = ~P[7];   // v <= 8 leaves bit 7 clear; 0xFF sets it
    T[0] = occ;
    ThermoFill<VMAX, 1>::run(occ, P[0], P[1], P[2], P[3], T);
}

// T[M] of a thermometer code, zero above VMAX.
template <int VMAX, int M>
__host__ __device__ inline uint32_t thermo_at(const uint32_t (&T)[VMAX + 1]) {
    if constexpr (M <= VMAX) return T[M];
    else return 0u;
}

// Bytes of a word from its thermometer planes: 0xFF where T[0] is clear, else
// v = the number of planes m >= 1 that hold the cell.
template <int VMAX>
__host__ __device__ inline void thermo_to_bytes(const uint32_t (&T)[VMAX + 1], uint32_t (&d)[8]) {
    const uint32_t t1 = thermo_at<VMAX, 1>(T), t2 = thermo_at<VMAX, 2>(T);
    const uint32_t t3 = thermo_at<VMAX, 3>(T), t4 = thermo_at<VMAX, 4>(T);
    const uint32_t t5 = thermo_at<VMAX, 5>(T), t6 = thermo_at<VMAX, 6>(T);
    const uint32_t t7 = thermo_at<VMAX, 7>(T), t8 = thermo_at<VMAX, 8>(T);
    const uint32_t e = ~T[0];
    // binary digits of v from the thermometer: bit i of v is set where v lies
    // in a range [j 2^i, (j + 1) 2^i) with j odd
    const uint32_t b0 = (t1 & ~t2) | (t3 & ~t4) | (t5 & ~t6) | (t7 & ~t8);
    const uint32_t b1 = (t2 & ~t4) | (t6 & ~t8);
    const uint32_t b2 = t4 & ~t8;
    const uint32_t b3 = t8;
    const uint32_t P[8] = {b0 | e, b1 | e, b2 | e, b3 | e, e, e, e, e};
    bitplanes_to_bytes(P, d);
}

}  // namespace nasch
