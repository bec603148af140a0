// bitplanes.hpp -- conversion between the byte form of the road (one byte per
// cell: 0xFF empty, else the car's v <= 8) and the bit planes of the bit-sliced
// kernels, 32 cells at a time, by bit-matrix transposes in registers.
//
// A 32-cell word is eight 32-bit values d[0..7]: cell 4i + b is byte b of d[i].
// Such a byte is 0xFF or at most 8, so its low four bits (its code) identify it:
// code 15 only for an empty cell.  The four code planes N[0..3] hold, in bit c,
// bit k of cell c's code.  Packed two cells to a byte, the codes of eight cells
// fill one 32-bit value: in nibble word i (cells 8i .. 8i+7), byte j holds cell
// 8i + j in its low and cell 8i + 4 + j in its high nibble, so bit 8j + 4h + k
// is bit k of cell 8i + 4h + j.  Exchanging the index bits j and k (two delta
// swaps) puts bit k of the eight cells in byte k, and the code planes are
// those bytes side by side.  The thermometer planes the kernels use (T[0]
// occupancy, T[m] v >= m) follow from the code planes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nasch {

// Exchange the bits of x selected by m with the bits d places above them.
__host__ __device__ inline uint32_t delta_swap(uint32_t x, uint32_t m, int d) {
    const uint32_t t = (x ^ (x >> d)) & m;
    return x ^ t ^ (t << d);
}

// Bit 8j + 4h + k and bit 8k + 4h + j trade places (j, k in 0..3, h in 0..1):
// index bits 0 and 3 are exchanged 7 places apart, index bits 1 and 4 14
// places apart.  The map is its own inverse.
__host__ __device__ inline uint32_t nibble_transpose(uint32_t x) {
    return delta_swap(delta_swap(x, 0x00AA00AAu, 7), 0x0000CCCCu, 14);
}

// byte j of x, moved to byte position `to`
__host__ __device__ inline uint32_t byte_at(uint32_t x, int j, int to) {
    return ((x >> (8 * j)) & 0xFFu) << (8 * to);
}

// The four code planes of a 32-cell word of bytes.
__host__ __device__ inline void bytes_to_code_planes(const uint32_t (&d)[8], uint32_t (&N)[4]) {
    uint32_t n[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        n[i] = nibble_transpose((d[2 * i] & 0x0F0F0F0Fu) | ((d[2 * i + 1] << 4) & 0xF0F0F0F0u));
#pragma unroll
    for (int k = 0; k < 4; ++k)
        N[k] = byte_at(n[0], k, 0) | byte_at(n[1], k, 1) | byte_at(n[2], k, 2) | byte_at(n[3], k, 3);
}

// Each byte of x holds a code (0..8, or 15 for an empty cell); 15 becomes 0xFF.
// Only code 15 has both bit 3 and bit 0 set, so x & (x << 3) leaves 8 in those
// bytes and nothing elsewhere, and 8 * 30 = 0xF0 fills their high nibble.
__host__ __device__ inline uint32_t code_bytes(uint32_t x) {
    return x | ((x & (x << 3)) * 30u);
}

// The 32 bytes of a word from its code planes (the inverse).
__host__ __device__ inline void code_planes_to_bytes(const uint32_t (&N)[4], uint32_t (&d)[8]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t n = nibble_transpose(byte_at(N[0], i, 0) | byte_at(N[1], i, 1) |
                                            byte_at(N[2], i, 2) | byte_at(N[3], i, 3));
        d[2 * i] = code_bytes(n & 0x0F0F0F0Fu);
        d[2 * i + 1] = code_bytes((n >> 4) & 0x0F0F0F0Fu);
    }
}

// Occupancy from the code planes: only an empty cell has code bits 3 and 0 both set.
__host__ __device__ inline uint32_t code_occupied(const uint32_t (&N)[4]) {
    return ~(N[0] & N[3]);
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
    uint32_t N[4];
    bytes_to_code_planes(d, N);
    const uint32_t occ = code_occupied(N);
    T[0] = occ;
    ThermoFill<VMAX, 1>::run(occ, N[0], N[1], N[2], N[3], T);
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
    const uint32_t N[4] = {b0 | e, b1 | e, b2 | e, b3 | e};   // code 15 where empty
    code_planes_to_bytes(N, d);
}

}  // namespace nasch
