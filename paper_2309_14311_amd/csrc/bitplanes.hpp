// bitplanes.hpp -- conversion between the byte form of the road (one byte per
// cell: 0xFF empty, else the car's v <= 8) and the bit planes of the bit-sliced
// kernels, 32 cells at a time, by exchanges of index bits in registers.
//
// A 32-cell word is eight 32-bit values d[0..7]: cell c is byte c & 3 of
// d[c >> 2].  Such a byte is 0xFF or at most 8, so its low four bits (its
// code) identify it: code 15 only for an empty cell.  The four code planes
// N[0..3] hold, in bit c, bit k of cell c's code.  Label each code bit by the
// index bits of its cell c = (c4 c3 c2 c1 c0) and of the code bit k = (k1 k0);
// the bytes hold it in register (c4 c3 c2) at bit (c1 c0 . k1 k0) (a dot for
// the unused high nibble), the planes in register (k1 k0) at bit (c4 .. c0).
// Three exchanges of index bits get from one to the other:
//   1. pack two registers into one of nibbles: bit (c1 c0 c2 k1 k0) of
//      register (c4 c3): c2 moves into the bit index;
//   2. transpose the 4 x 4 bytes of those registers with byte permutes:
//      bit (c4 c3 c2 k1 k0) of register (c1 c0);
//   3. exchange k0 with c0 and k1 with c1 between pairs of registers
//      (masked shifts by 1 and 2): bit (c4 c3 c2 c1 c0) of register (k1 k0).
// On gfx950 a byte permute, like a shift, takes one 4-cycle issue slot and a
// three-input bitwise operation or an add half of one, so the steps use byte
// permutes for whole bytes and doubling adds for left shifts where they can.
// The way back runs the exchanges in reverse and turns code 15 into 0xFF with
// a byte-permute lookup.  The thermometer planes the kernels use (T[0]
// occupancy, T[m] v >= m) follow from the code planes.
//
// The byte permute is passed in (`perm`, the semantics of v_perm_b32: byte i
// of perm(hi, lo, sel) is byte sel_i of the eight bytes lo[0..3] hi[0..3] for
// sel_i <= 7, 0x00 for sel_i = 12 and 0xFF for sel_i >= 13), so that the same
// code runs on the device (HwPerm, the instruction) and in a host check that
// models it.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nasch {

// The device's byte permute.
struct HwPerm {
    __device__ uint32_t operator()(uint32_t hi, uint32_t lo, uint32_t sel) const {
        return __builtin_amdgcn_perm(hi, lo, sel);
    }
};

// Bitwise m ? a : b.  On the device one v_bitop3_b32 (truth table 0xCA over
// (m, a, b)): the compiler's own choice for this pattern, v_bfi_b32, like
// v_and_or_b32, issues in 4 cycles per wave64, v_bitop3_b32 in 2.
__host__ __device__ inline uint32_t select_bits(uint32_t m, uint32_t a, uint32_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(m, a, b, 0xCA);
#else
    return (a & m) | (b & ~m);
#endif
}

// (a & m) | c, on the device one v_bitop3_b32 (truth table 0xEA over (a, m, c)).
__host__ __device__ inline uint32_t and_or_bits(uint32_t a, uint32_t m, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, m, c, 0xEA);
#else
    return (a & m) | c;
#endif
}

// (a & m) | (b & ~m)
__host__ __device__ inline uint32_t bit_select(uint32_t a, uint32_t b, uint32_t m) {
    return select_bits(m, a, b);
}

// 4 x 4 byte transpose: byte i of out[j] = byte j of in[i].  Involution.
template <class Perm>
__host__ __device__ inline void byte_transpose4(const uint32_t (&in)[4], uint32_t (&out)[4],
                                                Perm perm) {
    // pairs of rows: bytes (in0.j, in1.j, in0.j+2, in1.j+2) for j = 0, 1
    const uint32_t t0 = perm(in[1], in[0], 0x06020400u);
    const uint32_t t1 = perm(in[1], in[0], 0x07030501u);
    const uint32_t t2 = perm(in[3], in[2], 0x06020400u);
    const uint32_t t3 = perm(in[3], in[2], 0x07030501u);
    out[0] = perm(t2, t0, 0x05040100u);
    out[2] = perm(t2, t0, 0x07060302u);
    out[1] = perm(t3, t1, 0x05040100u);
    out[3] = perm(t3, t1, 0x07060302u);
}

// Exchange bit-index bit s (mask m selects the bits where it is 0) with the
// register index bit that tells a from b: a keeps its bits where the index bit
// is 0 and takes b's from there (shifted up by 2^s); b takes a's bits where the
// index bit is 1 (shifted down) and keeps its own.  Involution.
template <int S>
__host__ __device__ inline void swap_bits(uint32_t& a, uint32_t& b, uint32_t m) {
    const uint32_t bl = b & m;
    uint32_t up;
    if constexpr (S == 0) up = bl + bl;            // << 1 as an add
    else up = bl << (1 << S);
    const uint32_t na = and_or_bits(a, m, up);
    b = bit_select(a >> (1 << S), b, m);
    a = na;
}

// The four code planes of a 32-cell word of bytes.
template <class Perm = HwPerm>
__host__ __device__ inline void bytes_to_code_planes(const uint32_t (&d)[8], uint32_t (&N)[4],
                                                     Perm perm = Perm()) {
    // 1. nibble word i: low nibbles from d[2i], high nibbles from d[2i + 1]
    uint32_t n[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) n[i] = bit_select(d[2 * i], d[2 * i + 1] << 4, 0x0F0F0F0Fu);
    // 2. byte transpose: register (c1 c0), byte (c4 c3)
    uint32_t m[4];
    byte_transpose4(n, m, perm);
    // 3. k0 <-> c0 (registers 0/1, 2/3), then k1 <-> c1 (registers 0/2, 1/3)
    swap_bits<0>(m[0], m[1], 0x55555555u);
    swap_bits<0>(m[2], m[3], 0x55555555u);
    swap_bits<1>(m[0], m[2], 0x33333333u);
    swap_bits<1>(m[1], m[3], 0x33333333u);
#pragma unroll
    for (int k = 0; k < 4; ++k) N[k] = m[k];
}

// The 32 bytes of a word from its code planes (the inverse): code 15 becomes
// 0xFF through a byte-permute lookup whose selectors 0..7 return themselves
// and 13..15 return 0xFF; selector 8 returns 0x00, so when code 8 (v = 8) may
// occur its bit 3 is ORed back in (a no-op for 0xFF).
template <bool MAY_HOLD_8 = true, class Perm = HwPerm>
__host__ __device__ inline void code_planes_to_bytes(const uint32_t (&N)[4], uint32_t (&d)[8],
                                                     Perm perm = Perm()) {
    uint32_t m[4] = {N[0], N[1], N[2], N[3]};
    swap_bits<1>(m[0], m[2], 0x33333333u);
    swap_bits<1>(m[1], m[3], 0x33333333u);
    swap_bits<0>(m[0], m[1], 0x55555555u);
    swap_bits<0>(m[2], m[3], 0x55555555u);
    uint32_t n[4];
    byte_transpose4(m, n, perm);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t lo = n[i] & 0x0F0F0F0Fu, hi = (n[i] >> 4) & 0x0F0F0F0Fu;
        d[2 * i] = perm(0x07060504u, 0x03020100u, lo);
        d[2 * i + 1] = perm(0x07060504u, 0x03020100u, hi);
        if constexpr (MAY_HOLD_8) {
            d[2 * i] = and_or_bits(lo, 0x08080808u, d[2 * i]);
            d[2 * i + 1] = and_or_bits(hi, 0x08080808u, d[2 * i + 1]);
        }
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
template <int VMAX, class Perm = HwPerm>
__host__ __device__ inline void bytes_to_thermo(const uint32_t (&d)[8], uint32_t (&T)[VMAX + 1],
                                                Perm perm = Perm()) {
    uint32_t N[4];
    bytes_to_code_planes(d, N, perm);
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
template <int VMAX, class Perm = HwPerm>
__host__ __device__ inline void thermo_to_bytes(const uint32_t (&T)[VMAX + 1], uint32_t (&d)[8],
                                                Perm perm = Perm()) {
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
    code_planes_to_bytes<(VMAX >= 8)>(N, d, perm);
}

}  // namespace nasch
