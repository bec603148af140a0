// Host check of the byte <-> code-plane and thermometer conversions of the bit-sliced kernels
// (bitplanes.hpp) against cell-by-cell definitions; prints "ok" or the first
// mismatch and exits non-zero.
#include <cstdio>
#include <cstdlib>
#include <random>

#include "bitplanes.hpp"

using namespace nasch;

static uint8_t cell_byte(const uint32_t (&d)[8], int c) { return (d[c >> 2] >> (8 * (c & 3))) & 0xFF; }

// A model of the device's byte permute (v_perm_b32): byte i of the result is
// selected by byte i of sel from the eight bytes lo[0..3] hi[0..3]; 8..11 give
// the sign of bytes 1, 3, 5, 7 spread over the byte, 12 gives 0x00 and 13 and
// above give 0xFF.
struct ModelPerm {
    uint32_t operator()(uint32_t hi, uint32_t lo, uint32_t sel) const {
        const uint64_t data = ((uint64_t)hi << 32) | lo;
        uint32_t out = 0;
        for (int i = 0; i < 4; ++i) {
            const uint32_t s = (sel >> (8 * i)) & 0xFFu;
            uint32_t b;
            if (s <= 7) b = (uint32_t)(data >> (8 * s)) & 0xFFu;
            else if (s <= 11) b = ((data >> (8 * (2 * (s - 8) + 1) + 7)) & 1u) ? 0xFFu : 0u;
            else if (s == 12) b = 0u;
            else b = 0xFFu;
            out |= b << (8 * i);
        }
        return out;
    }
};

// A random 32-cell word of road bytes: each cell 0xFF (empty) or, with
// probability density/32 for a random density, a velocity v <= vmax.
static void random_word(std::mt19937_64& rng, uint32_t vmax, uint32_t (&d)[8]) {
    const int density = (int)(rng() % 33);
    for (int i = 0; i < 8; ++i) d[i] = 0u;
    for (int c = 0; c < 32; ++c) {
        const uint32_t v = (rng() % 32 < (uint64_t)density) ? (uint32_t)(rng() % (vmax + 1)) : 0xFFu;
        d[c >> 2] |= v << (8 * (c & 3));
    }
}

template <int VMAX>
static int check_thermo(std::mt19937_64& rng) {
    for (int it = 0; it < 20000; ++it) {
        uint32_t d[8];
        random_word(rng, VMAX, d);
        uint32_t T[VMAX + 1];
        bytes_to_thermo<VMAX>(d, T, ModelPerm());
        for (int c = 0; c < 32; ++c) {
            const uint32_t b = cell_byte(d, c);
            if (((T[0] >> c) & 1u) != (b != 0xFFu ? 1u : 0u)) return printf("vmax %d: occupancy of cell %d\n", VMAX, c), 1;
            for (int m = 1; m <= VMAX; ++m)
                if (((T[m] >> c) & 1u) != ((b != 0xFFu && b >= (uint32_t)m) ? 1u : 0u))
                    return printf("vmax %d: plane %d of cell %d (byte %u)\n", VMAX, m, c, b), 1;
        }
        uint32_t back[8];
        thermo_to_bytes<VMAX>(T, back, ModelPerm());
        for (int i = 0; i < 8; ++i)
            if (back[i] != d[i]) return printf("vmax %d: bytes back, word %d: %08x vs %08x\n", VMAX, i, back[i], d[i]), 1;
    }
    return 0;
}

int main() {
    std::mt19937_64 rng(12345);
    // the byte transpose: byte i of out[j] is byte j of in[i]
    for (int it = 0; it < 1000; ++it) {
        uint32_t in[4], out[4];
        for (auto& w : in) w = (uint32_t)rng();
        byte_transpose4(in, out, ModelPerm());
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j)
                if (((out[j] >> (8 * i)) & 0xFFu) != ((in[i] >> (8 * j)) & 0xFFu))
                    return printf("byte transpose %d %d\n", i, j), 1;
    }
    // code planes of every road byte value, and the way back
    for (int it = 0; it < 100000; ++it) {
        uint32_t d[8], N[4], back[8];
        random_word(rng, 8, d);
        bytes_to_code_planes(d, N, ModelPerm());
        for (int c = 0; c < 32; ++c) {
            for (int k = 0; k < 4; ++k)
                if (((N[k] >> c) & 1u) != ((cell_byte(d, c) >> k) & 1u))
                    return printf("code plane %d, cell %d\n", k, c), 1;
            if (((code_occupied(N) >> c) & 1u) != (cell_byte(d, c) != 0xFFu ? 1u : 0u))
                return printf("occupancy of cell %d\n", c), 1;
        }
        code_planes_to_bytes(N, back, ModelPerm());
        for (int i = 0; i < 8; ++i)
            if (back[i] != d[i]) return printf("round trip word %d: %08x vs %08x\n", i, back[i], d[i]), 1;
    }
    if (check_thermo<0>(rng) || check_thermo<1>(rng) || check_thermo<2>(rng) || check_thermo<3>(rng) ||
        check_thermo<4>(rng) || check_thermo<5>(rng) || check_thermo<6>(rng) || check_thermo<7>(rng) ||
        check_thermo<8>(rng))
        return 1;
    printf("ok\n");
    return 0;
}
