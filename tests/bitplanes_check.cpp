// Host check of the byte <-> code-plane and thermometer conversions of the bit-sliced kernels
// (bitplanes.hpp) against cell-by-cell definitions; prints "ok" or the first
// mismatch and exits non-zero.
#include <cstdio>
#include <cstdlib>
#include <random>

#include "bitplanes.hpp"

using namespace nasch;

static uint8_t cell_byte(const uint32_t (&d)[8], int c) { return (d[c >> 2] >> (8 * (c & 3))) & 0xFF; }

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
        bytes_to_thermo<VMAX>(d, T);
        for (int c = 0; c < 32; ++c) {
            const uint32_t b = cell_byte(d, c);
            if (((T[0] >> c) & 1u) != (b != 0xFFu ? 1u : 0u)) return printf("vmax %d: occupancy of cell %d\n", VMAX, c), 1;
            for (int m = 1; m <= VMAX; ++m)
                if (((T[m] >> c) & 1u) != ((b != 0xFFu && b >= (uint32_t)m) ? 1u : 0u))
                    return printf("vmax %d: plane %d of cell %d (byte %u)\n", VMAX, m, c, b), 1;
        }
        uint32_t back[8];
        thermo_to_bytes<VMAX>(T, back);
        for (int i = 0; i < 8; ++i)
            if (back[i] != d[i]) return printf("vmax %d: bytes back, word %d: %08x vs %08x\n", VMAX, i, back[i], d[i]), 1;
    }
    return 0;
}

int main() {
    std::mt19937_64 rng(12345);
    // the nibble transpose exchanges bits 8j + 4h + k and 8k + 4h + j
    for (int p = 0; p < 32; ++p) {
        const int k = p & 3, h = (p >> 2) & 1, j = p >> 3;
        if (nibble_transpose(1u << p) != 1u << (8 * k + 4 * h + j))
            return printf("nibble transpose of bit %d\n", p), 1;
    }
    // code planes of every road byte value, and the way back
    for (int it = 0; it < 100000; ++it) {
        uint32_t d[8], N[4], back[8];
        random_word(rng, 8, d);
        bytes_to_code_planes(d, N);
        for (int c = 0; c < 32; ++c) {
            for (int k = 0; k < 4; ++k)
                if (((N[k] >> c) & 1u) != ((cell_byte(d, c) >> k) & 1u))
                    return printf("code plane %d, cell %d\n", k, c), 1;
            if (((code_occupied(N) >> c) & 1u) != (cell_byte(d, c) != 0xFFu ? 1u : 0u))
                return printf("occupancy of cell %d\n", c), 1;
        }
        code_planes_to_bytes(N, back);
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
