// Host check of the byte <-> bit-plane conversions of the bit-sliced kernels
// (bitplanes.hpp) against cell-by-cell definitions; prints "ok" or the first
// mismatch and exits non-zero.
#include <cstdio>
#include <cstdlib>
#include <random>

#include "bitplanes.hpp"

using namespace nasch;

static uint8_t cell_byte(const uint32_t (&d)[8], int c) { return (d[c >> 2] >> (8 * (c & 3))) & 0xFF; }

template <int VMAX>
static int check_thermo(std::mt19937_64& rng) {
    for (int it = 0; it < 20000; ++it) {
        uint32_t d[8] = {};
        const int density = (int)(rng() % 33);
        for (int c = 0; c < 32; ++c) {
            const uint32_t v = (rng() % 32 < (uint64_t)density) ? (uint32_t)(rng() % (VMAX + 1)) : 0xFFu;
            d[c >> 2] |= v << (8 * (c & 3));
        }
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
    for (int it = 0; it < 100000; ++it) {
        uint32_t d[8], P[8], back[8];
        for (int i = 0; i < 8; ++i) d[i] = (uint32_t)rng();
        bytes_to_bitplanes(d, P);
        for (int c = 0; c < 32; ++c)
            for (int k = 0; k < 8; ++k)
                if (((P[k] >> c) & 1u) != ((cell_byte(d, c) >> k) & 1u))
                    return printf("bit plane %d, cell %d\n", k, c), 1;
        bitplanes_to_bytes(P, back);
        for (int i = 0; i < 8; ++i)
            if (back[i] != d[i]) return printf("round trip word %d\n", i), 1;
    }
    if (check_thermo<0>(rng) || check_thermo<1>(rng) || check_thermo<2>(rng) || check_thermo<3>(rng) ||
        check_thermo<4>(rng) || check_thermo<5>(rng) || check_thermo<6>(rng) || check_thermo<7>(rng) ||
        check_thermo<8>(rng))
        return 1;
    printf("ok\n");
    return 0;
}
