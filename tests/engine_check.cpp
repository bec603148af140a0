// Host check of the tiling arithmetic of the runtime (engine.hpp): the k-step
// tile geometry of a ring, the agent tiling, and the agent form's choice of
// cars per lane, against their definitions; prints "ok" or the first failure
// and exits non-zero.
#include <cmath>
#include <cstdio>

#include "engine.hpp"

using namespace nasch;

static int check_kstep() {
    const uint32_t Ls[] = {1, 2, 31, 32, 33, 1000, 2047, 2048, 2049, 4096, 8191, 8192, 8193,
                           65536, 100003, 1u << 20, 1u << 30, 2147483647u};
    const uint32_t ks[] = {1, 2, 8, 16, 24, 32, 48, 64, 100, 126, 127, 252, 253, 508, 509};
    for (uint32_t q = 1; q <= 4; ++q)
        for (uint32_t vmax = 0; vmax <= 8; ++vmax)
            for (uint32_t k : ks) {
                const uint64_t seg = kstep_segment(q);
                const uint64_t H = ((uint64_t)k * vmax + 31) / 32 * 32;
                const bool fits = seg >= 2 * H + 32;
                if (vmax > 0 && fits != (k <= kstep_max_k(vmax, q)))
                    return printf("max k: q %u vmax %u k %u\n", q, vmax, k), 1;
                for (uint32_t L : Ls) {
                    uint32_t own = 0, halo = 0, nt = 0;
                    const bool ok = kstep_geometry(L, vmax, k, q, &own, &halo, &nt);
                    if (ok != fits) return printf("geometry: L %u q %u vmax %u k %u\n", L, q, vmax, k), 1;
                    if (!ok) continue;
                    if (halo % 32 || halo < (uint64_t)k * vmax || own + 2ull * halo > seg)
                        return printf("halo: L %u q %u vmax %u k %u\n", L, q, vmax, k), 1;
                    if ((uint64_t)nt * own < L || (uint64_t)(nt - 1) * own >= L)
                        return printf("tiles: L %u q %u vmax %u k %u\n", L, q, vmax, k), 1;
                    if (nt > 1 && own % 32) return printf("own: L %u\n", L), 1;
                }
            }
    return 0;
}

// The autotuner's candidates: the fixed set for every q, and for rings that
// fit one segment the deepest single-tile block (and half of it).
static int check_candidates() {
    RingDesc r{};
    r.L = 1000;
    r.vmax = 5;
    const std::vector<RingDesc> ref{r};
    uint32_t deepest = 0;
    for (auto kq : kstep_candidates(ref)) {
        uint32_t o, h, n;
        if (!kstep_geometry(r.L, r.vmax, kq.first, kq.second, &o, &h, &n))
            return printf("candidate (%u, %u) has no geometry\n", kq.first, kq.second), 1;
        if (kq.first > 64u && n != 1)
            return printf("deep candidate (%u, %u) is not one tile\n", kq.first, kq.second), 1;
        deepest = std::max(deepest, kq.first);
    }
    // q = 4: a 8192-cell segment holds L = 1000 beside halos of up to 3584 cells
    if (deepest < 600u) return printf("deepest candidate %u\n", deepest), 1;
    RingDesc big = r;
    big.L = 1u << 20;
    for (auto kq : kstep_candidates({big}))
        if (kq.first > 64u) return printf("deep candidate for a multi-tile ring\n"), 1;
    return 0;
}

// The one-step kernel's tiles: cover L, owned cells a multiple of 32 when there
// are several tiles, a one-word halo.
static int check_onestep() {
    const uint32_t Ls[] = {1, 31, 32, 1983, 1984, 1985, 4000, 8128, 100003, 1u << 30, 2147483647u};
    for (uint32_t q = 1; q <= 2; ++q)
        for (uint32_t L : Ls) {
            uint32_t own, halo, nt;
            onestep_geometry(L, q, &own, &halo, &nt);
            if ((uint64_t)nt * own < L || (uint64_t)(nt - 1) * own >= L || halo != 32u ||
                (nt > 1 && (own % 32u || own != 32u * (64u * q - 2u))))
                return printf("onestep geometry: L %u q %u\n", L, q), 1;
        }
    return 0;
}

static int check_agent() {
    const uint32_t Ns[] = {1, 7, 8, 255, 256, 257, 1000, 65536, 67108864u};
    for (uint32_t cpl = 1; cpl <= 10; ++cpl)
        for (uint32_t k = 1; k <= 600; k += 7)
            for (uint32_t N : Ns) {
                uint32_t own = 0, nt = 0;
                const bool ok = agent_geometry(N, k, cpl, &own, &nt);
                const bool want = cpl >= kAgentMinCarsPerLane && cpl <= kAgentMaxCarsPerLane &&
                                  (k + 7) / 8 * 8 + 8 <= 64 * cpl;
                if (ok != want) return printf("agent geometry: cpl %u k %u N %u\n", cpl, k, N), 1;
                if (!ok) continue;
                if (own % 8 || own + k > 64 * cpl || (uint64_t)nt * own < N ||
                    (uint64_t)(nt - 1) * own >= N)
                    return printf("agent tiles: cpl %u k %u N %u\n", cpl, k, N), 1;
            }
    // cars per lane: the fewest table passes per car, ties to more cars
    if (agent_cars_per_lane(0, 1000) != kAgentMaxCarsPerLane) return printf("N = 0\n"), 1;
    for (int i = 1; i < 1000; ++i) {
        const uint64_t L = 1u << 20, N = L * i / 1000;
        if (N == 0) continue;
        const double rho = (double)N / (double)L;
        uint32_t best = 0;
        double bc = 0;
        for (uint32_t c = kAgentMaxCarsPerLane; c >= kAgentMinCarsPerLane; --c) {
            const double cost = std::ceil((2.1 * c / rho + 2.0) / 64.0) / c;
            if (best == 0 || cost < bc * (1.0 - 1e-9)) best = c, bc = cost;
        }
        if (agent_cars_per_lane(N, L) != best) return printf("cars per lane at rho %g\n", rho), 1;
    }
    const struct { double rho; uint32_t c; } pins[] = {{0.05, 6}, {0.2, 5}, {0.25, 7}, {0.3, 8}, {0.9, 8}};
    for (const auto& p : pins)
        if (agent_cars_per_lane((uint64_t)(p.rho * 1048576), 1048576) != p.c)
            return printf("cars per lane pin at rho %g\n", p.rho), 1;
    return 0;
}

int main() {
    if (check_kstep() || check_agent() || check_candidates() || check_onestep()) return 1;
    printf("ok\n");
    return 0;
}
