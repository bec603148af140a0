// launchers.hpp -- host-side entry points of the kernel translation units.
// Each returns the hipError_t of its launch (hipSuccess = 0).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nasch_device.hpp"

namespace nasch {

// Launch and report the launch's own error: a stale error left by an earlier
// call whose status was deliberately ignored is cleared first.
#define NASCH_LAUNCH(...)                 \
    do {                                  \
        (void)hipGetLastError();          \
        hipLaunchKernelGGL(__VA_ARGS__);  \
    } while (0)

// ---- init (init.hip) ----------------------------------------------------------
// Grid at t = 0 for cells [0, L): EMPTY, or the initial velocity where the
// placement puts a car.  `tab` (init_tab_words(feistel_bits(L)) words, or
// null) receives the placement's round-function table on the way.
hipError_t launch_init_grid(uint8_t* g, uint32_t L, uint32_t N, uint32_t vmax, uint32_t init_v,
                            SlowParams sp, hipStream_t s, uint32_t* tab = nullptr);
// Fill the round-function tables of the rings whose tab is set: chunk c fills
// entries [chunks[c].first, +256) of ring chunks[c].ring's table.
hipError_t launch_init_tables(const InitRing* rings, const InitChunk* chunks, uint32_t n_chunks,
                              hipStream_t s);
// Scatter the cars of many rings (grids must already be EMPTY): one thread per
// car, chunk c places cars [chunks[c].first, +kInitChunk) of ring chunks[c].ring.
hipError_t launch_init_scatter(const InitRing* rings, const InitChunk* chunks, uint32_t n_chunks,
                               hipStream_t s);
// Occupied-cell count of each chunk of kCompactChunk cells.
constexpr uint32_t kCompactChunk = 65536;
hipError_t launch_count_chunks(const uint8_t* g, uint32_t L, uint32_t* counts, hipStream_t s);
// Writes x, v of the occupied cells in ascending order; offsets[c] is the
// exclusive prefix of counts.
hipError_t launch_compact_chunks(const uint8_t* g, uint32_t L, const uint32_t* offsets,
                                 int32_t* x, uint8_t* v, hipStream_t s);
// Grid of an agent state: fill with EMPTY, then g[x[i]] = v[i].
hipError_t launch_agent_to_grid(const int32_t* x, const uint8_t* v, uint32_t N, uint8_t* g,
                                uint32_t L, hipStream_t s);
// Byte form <-> bit-plane form of roads (see RingDesc): a batch of jobs cut into
// chunks of kConvChunk words, or one job.
hipError_t launch_bytes_to_planes(const ConvJob* jobs, const ConvChunk* chunks, uint32_t n_chunks,
                                  hipStream_t s);
hipError_t launch_planes_to_bytes(const ConvJob* jobs, const ConvChunk* chunks, uint32_t n_chunks,
                                  hipStream_t s);
hipError_t launch_bytes_to_planes_one(const ConvJob& job, hipStream_t s);
hipError_t launch_planes_to_bytes_one(const ConvJob& job, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t value, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, hipStream_t s);
hipError_t launch_clock_advance(Clock* clk, uint32_t T, uint32_t nlaunch, hipStream_t s);
// F(t) of each step of a launch from the per-item partials it wrote:
// partials[s * n_items + item], items of a ring contiguous from ring.first_item;
// added into the ring's zero-initialised flux log.  max_tiles bounds ring.ntiles.
hipError_t launch_fold_ring_flux(const RingDesc* rings, const uint32_t* log_rings, uint32_t n_log,
                                 uint32_t max_tiles, const uint32_t* partials, uint32_t n_items,
                                 uint32_t k, const Clock* clk, uint32_t s_off, hipStream_t s);
hipError_t launch_fold_agent_flux(const AgentDesc* a, const uint32_t* partials, uint32_t n_items,
                                  uint32_t k, const Clock* clk, uint32_t s_off, hipStream_t s);

// ---- grid, bit-sliced, k steps per launch (grid_kstep.hip) --------------------
// Cells per wave segment for q words of 32 cells per lane.
constexpr uint32_t kstep_segment(uint32_t q) { return 64u * 32u * q; }
// vmax = kMixedVmax launches the kernel that branches on each ring's vmax;
// otherwise every item's ring must have this vmax.  open selects the open-road
// specialisation (every ring open, one vmax).
constexpr uint32_t kMixedVmax = 0xFFu;
hipError_t launch_grid_kstep(uint32_t vmax, bool open, uint32_t q, const RingDesc* rings,
                             const TileItem* items, uint32_t n_items, uint32_t* partials,
                             uint32_t k, const Clock* clk, uint32_t s_off, uint32_t launch_idx,
                             hipStream_t s);

// ---- grid, one step per launch on the byte form (grid_onestep.hip) -----------
// A wave handles a tile of 64 q words: a halo word at each end and the owned
// words in between; blocks of kOneStepThreads lanes hold independent waves.
constexpr uint32_t kOneStepThreads = 512;
// Words per lane of the one-step kernel.
constexpr uint32_t kOneStepQ = 1;
// F(t) of a one-step launch: every block stores its sum as one uint32 partial,
// and kFoldBlocks waves add the partials up in chunks (atomic adds into the
// zero-initialised log entry).
constexpr uint32_t kFoldBlocks = 64;

// Chunk c of m (m <= 64 chunks) of n uint32 F(t) partials, added by one wave
// (all 64 lanes active) and returned to every lane.  A partial is below 2^20
// and a chunk holds at most 2^16 of them, so a lane's sum stays below 2^30:
// its low 16 bits and the rest are added across the wave separately.
__device__ __forceinline__ unsigned long long chunk_sum(const uint32_t* __restrict__ partials,
                                                        uint32_t n, uint32_t c, uint32_t m,
                                                        uint32_t lane) {
    const uint32_t per = (n + m - 1u) / m;
    const uint32_t lo = min(c * per, n), hi = min(lo + per, n);
    uint32_t acc = 0u;
#pragma unroll 8
    for (uint32_t i = lo + lane; i < hi; i += 64u) acc += partials[i];   // 8 loads in flight
    const uint32_t tl = wave_total(acc & 0xFFFFu);
    const uint32_t th = wave_total(acc >> 16);
    return (unsigned long long)tl + ((unsigned long long)th << 16);
}

// Tile geometry of the one-step kernel: owned cells per tile (a ring that fits
// one tile is one tile owning all L cells), the one-word halo, tile count.
inline void onestep_geometry(uint32_t L, uint32_t q, uint32_t* own, uint32_t* halo,
                             uint32_t* ntiles) {
    const uint32_t own_full = 32u * (64u * q - 2u);
    if (L <= own_full) {
        *own = L;
        *ntiles = 1;
    } else {
        *own = own_full;
        *ntiles = (uint32_t)(((uint64_t)L + own_full - 1) / own_full);
    }
    *halo = 32u;
}
// F(t) partials of a one-step launch over ntiles tiles (one uint32 per block).
uint32_t onestep_partials(uint32_t ntiles);
// One step of the ring at `ring` (geometry from onestep_geometry with q =
// kOneStepQ, ntiles tiles): reads ring.buf[parity], writes the other buffer;
// with `log`, F(t) is added into the ring's flux log entry (which must be 0),
// through `scratch` (2 onestep_partials(ntiles) words: a launch folds the
// previous launch's partials while storing its own).  A run of launches
// s_off = 0, 1, ... folds launch i's partials in launch i + 1 (first: the
// run's first launch, whose predecessor's partials are folded already) and
// after the last one (last: in a launch of their own).  open: the ring is an
// open road.
hipError_t launch_grid_onestep(uint32_t vmax, bool open, uint32_t ntiles, const RingDesc* ring,
                               uint32_t* scratch, bool log, const Clock* clk, uint32_t s_off,
                               uint32_t launch_idx, bool first, bool last, hipStream_t s);
// One step t of a single ring given by value: reads R.buf[0], writes R.buf[1]
// (R.own and R.ntiles from onestep_geometry, R.flux_acc null), with scratch
// `scratch` of onestep_partials(R.ntiles) words; *flux = F(t) when flux is
// not null.
hipError_t launch_grid_onestep_direct(const RingDesc& R, uint32_t* scratch, uint32_t t,
                                      unsigned long long* flux, hipStream_t s);

// ---- agent (agent.hip) --------------------------------------------------------
// k steps per launch: each wave holds 64 * cpl consecutive cars (cpl cars per
// lane, kAgentMinCarsPerLane to kAgentMaxCarsPerLane) and writes back the first
// own of them, own <= 64 cpl - k (fewer steps than the tiling's k are correct
// too; one step per launch is the one-step kernel).  F(t) of wave w and step s
// goes to partials[s ntiles + w].  A run of one-step launches (k = 1, s_off =
// 0, 1, ...) may pass `prev`, the previous launch's partials (s_off >= 1): the
// launch then adds them into their log entry itself, and only the run's last
// launch needs launch_fold_agent_flux.
constexpr uint32_t kAgentMinCarsPerLane = 4;
constexpr uint32_t kAgentMaxCarsPerLane = 8;
hipError_t launch_agent_kstep(const AgentDesc* a, uint32_t cpl, uint32_t own, uint32_t ntiles,
                              uint32_t* partials, const uint32_t* prev, uint32_t k,
                              const Clock* clk, uint32_t s_off, uint32_t launch_idx,
                              hipStream_t s);

}  // namespace nasch
