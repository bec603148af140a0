// runtime.hip -- the C ABI of libnasch for single simulations and batches.
// Entry points are declared and documented in include/nasch.h.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "engine.hpp"
#include "nasch.h"

using namespace nasch;

namespace {
constexpr uint32_t kDefaultK = 32;
constexpr uint32_t kDefaultQ = 4;
constexpr uint32_t kDefaultAgentK = 32;

// Default (k, q) for a ring: the largest segment, k = 32 or the most it admits.
void default_tuning(uint32_t L, uint32_t vmax, uint32_t* k, uint32_t* q) {
    *q = kDefaultQ;
    if (L <= 2048) *q = 1;
    *k = std::min(kDefaultK, kstep_max_k(vmax, *q));
    if (*k == 0) *k = 1;
}
}  // namespace

struct nasch_sim {
    // model
    uint64_t L = 0, N = 0, seed = 0;
    uint32_t vmax = 0, thr = 0, replica = 0, rep = 0, init_v = 0;
    double p = 0;
    bool open = false;        // open road (grid form only)
    // tuning
    uint32_t kernel = NASCH_KERNEL_KSTEP, k = kDefaultK, q = kDefaultQ, use_graph = 0;
    // stream and status
    hipStream_t stream = nullptr;
    bool own_stream = false;
    HipStatus st;
    // step counter (host mirror of the device clock)
    uint64_t t = 0;
    uint32_t parity = 0;
    Clock* d_clk = nullptr;
    // grid representation: bytes (one-step kernel, snapshots) and bit planes
    // (temporal-blocked kernel); the current state is at index `parity` in the
    // forms marked valid
    uint8_t* grid[2] = {nullptr, nullptr};
    uint32_t* planes[2] = {nullptr, nullptr};
    bool bytes_ok = true, planes_ok = false;
    GridEngine eng;           // one ring, its tiles (bit planes, k steps per launch)
    GridEngine eng1;          // the same ring for the one-step kernel (bytes, k = 1)
    uint32_t* os_partials = nullptr;   // agent F(t) partials
    size_t os_partials_cap = 0;
    // agent representation
    int32_t* ax[2] = {nullptr, nullptr};
    uint8_t* av[2] = {nullptr, nullptr};
    AgentDesc h_agent{};
    AgentDesc* d_agent = nullptr;
    // tiling of the agent k-step kernel: cars per lane, cars written back per
    // wave, waves.  The one-step launches keep a tiling of their own, eight cars
    // per lane, whose vector loads and stores keep that HBM-bound kernel at speed.
    uint32_t agent_cpl = kAgentMaxCarsPerLane, agent_own = 0, agent_ntiles = 0;
    uint32_t agent_own1 = 0, agent_ntiles1 = 0;
    uint8_t* agent_grid = nullptr;  // scratch grid for snapshots
    uint32_t* mlcg_pow = nullptr;   // jump table of the shared stream
    uint32_t rng = NASCH_RNG_KEYED;
    // F(t) log: flux[t - log_t0]
    unsigned long long* flux = nullptr;
    uint64_t flux_cap = 0, log_t0 = 0;
    GraphCache graphs;
    uint64_t dev_bytes = 0;

    ~nasch_sim();
    int fail() { return NASCH_EDEVICE; }
    bool ok(hipError_t e) { return st.ok(e); }
    int ensure_log(uint64_t steps);
    int refresh_descs();
    int enqueue_steps(uint64_t T);
    int set_tuning(uint32_t kern, uint32_t kk, uint32_t qq);
    const uint8_t* current_grid_device();
    ConvJob conv_job() const {
        return ConvJob{grid[parity], planes[parity], (uint32_t)L, plane_words(L), vmax, 0u};
    }
    // make the bit planes (or the bytes) of the current state valid
    bool need_planes() {
        if (planes_ok) return true;
        if (!ok(launch_bytes_to_planes_one(conv_job(), stream))) return false;
        planes_ok = true;
        return true;
    }
    bool need_bytes() {
        if (bytes_ok) return true;
        if (!ok(launch_planes_to_bytes_one(conv_job(), stream))) return false;
        bytes_ok = true;
        return true;
    }
    // Captured graphs bake the partials pointer in: a new buffer drops them.
    int ensure_os_partials(size_t n) {
        if (n <= os_partials_cap) return NASCH_OK;
        graphs.clear();
        if (stream) (void)hipStreamSynchronize(stream);
        if (os_partials) (void)hipFree(os_partials);
        os_partials = nullptr;
        os_partials_cap = 0;
        if (!ok(dev_alloc(&os_partials, n))) return NASCH_ENOMEM;
        os_partials_cap = n;
        return NASCH_OK;
    }
};

nasch_sim::~nasch_sim() {
    graphs.clear();
    eng.release();
    eng1.release();
    // agent_grid aliases grid[0]
    void* ps[] = {d_clk, grid[0], grid[1], planes[0], planes[1], ax[0], ax[1], av[0],
                  av[1], d_agent, flux, os_partials, mlcg_pow};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    (void)hipGetLastError();  // errors of the teardown are not reported to later calls
}

// Keep room in the flux log for `steps` more steps from t.
int nasch_sim::ensure_log(uint64_t steps) {
    const uint64_t need = t + steps - log_t0;
    if (need <= flux_cap) return NASCH_OK;
    uint64_t cap = std::max<uint64_t>(need, std::max<uint64_t>(1024, flux_cap * 2));
    unsigned long long* nf = nullptr;
    if (!ok(dev_alloc(&nf, cap))) return NASCH_ENOMEM;
    if (!ok(launch_fill_u64(nf, cap, stream))) { (void)hipFree(nf); return fail(); }
    if (flux && flux_cap) {
        if (!ok(hipMemcpyAsync(nf, flux, flux_cap * sizeof(unsigned long long),
                               hipMemcpyDeviceToDevice, stream))) {
            (void)hipFree(nf);
            return fail();
        }
    }
    if (!ok(hipStreamSynchronize(stream))) { (void)hipFree(nf); return fail(); }
    if (flux) (void)hipFree(flux);
    dev_bytes += (cap - flux_cap) * sizeof(unsigned long long);
    flux = nf;
    flux_cap = cap;
    return refresh_descs();
}

// Push the descriptors (pointers, geometry) to the device.
int nasch_sim::refresh_descs() {
    if (rep == NASCH_REP_GRID) {
        for (GridEngine* g : {&eng, &eng1}) {
            RingDesc& r = g->rings[0];
            r.flux_log = flux;
            r.log_t0 = log_t0;
            if (!ok(g->upload_rings(stream))) return fail();
        }
    } else {
        h_agent.flux_log = flux;
        h_agent.log_t0 = log_t0;
        if (!ok(hipMemcpyAsync(d_agent, &h_agent, sizeof(AgentDesc), hipMemcpyHostToDevice, stream)))
            return fail();
    }
    if (!ok(hipStreamSynchronize(stream))) return fail();
    return NASCH_OK;
}

int nasch_sim::set_tuning(uint32_t kern, uint32_t kk, uint32_t qq) {
    if (kern == NASCH_KERNEL_AUTO) kern = NASCH_KERNEL_KSTEP;
    if (kern != NASCH_KERNEL_ONESTEP && kern != NASCH_KERNEL_KSTEP) return NASCH_EINVAL;
    if (kk == 0) kk = k;
    if (qq == 0) qq = q;
    if (rep == NASCH_REP_GRID) {
        if (kern == NASCH_KERNEL_KSTEP) {
            uint32_t o, h, n;
            if (!kstep_geometry((uint32_t)L, vmax, kk, qq, &o, &h, &n)) return NASCH_EINVAL;
            if (eng.k != kk || eng.q != qq) {
                if (!ok(eng.set_geometry(kk, qq, stream))) return fail();
                graphs.clear();
            }
        }
    } else {
        // the agent form's q is the number of cars per lane of the k-step tiling
        if (qq < kAgentMinCarsPerLane || qq > kAgentMaxCarsPerLane) return NASCH_EINVAL;
        if (kern == NASCH_KERNEL_KSTEP || qq != agent_cpl) {
            uint32_t own, ntiles;
            if (!agent_geometry((uint32_t)N, kk, qq, &own, &ntiles)) return NASCH_EINVAL;
            int rc = ensure_os_partials((size_t)ntiles * kk);
            if (rc) return rc;
            if (agent_own != own || agent_ntiles != ntiles || agent_cpl != qq) {
                agent_own = own;
                agent_ntiles = ntiles;
                agent_cpl = qq;
                graphs.clear();
            }
        }
    }
    kernel = kern;
    k = kk;
    q = qq;
    return NASCH_OK;
}

// The launches of T steps followed by the clock update (not synchronised).
int nasch_sim::enqueue_steps(uint64_t T) {
    const bool grid_kstep = rep == NASCH_REP_GRID && kernel != NASCH_KERNEL_ONESTEP;
    if (rep == NASCH_REP_GRID && !(grid_kstep ? need_planes() : need_bytes())) return fail();
    auto body = [&]() -> hipError_t {
        uint32_t nl = 0;
        if (rep == NASCH_REP_GRID) {
            if (kernel == NASCH_KERNEL_ONESTEP) {
                hipError_t e = eng1.enqueue(T, d_clk, stream);
                if (e != hipSuccess) return e;
                nl = eng1.launches_for(T);
            } else {
                hipError_t e = eng.enqueue(T, d_clk, stream);
                if (e != hipSuccess) return e;
                nl = eng.launches_for(T);
            }
        } else {
            if (kernel == NASCH_KERNEL_ONESTEP) {
                // one step per launch: the k-step kernel with one step, on the
                // one-step tiling.  The partials of consecutive launches
                // alternate between two sets; each launch folds the previous
                // one's, and a fold launch the last one's.
                const auto set = [&](uint64_t i) {
                    return os_partials + (size_t)(i & 1u) * agent_ntiles1;
                };
                for (uint64_t i = 0; i < T; ++i) {
                    hipError_t e = launch_agent_kstep(d_agent, kAgentMaxCarsPerLane, agent_own1,
                                                      agent_ntiles1, set(i),
                                                      i ? set(i - 1u) : nullptr, 1u, d_clk,
                                                      (uint32_t)i, (uint32_t)i, stream);
                    if (e == hipSuccess && i + 1u == T)
                        e = launch_fold_agent_flux(d_agent, set(i), agent_ntiles1, 1u, d_clk,
                                                   (uint32_t)i, stream);
                    if (e != hipSuccess) return e;
                }
                nl = (uint32_t)T;
            } else {
                nl = (uint32_t)((T + k - 1) / k);
                for (uint32_t i = 0; i < nl; ++i) {
                    const uint32_t ki = (uint32_t)std::min<uint64_t>(k, T - (uint64_t)i * k);
                    hipError_t e = launch_agent_kstep(d_agent, agent_cpl, agent_own,
                                                      agent_ntiles, os_partials, nullptr, ki,
                                                      d_clk, i * k, i, stream);
                    if (e == hipSuccess)
                        e = launch_fold_agent_flux(d_agent, os_partials, agent_ntiles, ki, d_clk,
                                                   i * k, stream);
                    if (e != hipSuccess) return e;
                }
            }
        }
        return launch_clock_advance(d_clk, (uint32_t)T, nl, stream);
    };
    hipError_t e;
    if (use_graph) {
        e = graphs.run(std::make_tuple(T, kernel, k, q, eng.version), stream, body);
    } else {
        e = body();
    }
    if (!ok(e)) return fail();
    uint32_t nl;
    if (kernel == NASCH_KERNEL_ONESTEP) nl = (uint32_t)T;
    else if (rep == NASCH_REP_GRID) nl = eng.launches_for(T);
    else nl = (uint32_t)((T + k - 1) / k);
    t += T;
    parity ^= nl & 1u;
    if (rep == NASCH_REP_GRID) {
        planes_ok = grid_kstep;
        bytes_ok = !grid_kstep;
    }
    return NASCH_OK;
}

const uint8_t* nasch_sim::current_grid_device() {
    if (rep == NASCH_REP_GRID) return need_bytes() ? grid[parity] : nullptr;
    if (!ok(launch_agent_to_grid(ax[parity], av[parity], (uint32_t)N, agent_grid, (uint32_t)L,
                                 stream)))
        return nullptr;
    return agent_grid;
}

// Agent vectors from the grid in grid[0] (used at init and restore).
static int agent_from_grid(nasch_sim* h, const uint8_t* d_grid) {
    const uint32_t chunks = (uint32_t)((h->L + kCompactChunk - 1) / kCompactChunk);
    uint32_t* d_counts = nullptr;
    if (!h->ok(dev_alloc(&d_counts, chunks))) return NASCH_ENOMEM;
    std::vector<uint32_t> counts(chunks), offs(chunks);
    int rc = NASCH_OK;
    if (!h->ok(launch_count_chunks(d_grid, (uint32_t)h->L, d_counts, h->stream)) ||
        !h->ok(hipMemcpyAsync(counts.data(), d_counts, chunks * sizeof(uint32_t),
                              hipMemcpyDeviceToHost, h->stream)) ||
        !h->ok(hipStreamSynchronize(h->stream))) {
        rc = NASCH_EDEVICE;
    } else {
        uint64_t acc = 0;
        for (uint32_t c = 0; c < chunks; ++c) {
            offs[c] = (uint32_t)acc;
            acc += counts[c];
        }
        if (acc != h->N) {
            rc = NASCH_EINVAL;
        } else if (!h->ok(hipMemcpyAsync(d_counts, offs.data(), chunks * sizeof(uint32_t),
                                         hipMemcpyHostToDevice, h->stream)) ||
                   !h->ok(launch_compact_chunks(d_grid, (uint32_t)h->L, d_counts,
                                                h->ax[h->parity], h->av[h->parity], h->stream)) ||
                   !h->ok(hipStreamSynchronize(h->stream))) {
            rc = NASCH_EDEVICE;
        }
    }
    (void)hipFree(d_counts);
    return rc;
}

extern "C" {

void nasch_default_opts(nasch_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->rep = NASCH_REP_GRID;
    o->init_v = NASCH_INIT_V_ZERO;
    o->kernel = NASCH_KERNEL_AUTO;
}

const char* nasch_strerror(int s) {
    switch (s) {
        case NASCH_OK: return "ok";
        case NASCH_EINVAL: return "invalid argument";
        case NASCH_ENOMEM: return "out of memory";
        case NASCH_EDEVICE: return "HIP device error";
        case NASCH_ERANGE: return "step counter would reach 2^32";
        case NASCH_ESTATE: return "invalid state for this call";
        case NASCH_EBUSY: return "busy";
        case NASCH_ENOTFOUND: return "not found";
        default: return "unknown status";
    }
}

int nasch_init(nasch_sim** out, uint64_t L, uint64_t N, uint32_t vmax, double p, uint64_t seed,
               const nasch_opts* opts) {
    if (!out) return NASCH_EINVAL;
    *out = nullptr;
    nasch_opts o;
    nasch_default_opts(&o);
    if (opts) o = *opts;
    // the agent form's kernels take any vmax up to 254, the grid form's up to 8
    int rc = validate_params(L, N, vmax, p,
                             o.rep == NASCH_REP_AGENT ? NASCH_MAX_VMAX_AGENT : NASCH_MAX_VMAX);
    if (rc) return rc;
    if (o.rep > NASCH_REP_AGENT || o.init_v > NASCH_INIT_V_UNIFORM || o.kernel > NASCH_KERNEL_KSTEP ||
        o.rng > NASCH_RNG_STREAM)
        return NASCH_EINVAL;
    if (o.rng == NASCH_RNG_STREAM && o.rep != NASCH_REP_AGENT) return NASCH_EINVAL;
    if (o.boundary > NASCH_BOUNDARY_OPEN || o.reserved != 0) return NASCH_EINVAL;
    const bool open = o.boundary == NASCH_BOUNDARY_OPEN;
    if (open) {
        // alpha, beta in [0, 1] (NaN fails both comparisons)
        if (o.rep != NASCH_REP_GRID || !(o.alpha >= 0.0 && o.alpha <= 1.0) ||
            !(o.beta >= 0.0 && o.beta <= 1.0))
            return NASCH_EINVAL;
    }
    std::unique_ptr<nasch_sim> h(new (std::nothrow) nasch_sim());
    if (!h) return NASCH_ENOMEM;
    h->L = L; h->N = N; h->vmax = vmax; h->p = p; h->seed = seed;
    h->thr = threshold_of(p);
    h->replica = o.replica; h->rep = o.rep; h->init_v = o.init_v;
    h->use_graph = o.use_graph;
    h->open = open;
    if (o.stream) {
        h->stream = (hipStream_t)o.stream;
    } else {
        if (!h->ok(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking))) return NASCH_EDEVICE;
        h->own_stream = true;
    }
    const SlowParams sp = slow_params(seed, o.replica, p);
    if (!h->ok(dev_alloc(&h->d_clk, 1))) return NASCH_ENOMEM;
    const Clock c0{0u, 0u};
    if (!h->ok(hipMemcpyAsync(h->d_clk, &c0, sizeof(Clock), hipMemcpyHostToDevice, h->stream)))
        return NASCH_EDEVICE;

    // initial grid (both representations start from it)
    uint8_t* g0 = nullptr;
    if (!h->ok(dev_alloc(&h->grid[0], L))) return NASCH_ENOMEM;
    g0 = h->grid[0];
    {
        // the placement's round-function table, for the init only (stream-ordered)
        uint32_t* tab = nullptr;
        const size_t tb = init_tab_words(feistel_bits(L)) * sizeof(uint32_t);
        if (!h->ok(hipMallocAsync((void**)&tab, tb, h->stream))) return NASCH_ENOMEM;
        const bool placed =
            h->ok(launch_init_grid(g0, (uint32_t)L, (uint32_t)N, vmax, o.init_v, sp, h->stream, tab));
        const bool freed = h->ok(hipFreeAsync(tab, h->stream));
        if (!placed || !freed) return NASCH_EDEVICE;
    }
    h->dev_bytes += L;

    if (o.rep == NASCH_REP_GRID) {
        const uint64_t pw = (uint64_t)(vmax + 1) * plane_words(L);
        if (!h->ok(dev_alloc(&h->grid[1], L)) || !h->ok(dev_alloc(&h->planes[0], pw)) ||
            !h->ok(dev_alloc(&h->planes[1], pw)))
            return NASCH_ENOMEM;
        h->dev_bytes += L + 8 * pw;
        RingDesc r{};
        r.buf[0] = h->grid[0];
        r.buf[1] = h->grid[1];
        r.pl[0] = h->planes[0];
        r.pl[1] = h->planes[1];
        r.nw = plane_words(L);
        r.L = (uint32_t)L;
        r.vmax = vmax;
        r.sp = sp;
        r.t_end = 0xFFFFFFFFu;
        r.warmup = ~0ull;
        if (open) {
            // gate thresholds floor(alpha 2^32), floor(beta 2^32): exact in binary64
            r.open = 1u;
            r.thr_in = (uint64_t)std::floor(std::ldexp(o.alpha, 32));
            r.thr_out = (uint64_t)std::floor(std::ldexp(o.beta, 32));
        }
        h->eng.rings.push_back(r);
        h->eng1.rings.push_back(r);
        h->eng1.onestep = true;
        if (!h->ok(h->eng1.set_geometry(1, kOneStepQ, h->stream))) return NASCH_EDEVICE;
        uint32_t kk = o.k, qq = o.q;
        uint32_t dk, dq;
        default_tuning((uint32_t)L, vmax, &dk, &dq);
        if (!qq) qq = dq;
        if (!kk) kk = std::min(dk, std::max(1u, kstep_max_k(vmax, qq)));
        h->k = kk; h->q = qq;
        uint32_t kern = o.kernel == NASCH_KERNEL_AUTO ? NASCH_KERNEL_KSTEP : o.kernel;
        // geometry of the k-step kernel is needed even when starting one-step
        uint32_t ow, ha, nt;
        if (!kstep_geometry((uint32_t)L, vmax, kk, qq, &ow, &ha, &nt)) return NASCH_EINVAL;
        if (!h->ok(h->eng.set_geometry(kk, qq, h->stream))) return NASCH_EDEVICE;
        h->kernel = kern;
    } else {
        if (!h->ok(dev_alloc(&h->ax[0], N)) || !h->ok(dev_alloc(&h->ax[1], N)) ||
            !h->ok(dev_alloc(&h->av[0], N)) || !h->ok(dev_alloc(&h->av[1], N)) ||
            !h->ok(dev_alloc(&h->d_agent, 1)))
            return NASCH_ENOMEM;
        h->agent_grid = g0;  // the init grid doubles as the snapshot scratch
        h->dev_bytes += 10 * N;
        AgentDesc& a = h->h_agent;
        a.x[0] = h->ax[0]; a.x[1] = h->ax[1];
        a.v[0] = h->av[0]; a.v[1] = h->av[1];
        a.N = (uint32_t)N; a.L = (uint32_t)L; a.vmax = vmax;
        a.sp = sp;
        a.warmup = ~0ull;
        a.rng = o.rng;
        h->rng = o.rng;
        if (o.rng == NASCH_RNG_STREAM) {
            // stream constants: x0, threshold, a^N and its inverse, jump table
            auto mpow = [](uint32_t b, uint64_t e) {
                uint32_t r = 1u;
                while (e) {
                    if (e & 1u) r = mlcg_mul(r, b);
                    b = mlcg_mul(b, b);
                    e >>= 1;
                }
                return r;
            };
            a.mlcg_x0 = (uint32_t)(seed % kMlcgM);
            if (!a.mlcg_x0) a.mlcg_x0 = 1u;
            a.mlcg_thr = (uint32_t)std::ceil(p * 2147483647.0);
            a.mlcg_aN = mpow(kMlcgA, N);
            a.mlcg_inv_aN = mpow(a.mlcg_aN, kMlcgM - 2u);
            std::vector<uint32_t> tab(256);
            uint32_t base = kMlcgA;   // a^(16^j)
            for (int j = 0; j < 16; ++j) {
                tab[16 * j] = 1u;
                for (int d = 1; d < 16; ++d) tab[16 * j + d] = mlcg_mul(tab[16 * j + d - 1], base);
                base = mlcg_mul(tab[16 * j + 15], base);
            }
            if (!h->ok(dev_alloc(&h->mlcg_pow, 256))) return NASCH_ENOMEM;
            if (!h->ok(hipMemcpy(h->mlcg_pow, tab.data(), 256 * sizeof(uint32_t),
                                 hipMemcpyHostToDevice)))
                return NASCH_EDEVICE;
            a.mlcg_pow = h->mlcg_pow;
        }
        uint32_t kk = o.k ? o.k : kDefaultAgentK;
        // cars per lane: the shared stream draws no blocks, so it takes the most
        const uint32_t cpl =
            o.q ? o.q
                : (o.rng == NASCH_RNG_STREAM ? kAgentMaxCarsPerLane : agent_cars_per_lane(N, L));
        if (!agent_geometry((uint32_t)N, kk, cpl, &h->agent_own, &h->agent_ntiles) ||
            !agent_geometry((uint32_t)N, 1u, kAgentMaxCarsPerLane, &h->agent_own1,
                            &h->agent_ntiles1))
            return NASCH_EINVAL;
        h->agent_cpl = cpl;
        rc = h->ensure_os_partials(
            std::max((size_t)h->agent_ntiles * kk, 2u * (size_t)h->agent_ntiles1));
        if (rc) return rc;
        h->k = kk;
        h->q = cpl;
        h->kernel = o.kernel == NASCH_KERNEL_AUTO ? NASCH_KERNEL_KSTEP : o.kernel;
        rc = agent_from_grid(h.get(), g0);
        if (rc) return rc;
    }
    rc = h->ensure_log(1024);
    if (rc) return rc;
    rc = h->refresh_descs();
    if (rc) return rc;
    if (!h->ok(hipStreamSynchronize(h->stream))) return NASCH_EDEVICE;
    *out = h.release();
    return NASCH_OK;
}

int nasch_step_n(nasch_sim* h, uint64_t T) {
    if (!h) return NASCH_EINVAL;
    if (T == 0) return NASCH_OK;
    if (h->t + T > 0xFFFFFFFFull) return NASCH_ERANGE;
    int rc = h->ensure_log(T);
    if (rc) return rc;
    return h->enqueue_steps(T);
}

int nasch_reserve_log(nasch_sim* h, uint64_t steps) {
    if (!h) return NASCH_EINVAL;
    if (h->t + steps > 0xFFFFFFFFull) return NASCH_ERANGE;
    return h->ensure_log(steps);
}

int nasch_timed_step_n(nasch_sim* h, uint64_t T, double* ms) {
    if (!h) return NASCH_EINVAL;
    if (h->t + T > 0xFFFFFFFFull) return NASCH_ERANGE;
    int rc = h->ensure_log(T);
    if (rc) return rc;
    hipEvent_t a = nullptr, b = nullptr;
    if (!h->ok(hipEventCreate(&a)) || !h->ok(hipEventCreate(&b))) return NASCH_EDEVICE;
    rc = NASCH_OK;
    if (!h->ok(hipEventRecord(a, h->stream))) rc = NASCH_EDEVICE;
    if (!rc && T) rc = h->enqueue_steps(T);
    if (!rc && !h->ok(hipEventRecord(b, h->stream))) rc = NASCH_EDEVICE;
    if (!rc && !h->ok(hipEventSynchronize(b))) rc = NASCH_EDEVICE;
    float f = 0;
    if (!rc && !h->ok(hipEventElapsedTime(&f, a, b))) rc = NASCH_EDEVICE;
    if (ms) *ms = f;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return rc;
}

int nasch_flux(nasch_sim* h, uint64_t t0, uint64_t count, uint64_t* out) {
    if (!h || (count && !out)) return NASCH_EINVAL;
    if (t0 < h->log_t0 || t0 + count > h->t) return NASCH_EINVAL;
    if (count == 0) return NASCH_OK;
    if (!h->ok(hipMemcpyAsync(out, h->flux + (t0 - h->log_t0), count * sizeof(uint64_t),
                              hipMemcpyDeviceToHost, h->stream)) ||
        !h->ok(hipStreamSynchronize(h->stream)))
        return NASCH_EDEVICE;
    return NASCH_OK;
}

int nasch_snapshot_range(nasch_sim* h, uint64_t start, uint64_t len, uint8_t* out) {
    if (!h || (len && !out)) return NASCH_EINVAL;
    if (len == 0) return NASCH_OK;
    const uint8_t* g = h->current_grid_device();
    if (!g) return NASCH_EDEVICE;
    uint64_t done = 0;
    uint64_t pos = start % h->L;
    while (done < len) {
        const uint64_t n = std::min(len - done, h->L - pos);
        if (!h->ok(hipMemcpyAsync(out + done, g + pos, n, hipMemcpyDeviceToHost, h->stream)))
            return NASCH_EDEVICE;
        done += n;
        pos = 0;
    }
    if (!h->ok(hipStreamSynchronize(h->stream))) return NASCH_EDEVICE;
    return NASCH_OK;
}

int nasch_snapshot(nasch_sim* h, uint8_t* out, uint64_t* t_out) {
    if (!h) return NASCH_EINVAL;
    if (out) {
        int rc = nasch_snapshot_range(h, 0, h->L, out);
        if (rc) return rc;
    }
    if (t_out) *t_out = h->t;
    return NASCH_OK;
}

int nasch_agent_state(nasch_sim* h, int32_t* x, uint8_t* v) {
    if (!h) return NASCH_EINVAL;
    if (h->rep != NASCH_REP_AGENT) return NASCH_ESTATE;
    if (x && h->N &&
        !h->ok(hipMemcpyAsync(x, h->ax[h->parity], h->N * sizeof(int32_t), hipMemcpyDeviceToHost,
                              h->stream)))
        return NASCH_EDEVICE;
    if (v && h->N &&
        !h->ok(hipMemcpyAsync(v, h->av[h->parity], h->N, hipMemcpyDeviceToHost, h->stream)))
        return NASCH_EDEVICE;
    if (!h->ok(hipStreamSynchronize(h->stream))) return NASCH_EDEVICE;
    return NASCH_OK;
}

int nasch_restore(nasch_sim* h, const uint8_t* grid, uint64_t t) {
    if (!h || !grid) return NASCH_EINVAL;
    if (t > 0xFFFFFFFFull) return NASCH_ERANGE;
    uint64_t cars = 0;
    for (uint64_t i = 0; i < h->L; ++i) {
        if (grid[i] == 0xFF) continue;
        if (grid[i] > h->vmax) return NASCH_EINVAL;
        ++cars;
    }
    if (!h->open && cars != h->N) return NASCH_EINVAL;   // an open road changes its car count
    if (!h->ok(hipStreamSynchronize(h->stream))) return NASCH_EDEVICE;
    h->parity = 0;
    h->t = t;
    h->bytes_ok = true;    // the restored bytes go to grid[0]; the planes follow on demand
    h->planes_ok = false;
    const Clock c{(uint32_t)t, 0u};
    if (!h->ok(hipMemcpyAsync(h->d_clk, &c, sizeof(Clock), hipMemcpyHostToDevice, h->stream)))
        return NASCH_EDEVICE;
    uint8_t* g = h->rep == NASCH_REP_GRID ? h->grid[0] : h->agent_grid;
    if (!h->ok(hipMemcpyAsync(g, grid, h->L, hipMemcpyHostToDevice, h->stream)) ||
        !h->ok(hipStreamSynchronize(h->stream)))
        return NASCH_EDEVICE;
    if (h->rep == NASCH_REP_AGENT) {
        int rc = agent_from_grid(h, g);
        if (rc) return rc;
    }
    // forget the old flux log
    h->log_t0 = t;
    if (h->flux && !h->ok(launch_fill_u64(h->flux, h->flux_cap, h->stream))) return NASCH_EDEVICE;
    int rc = h->refresh_descs();
    if (rc) return rc;
    return NASCH_OK;
}

int nasch_restore_agent(nasch_sim* h, const int32_t* x, const uint8_t* v, uint64_t t) {
    if (!h || (h->N && (!x || !v))) return NASCH_EINVAL;
    if (h->rep != NASCH_REP_AGENT) return NASCH_ESTATE;
    if (t > 0xFFFFFFFFull) return NASCH_ERANGE;
    uint64_t descents = 0;
    std::vector<uint8_t> seen(h->L, 0);
    for (uint64_t i = 0; i < h->N; ++i) {
        if (x[i] < 0 || (uint64_t)x[i] >= h->L || v[i] > h->vmax || seen[x[i]]) return NASCH_EINVAL;
        seen[x[i]] = 1;
        if (i + 1 < h->N && x[i + 1] < x[i]) ++descents;
    }
    if (descents > 1) return NASCH_EINVAL;
    if (!h->ok(hipStreamSynchronize(h->stream))) return NASCH_EDEVICE;
    h->parity = 0;
    h->t = t;
    const Clock c{(uint32_t)t, 0u};
    if (!h->ok(hipMemcpyAsync(h->d_clk, &c, sizeof(Clock), hipMemcpyHostToDevice, h->stream)))
        return NASCH_EDEVICE;
    if (h->N && (!h->ok(hipMemcpyAsync(h->ax[0], x, h->N * sizeof(int32_t), hipMemcpyHostToDevice,
                                       h->stream)) ||
                 !h->ok(hipMemcpyAsync(h->av[0], v, h->N, hipMemcpyHostToDevice, h->stream))))
        return NASCH_EDEVICE;
    if (!h->ok(hipStreamSynchronize(h->stream))) return NASCH_EDEVICE;
    h->log_t0 = t;
    if (h->flux && !h->ok(launch_fill_u64(h->flux, h->flux_cap, h->stream))) return NASCH_EDEVICE;
    return h->refresh_descs();
}

int nasch_writer_frame(nasch_writer* w, nasch_sim* h) {
    if (!w || !h) return NASCH_EINVAL;
    if (nasch_writer_length(w) != h->L) return NASCH_EINVAL;
    const uint8_t* g = h->current_grid_device();
    if (!g) return NASCH_EDEVICE;
    return nasch_writer_enqueue_device(w, g, h->t, h->stream);
}

int nasch_set_tuning(nasch_sim* h, uint32_t kernel, uint32_t k, uint32_t q) {
    if (!h) return NASCH_EINVAL;
    return h->set_tuning(kernel, k, q);
}

int nasch_get_info(const nasch_sim* h, nasch_info* info) {
    if (!h || !info) return NASCH_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->L = h->L; info->N = h->N; info->t = h->t;
    info->vmax = h->vmax; info->thr = h->thr; info->replica = h->replica; info->rep = h->rep;
    info->init_v = h->init_v; info->kernel = h->kernel; info->k = h->k; info->q = h->q;
    info->seed = h->seed;
    info->device_bytes = h->dev_bytes;
    return NASCH_OK;
}

int nasch_last_device_error(const nasch_sim* h) { return h ? h->st.err : 0; }

int nasch_thread_last_device_error(void) { return thread_last_hip_error(); }

void nasch_free(nasch_sim* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    delete h;
}

}  // extern "C"

extern "C" int nasch_autotune(nasch_sim* h) {
    if (!h) return NASCH_EINVAL;
    if (h->rep == NASCH_REP_GRID) {
        uint32_t bk = 0, bq = 0;
        double cups = 0;
        RingDesc cur = h->eng.rings[0];
        std::vector<RingDesc> rs{cur};
        if (!h->need_planes() || !h->ok(hipStreamSynchronize(h->stream))) return NASCH_EDEVICE;
        if (!h->ok(autotune_grid(rs, (uint32_t)h->t, h->parity, 256, h->stream, &bk, &bq, &cups)))
            return NASCH_EDEVICE;
        if (!bk) return NASCH_EINVAL;
        return h->set_tuning(NASCH_KERNEL_KSTEP, bk, bq);
    }
    // agent representation: time k on the real state, then put it back
    if (!h->ok(hipStreamSynchronize(h->stream))) return NASCH_EDEVICE;
    std::vector<uint8_t> snap(h->L);
    const uint64_t t0 = h->t;
    int rc = nasch_snapshot(h, snap.data(), nullptr);
    if (rc) return rc;
    const uint32_t ks[] = {8, 16, 32, 64, 128};
    uint32_t best_k = h->k;
    double best = 0;
    for (uint32_t kk : ks) {
        if (h->set_tuning(NASCH_KERNEL_KSTEP, kk, 0) != NASCH_OK) continue;
        const uint64_t T = std::max<uint64_t>(256, kk) / kk * kk;
        if (t0 + 2 * T > 0xFFFFFFFFull) break;
        double ms = 0;
        rc = nasch_step_n(h, kk);
        if (!rc) rc = nasch_timed_step_n(h, T, &ms);
        if (rc) return rc;
        if (ms > 0 && (double)T / ms > best) {
            best = (double)T / ms;
            best_k = kk;
        }
        rc = nasch_restore(h, snap.data(), t0);
        if (rc) return rc;
    }
    return h->set_tuning(NASCH_KERNEL_KSTEP, best_k, 0);
}
