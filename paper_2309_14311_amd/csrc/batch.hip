// batch.hip -- the batched ensemble: many independent rings in one device arena,
// advanced together by the temporal-blocked grid kernel (all rings' tiles in
// the same launches).  Entry points are documented in include/nasch.h.
//
// Each replica holds one byte grid (the initial placement and snapshots) and
// two bit-plane buffers (the state the kernel steps), 256-byte aligned.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "engine.hpp"
#include "nasch.h"

using namespace nasch;

struct nasch_batch {
    std::vector<nasch_replica> reps;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    HipStatus st;
    uint8_t* arena = nullptr;
    uint64_t arena_bytes = 0;
    unsigned long long* d_acc = nullptr;   // per replica: sum of F(t), t >= warmup
    unsigned long long* d_log = nullptr;   // per replica x log_steps: F(t)
    uint64_t log_steps = 0;
    Clock* d_clk = nullptr;
    uint64_t t = 0;
    uint32_t parity = 0;
    uint32_t use_graph = 0;
    GridEngine eng;
    GraphCache graphs;
    InitRing* d_init_rings = nullptr;     // placement of every replica, one launch
    InitChunk* d_init_chunks = nullptr;
    uint32_t n_init_chunks = 0;
    uint32_t* d_init_tabs = nullptr;      // every replica's placement round-function table
    ConvJob* d_conv_jobs = nullptr;       // byte grid -> planes pl[0] of every replica
    ConvChunk* d_conv_chunks = nullptr;
    uint32_t n_conv_chunks = 0;

    bool ok(hipError_t e) { return st.ok(e); }
    // Every replica at t = 0: the whole arena EMPTY, all cars scattered into
    // the byte grids, then the grids turned into bit planes.
    bool init_state() {
        return ok(launch_fill_u8(arena, arena_bytes, 0xFFu, stream)) &&
               ok(launch_init_scatter(d_init_rings, d_init_chunks, n_init_chunks, stream)) &&
               ok(launch_bytes_to_planes(d_conv_jobs, d_conv_chunks, n_conv_chunks, stream));
    }
    ~nasch_batch() {
        graphs.clear();
        eng.release();
        void* ps[] = {arena, d_acc, d_log, d_clk, d_init_rings, d_init_chunks, d_conv_jobs,
                      d_conv_chunks, d_init_tabs};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
        (void)hipGetLastError();
    }
    int enqueue(uint64_t T) {
        if (t + T > 0xFFFFFFFFull) return NASCH_ERANGE;
        if (d_log && t + T > log_steps) return NASCH_ERANGE;
        if (T == 0) return NASCH_OK;
        auto body = [&]() -> hipError_t {
            hipError_t e = eng.enqueue(T, d_clk, stream);
            if (e != hipSuccess) return e;
            return launch_clock_advance(d_clk, (uint32_t)T, eng.launches_for(T), stream);
        };
        hipError_t e = use_graph
                           ? graphs.run(std::make_tuple(T, 0u, eng.k, eng.q, eng.version), stream, body)
                           : body();
        if (!ok(e)) return NASCH_EDEVICE;
        t += T;
        parity ^= eng.launches_for(T) & 1u;
        return NASCH_OK;
    }
};

extern "C" {

void nasch_batch_default_opts(nasch_batch_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
}

int nasch_batch_init(nasch_batch** out, const nasch_replica* reps, uint32_t R,
                     const nasch_batch_opts* opts) {
    if (!out) return NASCH_EINVAL;
    *out = nullptr;
    if (!reps || R == 0) return NASCH_EINVAL;
    nasch_batch_opts o;
    nasch_batch_default_opts(&o);
    if (opts) o = *opts;
    if (o.keep_log && o.log_steps == 0) return NASCH_EINVAL;
    for (uint32_t r = 0; r < R; ++r) {
        const nasch_replica& p = reps[r];
        int rc = validate_params(p.L, p.N, p.vmax, p.p);
        if (rc) return rc;
        if (p.init_v > NASCH_INIT_V_UNIFORM || p.reserved || p.reserved2 ||
            p.boundary > NASCH_BOUNDARY_OPEN || p.boundary != reps[0].boundary)
            return NASCH_EINVAL;
        // gate probabilities in [0, 1] (NaN fails both comparisons)
        if (p.boundary == NASCH_BOUNDARY_OPEN &&
            !(p.alpha >= 0.0 && p.alpha <= 1.0 && p.beta >= 0.0 && p.beta <= 1.0))
            return NASCH_EINVAL;
    }
    std::unique_ptr<nasch_batch> b(new (std::nothrow) nasch_batch());
    if (!b) return NASCH_ENOMEM;
    b->reps.assign(reps, reps + R);
    b->use_graph = o.use_graph;
    if (o.stream) {
        b->stream = (hipStream_t)o.stream;
    } else {
        if (!b->ok(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking))) return NASCH_EDEVICE;
        b->own_stream = true;
    }
    std::vector<uint64_t> offs(R);
    uint64_t bytes = 0;
    auto grid_bytes = [](const nasch_replica& p) { return (p.L + 255) / 256 * 256; };
    auto plane_bytes = [](const nasch_replica& p) {
        return ((uint64_t)(p.vmax + 1) * plane_words(p.L) * 4u + 255) / 256 * 256;
    };
    for (uint32_t r = 0; r < R; ++r) {
        offs[r] = bytes;
        bytes += grid_bytes(reps[r]) + 2 * plane_bytes(reps[r]);
    }
    b->arena_bytes = bytes;
    if (!b->ok(dev_alloc(&b->arena, bytes)) || !b->ok(dev_alloc(&b->d_acc, R)) ||
        !b->ok(dev_alloc(&b->d_clk, 1)))
        return NASCH_ENOMEM;
    if (!b->ok(launch_fill_u64(b->d_acc, R, b->stream))) return NASCH_EDEVICE;
    if (o.keep_log) {
        b->log_steps = o.log_steps;
        if (!b->ok(dev_alloc(&b->d_log, (uint64_t)R * o.log_steps))) return NASCH_ENOMEM;
        if (!b->ok(launch_fill_u64(b->d_log, (uint64_t)R * o.log_steps, b->stream)))
            return NASCH_EDEVICE;
    }
    const Clock c0{0u, 0u};
    if (!b->ok(hipMemcpyAsync(b->d_clk, &c0, sizeof(Clock), hipMemcpyHostToDevice, b->stream)))
        return NASCH_EDEVICE;
    uint32_t vmax_all = 0;
    // the placement tables (filled once: they depend on L, seed and replica only)
    uint64_t tab_words = 0;
    for (uint32_t r = 0; r < R; ++r) tab_words += init_tab_words(feistel_bits(reps[r].L));
    if (!b->ok(dev_alloc(&b->d_init_tabs, tab_words))) return NASCH_ENOMEM;
    uint64_t tab_off = 0;
    std::vector<InitChunk> tab_chunks;
    std::vector<InitRing> init_rings;
    std::vector<InitChunk> init_chunks;
    std::vector<ConvJob> conv_jobs;
    std::vector<ConvChunk> conv_chunks;
    for (uint32_t r = 0; r < R; ++r) {
        const nasch_replica& p = reps[r];
        const uint64_t sz = grid_bytes(p), psz = plane_bytes(p);
        RingDesc d{};
        d.buf[0] = b->arena + offs[r];
        d.buf[1] = nullptr;
        d.pl[0] = reinterpret_cast<uint32_t*>(b->arena + offs[r] + sz);
        d.pl[1] = reinterpret_cast<uint32_t*>(b->arena + offs[r] + sz + psz);
        d.nw = plane_words(p.L);
        d.flux_log = b->d_log ? b->d_log + (uint64_t)r * b->log_steps : nullptr;
        d.flux_acc = b->d_acc + r;
        d.log_t0 = 0;
        d.warmup = p.warmup;
        d.L = (uint32_t)p.L;
        d.vmax = p.vmax;
        d.t_end = 0xFFFFFFFFu;
        d.sp = slow_params(p.seed, p.replica, p.p);
        if (p.boundary == NASCH_BOUNDARY_OPEN) {
            d.open = 1u;
            d.thr_in = (uint64_t)std::floor(std::ldexp(p.alpha, 32));
            d.thr_out = (uint64_t)std::floor(std::ldexp(p.beta, 32));
        }
        b->eng.rings.push_back(d);
        vmax_all = std::max(vmax_all, p.vmax);
        const uint32_t fb = feistel_bits(p.L);
        init_rings.push_back(InitRing{d.buf[0], (uint32_t)p.L, (uint32_t)p.N, p.vmax, p.init_v,
                                      fb, 0u, d.sp, b->d_init_tabs + tab_off});
        for (uint64_t e = 0; e < init_tab_words(fb); e += 256) tab_chunks.push_back(InitChunk{r, (uint32_t)e});
        tab_off += init_tab_words(fb);
        for (uint64_t c = 0; c < p.N; c += kInitChunk) init_chunks.push_back(InitChunk{r, (uint32_t)c});
        conv_jobs.push_back(ConvJob{d.buf[0], d.pl[0], d.L, d.nw, d.vmax, 0u});
        for (uint32_t w = 0; w < d.nw; w += kConvChunk) conv_chunks.push_back(ConvChunk{r, w});
    }
    b->n_init_chunks = (uint32_t)init_chunks.size();
    b->n_conv_chunks = (uint32_t)conv_chunks.size();
    if (!b->ok(dev_alloc(&b->d_init_rings, R)) ||
        !b->ok(dev_alloc(&b->d_init_chunks, init_chunks.size())) ||
        !b->ok(dev_alloc(&b->d_conv_jobs, R)) ||
        !b->ok(dev_alloc(&b->d_conv_chunks, conv_chunks.size())))
        return NASCH_ENOMEM;
    if (!b->ok(hipMemcpy(b->d_conv_jobs, conv_jobs.data(), R * sizeof(ConvJob),
                         hipMemcpyHostToDevice)) ||
        !b->ok(hipMemcpy(b->d_conv_chunks, conv_chunks.data(),
                         conv_chunks.size() * sizeof(ConvChunk), hipMemcpyHostToDevice)))
        return NASCH_EDEVICE;
    if (!b->ok(hipMemcpy(b->d_init_rings, init_rings.data(), R * sizeof(InitRing),
                         hipMemcpyHostToDevice)) ||
        (!init_chunks.empty() &&
         !b->ok(hipMemcpy(b->d_init_chunks, init_chunks.data(),
                          init_chunks.size() * sizeof(InitChunk), hipMemcpyHostToDevice))))
        return NASCH_EDEVICE;
    {
        InitChunk* d_tab_chunks = nullptr;
        if (!b->ok(dev_alloc(&d_tab_chunks, tab_chunks.size()))) return NASCH_ENOMEM;
        const bool filled =
            b->ok(hipMemcpy(d_tab_chunks, tab_chunks.data(), tab_chunks.size() * sizeof(InitChunk),
                            hipMemcpyHostToDevice)) &&
            b->ok(launch_init_tables(b->d_init_rings, d_tab_chunks, (uint32_t)tab_chunks.size(),
                                     b->stream)) &&
            b->ok(hipStreamSynchronize(b->stream));
        (void)hipFree(d_tab_chunks);
        if (!filled) return NASCH_EDEVICE;
    }
    if (!b->init_state()) return NASCH_EDEVICE;
    uint32_t q = o.q ? o.q : 4u;
    uint32_t k = o.k ? o.k : std::min(32u, std::max(1u, kstep_max_k(vmax_all, q)));
    if (!b->eng.geometry_ok(k, q)) return NASCH_EINVAL;
    if (!b->ok(b->eng.set_geometry(k, q, b->stream))) return NASCH_EDEVICE;
    if (!b->ok(hipStreamSynchronize(b->stream))) return NASCH_EDEVICE;
    *out = b.release();
    return NASCH_OK;
}

int nasch_batch_reset(nasch_batch* b) {
    if (!b) return NASCH_EINVAL;
    const uint32_t R = (uint32_t)b->reps.size();
    if (!b->init_state()) return NASCH_EDEVICE;
    if (!b->ok(launch_fill_u64(b->d_acc, R, b->stream))) return NASCH_EDEVICE;
    if (b->d_log && !b->ok(launch_fill_u64(b->d_log, (uint64_t)R * b->log_steps, b->stream)))
        return NASCH_EDEVICE;
    const Clock c0{0u, 0u};
    if (!b->ok(hipMemcpyAsync(b->d_clk, &c0, sizeof(Clock), hipMemcpyHostToDevice, b->stream)) ||
        !b->ok(hipStreamSynchronize(b->stream)))
        return NASCH_EDEVICE;
    b->t = 0;
    b->parity = 0;
    return NASCH_OK;
}

int nasch_batch_step_n(nasch_batch* b, uint64_t T) {
    if (!b) return NASCH_EINVAL;
    return b->enqueue(T);
}

int nasch_batch_timed_step_n(nasch_batch* b, uint64_t T, double* ms) {
    if (!b) return NASCH_EINVAL;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!b->ok(hipEventCreate(&e0)) || !b->ok(hipEventCreate(&e1))) return NASCH_EDEVICE;
    int rc = NASCH_OK;
    if (!b->ok(hipEventRecord(e0, b->stream))) rc = NASCH_EDEVICE;
    if (!rc) rc = b->enqueue(T);
    if (!rc && !b->ok(hipEventRecord(e1, b->stream))) rc = NASCH_EDEVICE;
    if (!rc && !b->ok(hipEventSynchronize(e1))) rc = NASCH_EDEVICE;
    float f = 0;
    if (!rc && !b->ok(hipEventElapsedTime(&f, e0, e1))) rc = NASCH_EDEVICE;
    if (ms) *ms = f;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int nasch_batch_flux_sums(nasch_batch* b, uint64_t* out) {
    if (!b || !out) return NASCH_EINVAL;
    if (!b->ok(hipMemcpyAsync(out, b->d_acc, b->reps.size() * sizeof(uint64_t),
                              hipMemcpyDeviceToHost, b->stream)) ||
        !b->ok(hipStreamSynchronize(b->stream)))
        return NASCH_EDEVICE;
    return NASCH_OK;
}

int nasch_batch_flux(nasch_batch* b, uint32_t r, uint64_t t0, uint64_t count, uint64_t* out) {
    if (!b || (count && !out)) return NASCH_EINVAL;
    if (r >= b->reps.size()) return NASCH_ENOTFOUND;
    if (!b->d_log) return NASCH_ESTATE;
    if (t0 + count > b->t) return NASCH_EINVAL;
    if (count == 0) return NASCH_OK;
    if (!b->ok(hipMemcpyAsync(out, b->d_log + (uint64_t)r * b->log_steps + t0,
                              count * sizeof(uint64_t), hipMemcpyDeviceToHost, b->stream)) ||
        !b->ok(hipStreamSynchronize(b->stream)))
        return NASCH_EDEVICE;
    return NASCH_OK;
}

int nasch_batch_snapshot(nasch_batch* b, uint32_t r, uint8_t* out, uint64_t* t_out) {
    if (!b) return NASCH_EINVAL;
    if (r >= b->reps.size()) return NASCH_ENOTFOUND;
    if (out) {
        // the replica's planes into its byte grid, then to the host
        const RingDesc& d = b->eng.rings[r];
        const ConvJob job{d.buf[0], d.pl[b->parity], d.L, d.nw, d.vmax, 0u};
        if (!b->ok(launch_planes_to_bytes_one(job, b->stream)) ||
            !b->ok(hipMemcpyAsync(out, d.buf[0], d.L, hipMemcpyDeviceToHost, b->stream)) ||
            !b->ok(hipStreamSynchronize(b->stream)))
            return NASCH_EDEVICE;
    }
    if (t_out) *t_out = b->t;
    return NASCH_OK;
}

// The checkpoint of a batch as the caller sees it is every replica's grid back
// to back.  On the device each replica gets a 256-byte aligned slice of a
// staging buffer instead (the conversion kernels move whole words with 16-byte
// accesses), and the host packs or unpacks the two layouts.
static uint64_t staged_bytes(const nasch_batch* b, std::vector<uint64_t>& offs) {
    uint64_t off = 0;
    offs.clear();
    for (const RingDesc& d : b->eng.rings) {
        offs.push_back(off);
        off += ((uint64_t)d.L + 255u) / 256u * 256u;
    }
    return off;
}

// Convert every replica between its planes pl[parity] and its staging slice,
// with a temporary device copy of the job table.
static int convert_staged(nasch_batch* b, uint8_t* d_stage, const std::vector<uint64_t>& offs,
                          uint32_t parity, bool to_planes) {
    std::vector<ConvJob> jobs;
    for (size_t r = 0; r < b->eng.rings.size(); ++r) {
        const RingDesc& d = b->eng.rings[r];
        jobs.push_back(ConvJob{d_stage + offs[r], d.pl[parity], d.L, d.nw, d.vmax, 0u});
    }
    ConvJob* d_jobs = nullptr;
    if (!b->ok(dev_alloc(&d_jobs, jobs.size()))) return NASCH_ENOMEM;
    int rc = NASCH_OK;
    if (!b->ok(hipMemcpyAsync(d_jobs, jobs.data(), jobs.size() * sizeof(ConvJob),
                              hipMemcpyHostToDevice, b->stream)) ||
        !b->ok(to_planes ? launch_bytes_to_planes(d_jobs, b->d_conv_chunks, b->n_conv_chunks,
                                                  b->stream)
                         : launch_planes_to_bytes(d_jobs, b->d_conv_chunks, b->n_conv_chunks,
                                                  b->stream)) ||
        !b->ok(hipStreamSynchronize(b->stream)))
        rc = NASCH_EDEVICE;
    (void)hipFree(d_jobs);
    return rc;
}

int nasch_batch_snapshot_all(nasch_batch* b, uint8_t* out, uint64_t* t_out) {
    if (!b || !out) return NASCH_EINVAL;
    std::vector<uint64_t> offs;
    const uint64_t staged = staged_bytes(b, offs);
    std::vector<uint8_t> host;
    uint8_t* d_stage = nullptr;
    if (!b->ok(hipStreamSynchronize(b->stream))) return NASCH_EDEVICE;
    try {
        host.resize(staged);
    } catch (const std::bad_alloc&) {
        return NASCH_ENOMEM;
    }
    if (!b->ok(dev_alloc(&d_stage, staged))) return NASCH_ENOMEM;
    int rc = convert_staged(b, d_stage, offs, b->parity, false);
    if (!rc && !b->ok(hipMemcpy(host.data(), d_stage, staged, hipMemcpyDeviceToHost)))
        rc = NASCH_EDEVICE;
    (void)hipFree(d_stage);
    if (rc) return rc;
    uint64_t pos = 0;
    for (size_t r = 0; r < b->eng.rings.size(); ++r) {
        std::memcpy(out + pos, host.data() + offs[r], b->eng.rings[r].L);
        pos += b->eng.rings[r].L;
    }
    if (t_out) *t_out = b->t;
    return NASCH_OK;
}

int nasch_batch_restore(nasch_batch* b, const uint8_t* grids, uint64_t t) {
    if (!b || !grids) return NASCH_EINVAL;
    if (t > 0xFFFFFFFFull) return NASCH_ERANGE;
    // validate everything before touching the device state
    uint64_t pos = 0;
    for (const nasch_replica& p : b->reps) {
        uint64_t cars = 0;
        for (uint64_t i = 0; i < p.L; ++i) {
            const uint8_t c = grids[pos + i];
            if (c == 0xFFu) continue;
            if (c > p.vmax) return NASCH_EINVAL;
            ++cars;
        }
        if (p.boundary != NASCH_BOUNDARY_OPEN && cars != p.N) return NASCH_EINVAL;
        pos += p.L;
    }
    std::vector<uint64_t> offs;
    const uint64_t staged = staged_bytes(b, offs);
    std::vector<uint8_t> host;
    try {
        host.assign(staged, 0xFFu);
    } catch (const std::bad_alloc&) {
        return NASCH_ENOMEM;
    }
    pos = 0;
    for (size_t r = 0; r < b->eng.rings.size(); ++r) {
        std::memcpy(host.data() + offs[r], grids + pos, b->eng.rings[r].L);
        pos += b->eng.rings[r].L;
    }
    const uint32_t R = (uint32_t)b->reps.size();
    uint8_t* d_stage = nullptr;
    if (!b->ok(hipStreamSynchronize(b->stream))) return NASCH_EDEVICE;
    if (!b->ok(dev_alloc(&d_stage, staged))) return NASCH_ENOMEM;
    int rc = NASCH_OK;
    if (!b->ok(hipMemcpy(d_stage, host.data(), staged, hipMemcpyHostToDevice))) rc = NASCH_EDEVICE;
    if (!rc) rc = convert_staged(b, d_stage, offs, 0u, true);
    (void)hipFree(d_stage);
    if (rc) return rc;
    const Clock c{(uint32_t)t, 0u};
    if (!b->ok(launch_fill_u64(b->d_acc, R, b->stream)) ||
        (b->d_log && !b->ok(launch_fill_u64(b->d_log, (uint64_t)R * b->log_steps, b->stream))) ||
        !b->ok(hipMemcpyAsync(b->d_clk, &c, sizeof(Clock), hipMemcpyHostToDevice, b->stream)) ||
        !b->ok(hipStreamSynchronize(b->stream)))
        return NASCH_EDEVICE;
    b->t = t;
    b->parity = 0;
    return NASCH_OK;
}

int nasch_batch_set_tuning(nasch_batch* b, uint32_t k, uint32_t q) {
    if (!b) return NASCH_EINVAL;
    if (k == 0) k = b->eng.k;
    if (q == 0) q = b->eng.q;
    if (!b->eng.geometry_ok(k, q)) return NASCH_EINVAL;
    if (k == b->eng.k && q == b->eng.q) return NASCH_OK;
    if (!b->ok(hipStreamSynchronize(b->stream))) return NASCH_EDEVICE;
    if (!b->ok(b->eng.set_geometry(k, q, b->stream))) return NASCH_EDEVICE;
    b->graphs.clear();
    return NASCH_OK;
}

int nasch_batch_autotune(nasch_batch* b, uint32_t* k_out, uint32_t* q_out) {
    if (!b) return NASCH_EINVAL;
    if (!b->ok(hipStreamSynchronize(b->stream))) return NASCH_EDEVICE;
    uint32_t bk = 0, bq = 0;
    double cups = 0;
    if (!b->ok(autotune_grid(b->eng.rings, (uint32_t)b->t, b->parity, 128, b->stream, &bk, &bq,
                             &cups)))
        return NASCH_EDEVICE;
    if (!bk) return NASCH_EINVAL;
    int rc = nasch_batch_set_tuning(b, bk, bq);
    if (rc) return rc;
    if (k_out) *k_out = bk;
    if (q_out) *q_out = bq;
    return NASCH_OK;
}

int nasch_batch_last_device_error(const nasch_batch* b) { return b ? b->st.err : 0; }

void nasch_batch_free(nasch_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
}

}  // extern "C"
