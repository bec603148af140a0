// server.hip -- serving loop: simulations submitted one by one and advanced on the
// GPU by continuous batching.  Entry points are documented in include/nasch.h.
//
// A scheduling thread owns the device.  Each iteration it
//   1. admits queued requests in arrival order while their footprint fits the
//      HBM budget and a slot is free (state allocated from a device arena,
//      initialised by the init kernel);
//   2. runs a burst of launches of the temporal-blocked grid kernel over every
//      live slot, each slot advancing from its own step counter (the burst
//      stops where the first slot finishes, and is a single launch while
//      requests wait for admission); the tile items are rebuilt only when
//      the set of live slots changes;
//   3. hands finished slots back: flux log and final grid are copied to the
//      caller's buffers, the result is queued for nasch_server_poll, and the
//      slot's memory is returned to the arena.
// A slot's results depend only on its own (L, N, vmax, p, seed, replica, T):
// the rule-3 draws are keyed by (seed, replica, t, x), never by the slot.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "engine.hpp"
#include "nasch.h"

using namespace nasch;

namespace {

// First-fit allocator over one device arena (offsets aligned to 256 bytes).
class Arena {
  public:
    void reset(uint64_t size) {
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    bool alloc(uint64_t n, uint64_t* off) {
        n = (n + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint64_t rest = it->second - n;
                const uint64_t start = it->first + n;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        n = (n + 255) / 256 * 256;
        used_ -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t used_ = 0;
};

struct Job {
    uint64_t id = 0;
    nasch_request req{};
    double t_submit = 0, t_admit = 0;
    uint64_t off = 0, bytes = 0;       // arena allocation
    uint32_t t = 0;                    // steps done
    uint32_t parity = 0;
    bool cancelled = false;
};

// Launches run back to back before the host looks at the slots again.
constexpr uint32_t kMaxBurst = 8;

// Layout of one slot: the byte grid (initial placement, final snapshot), two
// bit-plane buffers (the state the kernel steps), the flux log; each rounded
// up to 256 bytes.
uint64_t grid_bytes(const nasch_request& r) { return (r.L + 255) / 256 * 256; }
uint64_t plane_bytes(const nasch_request& r) {
    return ((uint64_t)(r.vmax + 1) * plane_words(r.L) * 4u + 255) / 256 * 256;
}
uint64_t footprint(const nasch_request& r) {
    return grid_bytes(r) + 2 * plane_bytes(r) + (8 * r.T + 255) / 256 * 256;
}
uint64_t log_offset(const nasch_request& r) { return grid_bytes(r) + 2 * plane_bytes(r); }

}  // namespace

struct nasch_server {
    nasch_server_opts opts{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    HipStatus st;
    uint8_t* arena_base = nullptr;
    Arena arena;
    Clock* d_clk = nullptr;   // stays {0, 0}: each slot carries its own t and parity
    GridEngine eng;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<Job>> pending;
    std::vector<std::unique_ptr<Job>> running;
    std::deque<nasch_result> done;
    std::vector<uint64_t> cancel_ids;
    uint64_t next_id = 1;
    uint64_t n_done = 0;
    // read by nasch_server_stats while the scheduling thread runs
    std::atomic<uint64_t> n_running{0}, launches{0};
    bool stop = false;
    std::thread worker;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void loop();
    enum class Admit { ok, no_room, device_error };
    Admit admit_one(Job& j);
    void finish(std::unique_ptr<Job> j, int status, uint64_t flux_sum);
};

nasch_server::Admit nasch_server::admit_one(Job& j) {
    const nasch_request& r = j.req;
    j.bytes = footprint(r);
    if (!arena.alloc(j.bytes, &j.off)) return Admit::no_room;
    uint8_t* base = arena_base + j.off;
    const SlowParams sp = slow_params(r.seed, r.replica, r.p);
    const ConvJob job{base, reinterpret_cast<uint32_t*>(base + grid_bytes(r)), (uint32_t)r.L,
                      plane_words(r.L), r.vmax, 0u};
    if (!st.ok(launch_init_grid(base, (uint32_t)r.L, (uint32_t)r.N, r.vmax, r.init_v, sp, stream)) ||
        !st.ok(launch_bytes_to_planes_one(job, stream)) ||
        !st.ok(launch_fill_u64(reinterpret_cast<unsigned long long*>(base + log_offset(r)), r.T,
                               stream))) {
        arena.release(j.off, j.bytes);
        j.bytes = 0;
        return Admit::device_error;
    }
    j.t = 0;
    j.parity = 0;
    j.t_admit = now();
    return Admit::ok;
}

void nasch_server::finish(std::unique_ptr<Job> j, int status, uint64_t flux_sum) {
    nasch_result res{};
    res.id = j->id;
    res.status = status;
    res.flux_sum = flux_sum;
    res.t_submit = j->t_submit;
    res.t_admit = j->t_admit;
    res.t_done = now();
    std::lock_guard<std::mutex> lk(mu);
    if (j->bytes) arena.release(j->off, j->bytes);
    done.push_back(res);
    ++n_done;
    cv_done.notify_all();
}

void nasch_server::loop() {
    const uint32_t k = opts.k, q = opts.q;
    std::vector<uint64_t> flux_host;
    bool dirty = true;   // the set of live slots changed: rebuild the tile items
    for (;;) {
        // ---- admission and cancellation
        std::vector<std::unique_ptr<Job>> admitted;
        std::vector<std::unique_ptr<Job>> cancelled_pending, failed;
        std::vector<uint64_t> cancels;
        bool waiting;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !pending.empty() || !running.empty() || !cancel_ids.empty(); });
            if (stop) return;
            cancels.swap(cancel_ids);
            for (uint64_t id : cancels) {
                for (auto it = pending.begin(); it != pending.end(); ++it) {
                    if ((*it)->id == id) {
                        cancelled_pending.push_back(std::move(*it));
                        pending.erase(it);
                        break;
                    }
                }
            }
            while (!pending.empty() && running.size() + admitted.size() < opts.max_slots) {
                Job& j = *pending.front();
                const Admit a = admit_one(j);
                if (a == Admit::no_room) break;   // head of line waits for memory
                (a == Admit::ok ? admitted : failed).push_back(std::move(pending.front()));
                pending.pop_front();
            }
            waiting = !pending.empty();
        }
        for (auto& j : cancelled_pending) finish(std::move(j), NASCH_ESTATE, 0);
        for (auto& j : failed) finish(std::move(j), NASCH_EDEVICE, 0);
        if (!admitted.empty()) dirty = true;
        for (auto& j : admitted) running.push_back(std::move(j));
        n_running = running.size();
        for (uint64_t id : cancels)
            for (auto& j : running)
                if (j && j->id == id) j->cancelled = true;
        if (running.empty()) continue;

        // ---- descriptors of the live slots (each at its own step and parity)
        eng.rings.resize(running.size());
        for (size_t i = 0; i < running.size(); ++i) {
            const Job& j = *running[i];
            const nasch_request& r = j.req;
            uint8_t* base = arena_base + j.off;
            RingDesc& d = eng.rings[i];
            if (dirty) {
                d = RingDesc{};
                d.buf[0] = base;
                d.buf[1] = nullptr;
                d.pl[0] = reinterpret_cast<uint32_t*>(base + grid_bytes(r));
                d.pl[1] = reinterpret_cast<uint32_t*>(base + grid_bytes(r) + plane_bytes(r));
                d.nw = plane_words(r.L);
                d.flux_log = reinterpret_cast<unsigned long long*>(base + log_offset(r));
                d.flux_acc = nullptr;
                d.log_t0 = 0;
                d.warmup = ~0ull;
                d.L = (uint32_t)r.L;
                d.vmax = r.vmax;
                d.t_end = (uint32_t)r.T;
                d.sp = slow_params(r.seed, r.replica, r.p);
            }
            d.t = j.t;
            d.parity = j.parity;
        }
        // ---- a burst of launches: none of them runs past the first slot to
        // finish, and only one while requests wait for admission
        uint32_t m = kMaxBurst;
        for (const auto& jp : running)
            m = std::min<uint64_t>(m, (jp->req.T - jp->t + k - 1) / k);
        if (waiting) m = 1;
        const hipError_t e_geo = dirty ? eng.set_geometry(k, q, stream) : eng.upload_rings(stream);
        dirty = false;
        if (!st.ok(e_geo) || !st.ok(eng.enqueue((uint64_t)m * k, d_clk, stream)) ||
            !st.ok(hipStreamSynchronize(stream))) {
            // a device failure ends every running request with an error
            for (auto& j : running) finish(std::move(j), NASCH_EDEVICE, 0);
            running.clear();
            n_running = 0;
            dirty = true;
            continue;
        }
        launches += m;
        // ---- bookkeeping and completions
        std::vector<std::unique_ptr<Job>> still;
        for (auto& jp : running) {
            Job& j = *jp;
            const uint64_t ran = std::min<uint64_t>((uint64_t)m * k, j.req.T - j.t);
            j.t += (uint32_t)ran;
            j.parity ^= m & 1u;
            if (j.cancelled) {
                finish(std::move(jp), NASCH_ESTATE, 0);
                dirty = true;
                continue;
            }
            if (j.t < j.req.T) {
                still.push_back(std::move(jp));
                continue;
            }
            dirty = true;
            const nasch_request& r = j.req;
            uint8_t* base = arena_base + j.off;
            flux_host.resize(r.T);
            int status = NASCH_OK;
            if (!st.ok(hipMemcpyAsync(flux_host.data(), base + log_offset(r), r.T * 8,
                                      hipMemcpyDeviceToHost, stream)))
                status = NASCH_EDEVICE;
            if (!status && r.grid_out) {
                // the final planes into the slot's byte grid, then to the host
                const ConvJob job{base,
                                  reinterpret_cast<uint32_t*>(base + grid_bytes(r) +
                                                              (j.parity ? plane_bytes(r) : 0)),
                                  (uint32_t)r.L, plane_words(r.L), r.vmax, 0u};
                if (!st.ok(launch_planes_to_bytes_one(job, stream)) ||
                    !st.ok(hipMemcpyAsync(r.grid_out, base, r.L, hipMemcpyDeviceToHost, stream)))
                    status = NASCH_EDEVICE;
            }
            if (!status && !st.ok(hipStreamSynchronize(stream))) status = NASCH_EDEVICE;
            uint64_t sum = 0;
            for (uint64_t f : flux_host) sum += f;
            if (!status && r.flux_out) std::memcpy(r.flux_out, flux_host.data(), r.T * 8);
            finish(std::move(jp), status, sum);
        }
        running.swap(still);
        n_running = running.size();
    }
}

extern "C" {

void nasch_server_default_opts(nasch_server_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
}

int nasch_server_create(nasch_server** out, const nasch_server_opts* opts) {
    if (!out) return NASCH_EINVAL;
    *out = nullptr;
    std::unique_ptr<nasch_server> s(new (std::nothrow) nasch_server());
    if (!s) return NASCH_ENOMEM;
    nasch_server_opts o;
    nasch_server_default_opts(&o);
    if (opts) o = *opts;
    if (!o.max_slots) o.max_slots = 4096;
    if (!o.k) o.k = 32;
    if (!o.q) o.q = 4;
    if (o.q > 4) return NASCH_EINVAL;
    if (kstep_max_k(NASCH_MAX_VMAX, o.q) < o.k) return NASCH_EINVAL;
    if (!o.hbm_budget) {
        size_t fr = 0, tot = 0;
        if (!s->st.ok(hipMemGetInfo(&fr, &tot))) return NASCH_EDEVICE;
        o.hbm_budget = fr / 2;
    }
    s->opts = o;
    if (o.stream) {
        s->stream = (hipStream_t)o.stream;
    } else {
        if (!s->st.ok(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking))) return NASCH_EDEVICE;
        s->own_stream = true;
    }
    if (!s->st.ok(dev_alloc(&s->arena_base, o.hbm_budget))) return NASCH_ENOMEM;
    s->arena.reset(o.hbm_budget);
    if (!s->st.ok(dev_alloc(&s->d_clk, 1))) return NASCH_ENOMEM;
    const Clock c0{0u, 0u};
    if (!s->st.ok(hipMemcpy(s->d_clk, &c0, sizeof(Clock), hipMemcpyHostToDevice))) return NASCH_EDEVICE;
    int dev = 0;
    (void)hipGetDevice(&dev);
    nasch_server* raw = s.get();
    raw->worker = std::thread([raw, dev] {
        (void)hipSetDevice(dev);
        raw->loop();
    });
    *out = s.release();
    return NASCH_OK;
}

int nasch_server_submit(nasch_server* s, const nasch_request* req, uint64_t* id) {
    if (!s || !req) return NASCH_EINVAL;
    int rc = validate_params(req->L, req->N, req->vmax, req->p);
    if (rc) return rc;
    if (req->init_v > NASCH_INIT_V_UNIFORM || req->T == 0 || req->T > 0xFFFFFFFFull)
        return NASCH_EINVAL;
    if (footprint(*req) > s->opts.hbm_budget) return NASCH_EINVAL;
    std::unique_ptr<Job> j(new (std::nothrow) Job());
    if (!j) return NASCH_ENOMEM;
    j->req = *req;
    j->t_submit = s->now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        j->id = s->next_id++;
        if (id) *id = j->id;
        s->pending.push_back(std::move(j));
    }
    s->cv_work.notify_one();
    return NASCH_OK;
}

int nasch_server_poll(nasch_server* s, nasch_result* out, uint32_t max, uint32_t* n,
                      uint32_t wait_ms) {
    if (!s || !n || (max && !out)) return NASCH_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (wait_ms && s->done.empty())
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    uint32_t c = 0;
    while (c < max && !s->done.empty()) {
        out[c++] = s->done.front();
        s->done.pop_front();
    }
    *n = c;
    return NASCH_OK;
}

int nasch_server_cancel(nasch_server* s, uint64_t id) {
    if (!s) return NASCH_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->cancel_ids.push_back(id);
    }
    s->cv_work.notify_one();
    return NASCH_OK;
}

int nasch_server_stats(nasch_server* s, uint64_t* pending, uint64_t* running, uint64_t* done,
                       uint64_t* bytes_in_use, uint64_t* launches) {
    if (!s) return NASCH_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (pending) *pending = s->pending.size();
    if (running) *running = s->n_running;
    if (done) *done = s->n_done;
    if (bytes_in_use) *bytes_in_use = s->arena.used();
    if (launches) *launches = s->launches;
    return NASCH_OK;
}

double nasch_server_now(nasch_server* s) { return s ? s->now() : 0.0; }

void nasch_server_destroy(nasch_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    s->eng.release();
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->d_clk) (void)hipFree(s->d_clk);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
