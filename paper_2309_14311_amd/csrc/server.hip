// server.hip -- serving loop: simulations submitted one by one and advanced on the
// GPU by continuous batching.  Entry points are documented in include/nasch.h.
//
// A scheduling thread owns the device.  Each iteration it
//   1. admits queued requests in arrival order while their footprint fits the
//      HBM budget and a slot is free (state allocated from a device arena,
//      initialised by the init kernel);
//   2. runs a burst of launches of the temporal-blocked grid kernel over the
//      live large rings, each slot advancing from its own step counter (the
//      burst stops where the first slot finishes, and is a single launch while
//      requests wait for admission), while the small rings run bursts of their
//      own on a second stream, started and collected as they finish; the tile
//      items are rebuilt only when a set of live slots changes;
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

// Every live slot of a chain of launches advances the same number of steps
// per launch, so a ring's steps cost as much wall time as the whole chain's.
// Rings of at most kSmallCells cells therefore run in a chain of their own on a
// second stream, kSmallBurst launches at a time on its own clock: the host
// starts it, goes on with the large rings' bursts, and collects it when it has
// finished.  Its launches are short, so a small ring's latency follows its own
// work instead of the arena's.
constexpr uint64_t kSmallCells = 65536;
constexpr uint32_t kSmallBurst = 4;
// The small chain takes as few 32-cell words per lane as the steps per launch
// allow (see small_q): a ring shorter than a wave's segment repeats around it,
// so the shortest segment wastes the least on them.
uint32_t small_q(uint32_t k, uint32_t q) {
    for (uint32_t qq = 1; qq < q; qq *= 2)
        if (kstep_max_k(NASCH_MAX_VMAX, qq) >= k) return qq;
    return q;
}

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
    hipStream_t stream = nullptr;     // admission, the large rings, results
    bool own_stream = false;
    hipStream_t stream_s = nullptr;   // the small rings' chain
    hipEvent_t ev_admit = nullptr;    // orders the small chain after admission
    hipEvent_t ev_small = nullptr;    // the small chain's burst has finished
    HipStatus st;
    uint8_t* arena_base = nullptr;
    Arena arena;
    Clock* d_clk = nullptr;   // stays {0, 0}: each slot carries its own t and parity
    uint32_t* d_init_tab = nullptr;   // placement round-function table of an admission
    GridEngine eng;           // the large rings
    GridEngine eng_s;         // the small rings
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<Job>> pending;
    std::vector<std::unique_ptr<Job>> running;     // large rings
    std::vector<std::unique_ptr<Job>> running_s;   // small rings in the chain (fixed while it runs)
    std::vector<std::unique_ptr<Job>> ready_s;     // admitted small rings waiting for the chain
    std::deque<nasch_result> done;
    std::vector<uint64_t> cancel_ids;
    uint64_t next_id = 1;
    uint64_t n_done = 0;
    // read by nasch_server_stats while the scheduling thread runs
    std::atomic<uint64_t> n_running{0}, launches{0};
    std::atomic<double> t_alive{0.0};   // last burst finished or work picked up
    bool stop = false;
    std::thread worker;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void loop();
    void describe(GridEngine& e, const std::vector<std::unique_ptr<Job>>& set, bool full);
    bool complete(std::vector<std::unique_ptr<Job>>& set, uint32_t m, std::vector<uint64_t>& flux_host);
    void fail_all();
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
    if (!st.ok(launch_init_grid(base, (uint32_t)r.L, (uint32_t)r.N, r.vmax, r.init_v, sp, stream,
                                d_init_tab)) ||
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

// Ring descriptors of a set of slots, each at its own step and parity; `full`
// rebuilds them (the set changed), else only the steps and parities move.
void nasch_server::describe(GridEngine& e, const std::vector<std::unique_ptr<Job>>& set,
                            bool full) {
    if (full) e.rings.resize(set.size());
    for (size_t i = 0; i < set.size(); ++i) {
        const Job& j = *set[i];
        const nasch_request& r = j.req;
        uint8_t* base = arena_base + j.off;
        RingDesc& d = e.rings[i];
        if (full) {
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
}

// Advance every slot of a set by the m launches it ran, hand back the finished
// and cancelled ones (results copied on the main stream) and keep the rest.
// Returns whether the set changed.
bool nasch_server::complete(std::vector<std::unique_ptr<Job>>& set, uint32_t m,
                            std::vector<uint64_t>& flux_host) {
    const uint32_t k = opts.k;
    bool changed = false;
    std::vector<std::unique_ptr<Job>> still;
    for (auto& jp : set) {
        Job& j = *jp;
        const uint64_t ran = std::min<uint64_t>((uint64_t)m * k, j.req.T - j.t);
        j.t += (uint32_t)ran;
        j.parity ^= m & 1u;
        if (j.cancelled) {
            finish(std::move(jp), NASCH_ESTATE, 0);
            changed = true;
            continue;
        }
        if (j.t < j.req.T) {
            still.push_back(std::move(jp));
            continue;
        }
        changed = true;
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
    set.swap(still);
    return changed;
}

// A device failure ends every live request with an error.
void nasch_server::fail_all() {
    (void)hipStreamSynchronize(stream);
    (void)hipStreamSynchronize(stream_s);
    for (auto* set : {&running, &running_s, &ready_s}) {
        for (auto& j : *set) finish(std::move(j), NASCH_EDEVICE, 0);
        set->clear();
    }
    n_running = 0;
}

void nasch_server::loop() {
    const uint32_t k = opts.k, q = opts.q, q_s = small_q(k, q);
    std::vector<uint64_t> flux_host;
    bool dirty = true;     // the set of large slots changed: rebuild their tile items
    bool dirty_s = true;   // the same for the small slots
    bool busy_s = false;   // the small chain has a burst in flight
    uint32_t m_s = 0;      // its launches
    for (;;) {
        // ---- admission and cancellation
        std::vector<std::unique_ptr<Job>> admitted;
        std::vector<std::unique_ptr<Job>> cancelled_pending, failed;
        std::vector<uint64_t> cancels;
        bool waiting;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                return stop || !pending.empty() || !running.empty() || !running_s.empty() ||
                       !ready_s.empty() || !cancel_ids.empty();
            });
            if (stop) return;
            t_alive = now();
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
            const size_t live = running.size() + running_s.size() + ready_s.size();
            while (!pending.empty() && live + admitted.size() < opts.max_slots) {
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
        for (auto& j : admitted) {
            if (j->req.L <= kSmallCells) {
                ready_s.push_back(std::move(j));
            } else {
                running.push_back(std::move(j));
                dirty = true;
            }
        }
        for (uint64_t id : cancels)
            for (auto* set : {&running, &running_s, &ready_s})
                for (auto& j : *set)
                    if (j && j->id == id) j->cancelled = true;
        // admitted small slots join the chain while it is idle
        if (!busy_s && !ready_s.empty()) {
            for (auto& j : ready_s) running_s.push_back(std::move(j));
            ready_s.clear();
            dirty_s = true;
        }
        n_running = running.size() + running_s.size() + ready_s.size();

        // ---- the small chain: when idle, a burst of kSmallBurst launches (or
        // up to the last of its slots to finish: one that finishes earlier idles,
        // the kernel stopping its steps at t_end), after the admission work on
        // the main stream; no launch starts a slot's steps past 2^32 - 1
        if (!busy_s && !running_s.empty()) {
            uint64_t most = 0, room = ~0ull;
            for (const auto& j : running_s) {
                most = std::max<uint64_t>(most, (j->req.T - j->t + k - 1) / k);
                room = std::min<uint64_t>(room, (0xFFFFFFFFull - j->t) / k);
            }
            m_s = (uint32_t)std::min<uint64_t>({(uint64_t)kSmallBurst, most,
                                                 std::max<uint64_t>(room, 1)});
            describe(eng_s, running_s, dirty_s);
            const hipError_t e_geo =
                dirty_s ? eng_s.set_geometry(k, q_s, stream_s) : eng_s.upload_rings(stream_s);
            dirty_s = false;
            if (!st.ok(hipEventRecord(ev_admit, stream)) ||
                !st.ok(hipStreamWaitEvent(stream_s, ev_admit, 0)) || !st.ok(e_geo) ||
                !st.ok(eng_s.enqueue((uint64_t)m_s * k, d_clk, stream_s)) ||
                !st.ok(hipEventRecord(ev_small, stream_s))) {
                fail_all();
                busy_s = false;
                dirty = dirty_s = true;
                continue;
            }
            busy_s = true;
            launches += m_s;
        }

        // ---- the large rings: a burst of launches, none of them past the first
        // slot to finish, and only one while requests wait for admission; with
        // no large rings the host waits for the small chain instead
        if (!running.empty()) {
            describe(eng, running, dirty);
            uint32_t m = kMaxBurst;
            for (const auto& jp : running)
                m = std::min<uint64_t>(m, (jp->req.T - jp->t + k - 1) / k);
            if (waiting) m = 1;
            const hipError_t e_geo = dirty ? eng.set_geometry(k, q, stream) : eng.upload_rings(stream);
            dirty = false;
            if (!st.ok(e_geo) || !st.ok(eng.enqueue((uint64_t)m * k, d_clk, stream)) ||
                !st.ok(hipStreamSynchronize(stream))) {
                fail_all();
                busy_s = false;
                dirty = dirty_s = true;
                continue;
            }
            launches += m;
            t_alive = now();
            if (complete(running, m, flux_host)) dirty = true;
        } else if (busy_s && !st.ok(hipEventSynchronize(ev_small))) {
            fail_all();
            busy_s = false;
            dirty = dirty_s = true;
            continue;
        }

        // ---- the small chain's burst, once it has finished
        if (busy_s) {
            const hipError_t e_s = hipEventQuery(ev_small);
            if (e_s == hipSuccess) {
                busy_s = false;
                t_alive = now();
                if (complete(running_s, m_s, flux_host)) dirty_s = true;
            } else if (e_s != hipErrorNotReady) {
                (void)st.ok(e_s);
                fail_all();
                busy_s = false;
                dirty = dirty_s = true;
                continue;
            }
        }
        n_running = running.size() + running_s.size() + ready_s.size();
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
    if (!s->st.ok(hipStreamCreateWithFlags(&s->stream_s, hipStreamNonBlocking)) ||
        !s->st.ok(hipEventCreateWithFlags(&s->ev_admit, hipEventDisableTiming)) ||
        !s->st.ok(hipEventCreateWithFlags(&s->ev_small, hipEventDisableTiming)))
        return NASCH_EDEVICE;
    if (!s->st.ok(dev_alloc(&s->arena_base, o.hbm_budget))) return NASCH_ENOMEM;
    s->arena.reset(o.hbm_budget);
    if (!s->st.ok(dev_alloc(&s->d_clk, 1))) return NASCH_ENOMEM;
    // one placement table serves every admission (they run in order on one stream)
    if (!s->st.ok(dev_alloc(&s->d_init_tab, init_tab_words(feistel_bits(NASCH_MAX_L)))))
        return NASCH_ENOMEM;
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
        // an idle server starts its liveness clock at the first new request
        if (s->pending.empty() && s->n_running == 0) s->t_alive = s->now();
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

int nasch_server_health(nasch_server* s, double* since, uint64_t* live) {
    if (!s) return NASCH_EINVAL;
    uint64_t n;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        n = s->pending.size() + s->n_running;
    }
    if (live) *live = n;
    if (since) *since = n ? std::max(0.0, s->now() - s->t_alive.load()) : 0.0;
    return NASCH_OK;
}

void nasch_server_destroy(nasch_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->stream_s) (void)hipStreamSynchronize(s->stream_s);
    s->eng.release();
    s->eng_s.release();
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->d_clk) (void)hipFree(s->d_clk);
    if (s->d_init_tab) (void)hipFree(s->d_init_tab);
    if (s->ev_admit) (void)hipEventDestroy(s->ev_admit);
    if (s->ev_small) (void)hipEventDestroy(s->ev_small);
    if (s->stream_s) (void)hipStreamDestroy(s->stream_s);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
