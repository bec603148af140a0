// output.hip -- the parameter file and the .npy output of the paper's starter code
// (Handout, "Starter Code": `key = value` parameters L, T, N, p, vmax, seed,
// outputprefix, per; output files <prefix>-dens.npy, <prefix>-velo.npy and
// <prefix>-time.npy holding density and velocity on the grid at the stored
// times, written every `per` steps).  Entry points are documented in
// include/nasch.h.
//
// A frame is the road at one step: dens[x] = 1 where a car is, else 0;
// velo[x] = the car's velocity there, else 0.  nasch_writer_frame enqueues the
// device-to-host copy of the grid on the simulation's stream (into one of a
// few pinned staging buffers) and returns; a writer thread waits for the copy,
// converts it and appends to the files, so file output overlaps the steps that
// follow (the paper's optional assignment item on parallelising I/O).
#include <hip/hip_runtime.h>

#include <cctype>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "engine.hpp"
#include "nasch.h"

using namespace nasch;

namespace {

constexpr size_t kNpyHeader = 128;  // fixed header size: the shape is patched at close
constexpr int kSlots = 4;

// A .npy (format 1.0) file whose first dimension grows as rows are appended.
struct NpyFile {
    FILE* f = nullptr;
    std::string descr;
    uint64_t row = 0;      // elements per row (0: 1-D)
    uint64_t rows = 0;
    bool open(const std::string& path, const char* d, uint64_t row_len) {
        f = std::fopen(path.c_str(), "wb");
        if (!f) return false;
        descr = d;
        row = row_len;
        return write_header();
    }
    bool write_header() {
        char dict[kNpyHeader];
        int n;
        if (row)
            n = std::snprintf(dict, sizeof dict, "{'descr': '%s', 'fortran_order': False, 'shape': (%llu, %llu), }",
                              descr.c_str(), (unsigned long long)rows, (unsigned long long)row);
        else
            n = std::snprintf(dict, sizeof dict, "{'descr': '%s', 'fortran_order': False, 'shape': (%llu,), }",
                              descr.c_str(), (unsigned long long)rows);
        if (n < 0 || (size_t)n + 11 > kNpyHeader) return false;
        unsigned char hdr[kNpyHeader];
        std::memset(hdr, ' ', kNpyHeader);
        const unsigned char magic[8] = {0x93, 'N', 'U', 'M', 'P', 'Y', 1, 0};
        std::memcpy(hdr, magic, 8);
        const uint16_t hl = (uint16_t)(kNpyHeader - 10);
        hdr[8] = (unsigned char)(hl & 0xFF);
        hdr[9] = (unsigned char)(hl >> 8);
        std::memcpy(hdr + 10, dict, (size_t)n);
        hdr[kNpyHeader - 1] = '\n';
        if (std::fseek(f, 0, SEEK_SET) != 0) return false;
        return std::fwrite(hdr, 1, kNpyHeader, f) == kNpyHeader && std::fseek(f, 0, SEEK_END) == 0;
    }
    bool append(const void* p, size_t bytes) {
        if (std::fwrite(p, 1, bytes, f) != bytes) return false;
        ++rows;
        return true;
    }
    bool close() {
        if (!f) return true;
        bool ok = write_header();
        ok = (std::fclose(f) == 0) && ok;
        f = nullptr;
        return ok;
    }
};

struct Slot {
    uint8_t* host = nullptr;   // pinned when the runtime has a device, else malloc'd
    bool pinned = false;
    hipEvent_t done = nullptr;
    uint64_t t = 0;
    bool busy = false;
    bool from_device = false;
};

std::string trim(const std::string& s) {
    size_t a = 0, b = s.size();
    while (a < b && std::isspace((unsigned char)s[a])) ++a;
    while (b > a && std::isspace((unsigned char)s[b - 1])) --b;
    return s.substr(a, b - a);
}

}  // namespace

struct nasch_writer {
    uint64_t L = 0;
    NpyFile dens, velo, time;
    Slot slots[kSlots];
    std::deque<int> queue;     // slots waiting to be written, in frame order
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false, failed = false;
    std::thread thread;
    std::vector<uint8_t> d_row, v_row;

    void run() {
        for (;;) {
            int s;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || !queue.empty(); });
                if (queue.empty()) return;
                s = queue.front();
                queue.pop_front();
            }
            Slot& sl = slots[s];
            bool ok = true;
            if (sl.from_device) ok = hipEventSynchronize(sl.done) == hipSuccess;
            if (ok) {
                for (uint64_t x = 0; x < L; ++x) {
                    const uint8_t c = sl.host[x];
                    d_row[x] = c != 0xFF;
                    v_row[x] = c != 0xFF ? c : 0;
                }
                const int64_t t = (int64_t)sl.t;
                ok = dens.append(d_row.data(), L) && velo.append(v_row.data(), L) &&
                     time.append(&t, sizeof t);
            }
            std::lock_guard<std::mutex> lk(mu);
            if (!ok) failed = true;
            sl.busy = false;
            cv.notify_all();
        }
    }
    // a free staging slot, waiting for the writer if all are busy
    int acquire() {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            for (int s = 0; s < kSlots; ++s)
                if (!slots[s].busy) {
                    slots[s].busy = true;
                    return s;
                }
            cv.wait(lk);
        }
    }
    void submit(int s) {
        std::lock_guard<std::mutex> lk(mu);
        queue.push_back(s);
        cv.notify_all();
    }
};

extern "C" {

int nasch_writer_open(nasch_writer** out, const char* prefix, uint64_t L) {
    if (!out) return NASCH_EINVAL;
    *out = nullptr;
    if (!prefix || L == 0 || L > NASCH_MAX_L) return NASCH_EINVAL;
    std::unique_ptr<nasch_writer> w(new (std::nothrow) nasch_writer());
    if (!w) return NASCH_ENOMEM;
    w->L = L;
    const std::string p(prefix);
    if (!w->dens.open(p + "-dens.npy", "|u1", L) || !w->velo.open(p + "-velo.npy", "|u1", L) ||
        !w->time.open(p + "-time.npy", "<i8", 0)) {
        w->dens.close();
        w->velo.close();
        w->time.close();
        return NASCH_EINVAL;
    }
    for (Slot& s : w->slots) {
        // pinned staging for asynchronous device frames; without a device
        // (host frames only) plain memory does
        if (hipHostMalloc((void**)&s.host, L, hipHostMallocDefault) == hipSuccess &&
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) == hipSuccess) {
            s.pinned = true;
        } else {
            (void)hipGetLastError();
            if (s.host) (void)hipHostFree(s.host);
            s.host = (uint8_t*)std::malloc(L);
            s.done = nullptr;
        }
        if (!s.host) {
            for (Slot& r : w->slots) {
                if (r.host) { if (r.pinned) (void)hipHostFree(r.host); else std::free(r.host); }
                if (r.done) (void)hipEventDestroy(r.done);
            }
            w->dens.close();
            w->velo.close();
            w->time.close();
            return NASCH_ENOMEM;
        }
    }
    w->d_row.resize(L);
    w->v_row.resize(L);
    nasch_writer* raw = w.get();
    raw->thread = std::thread([raw] { raw->run(); });
    *out = w.release();
    return NASCH_OK;
}

int nasch_writer_frame_host(nasch_writer* w, const uint8_t* grid, uint64_t t) {
    if (!w || !grid) return NASCH_EINVAL;
    const int s = w->acquire();
    std::memcpy(w->slots[s].host, grid, w->L);
    w->slots[s].t = t;
    w->slots[s].from_device = false;
    w->submit(s);
    return NASCH_OK;
}

int nasch_writer_close(nasch_writer* w) {
    if (!w) return NASCH_EINVAL;
    {
        std::lock_guard<std::mutex> lk(w->mu);
        w->stop = true;
    }
    w->cv.notify_all();
    if (w->thread.joinable()) w->thread.join();
    bool ok = !w->failed;
    ok = w->dens.close() && ok;
    ok = w->velo.close() && ok;
    ok = w->time.close() && ok;
    for (Slot& s : w->slots) {
        if (s.host) { if (s.pinned) (void)hipHostFree(s.host); else std::free(s.host); }
        if (s.done) (void)hipEventDestroy(s.done);
    }
    delete w;
    return ok ? NASCH_OK : NASCH_EINVAL;
}

int nasch_ini_read(const char* path, nasch_ini* out) {
    if (!path || !out) return NASCH_EINVAL;
    FILE* f = std::fopen(path, "r");
    if (!f) return NASCH_EINVAL;
    std::memset(out, 0, sizeof(*out));
    std::snprintf(out->outputprefix, sizeof out->outputprefix, "traffic");
    unsigned seen = 0;
    char line[1024];
    int rc = NASCH_OK;
    while (std::fgets(line, sizeof line, f)) {
        std::string s(line);
        const size_t hash = s.find_first_of("#;");
        if (hash != std::string::npos) s = s.substr(0, hash);
        s = trim(s);
        if (s.empty()) continue;
        const size_t eq = s.find('=');
        if (eq == std::string::npos) { rc = NASCH_EINVAL; break; }
        const std::string key = trim(s.substr(0, eq));
        std::string val = trim(s.substr(eq + 1));
        if (val.size() >= 2 && (val.front() == '"' || val.front() == '\'') && val.back() == val.front())
            val = val.substr(1, val.size() - 2);
        char* end = nullptr;
        if (key == "L") { out->L = std::strtoull(val.c_str(), &end, 10); seen |= 1; }
        else if (key == "T") { out->T = std::strtoull(val.c_str(), &end, 10); seen |= 2; }
        else if (key == "N") { out->N = std::strtoull(val.c_str(), &end, 10); seen |= 4; }
        else if (key == "p") { out->p = std::strtod(val.c_str(), &end); seen |= 8; }
        else if (key == "vmax") { out->vmax = (uint32_t)std::strtoul(val.c_str(), &end, 10); seen |= 16; }
        else if (key == "seed") { out->seed = std::strtoull(val.c_str(), &end, 10); seen |= 32; }
        else if (key == "per") { out->per = std::strtoull(val.c_str(), &end, 10); seen |= 64; }
        else if (key == "outputprefix") {
            if (val.size() >= sizeof out->outputprefix) { rc = NASCH_EINVAL; break; }
            std::snprintf(out->outputprefix, sizeof out->outputprefix, "%s", val.c_str());
            continue;
        } else {
            continue;  // unknown keys are ignored
        }
        if (!end || *end != '\0' || val.empty()) { rc = NASCH_EINVAL; break; }
    }
    std::fclose(f);
    if (rc) return rc;
    if ((seen & 63u) != 63u) return NASCH_EINVAL;   // L, T, N, p, vmax, seed are required
    return validate_params(out->L, out->N, out->vmax, out->p);
}

}  // extern "C"

// Device frames live beside the simulation internals (runtime.hip).
int nasch_writer_enqueue_device(nasch_writer* w, const uint8_t* d_grid, uint64_t t,
                                hipStream_t s) {
    const int slot = w->acquire();
    Slot& sl = w->slots[slot];
    if (!sl.pinned) {
        std::lock_guard<std::mutex> lk(w->mu);
        sl.busy = false;
        return NASCH_EDEVICE;
    }
    sl.t = t;
    sl.from_device = true;
    if (hipMemcpyAsync(sl.host, d_grid, w->L, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(sl.done, s) != hipSuccess) {
        std::lock_guard<std::mutex> lk(w->mu);
        sl.busy = false;
        return NASCH_EDEVICE;
    }
    w->submit(slot);
    return NASCH_OK;
}

uint64_t nasch_writer_length(const nasch_writer* w) { return w->L; }
