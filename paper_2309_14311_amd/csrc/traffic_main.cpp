// nasch_traffic -- command-line driver in the shape of the paper's starter code
// (Handout, "How to compile and run": `./traffic test.ini`): reads the parameter
// file, runs T steps on the GPU and, if per > 0, writes a frame every `per`
// steps (and at t = 0) to <outputprefix>-dens/velo/time.npy.  Prints the
// stepping time, which with per = 0 is the pure computation the assignment's
// scaling runs ask for.
//
// usage: nasch_traffic file.ini [--agent] [--stream] [--onestep]
#include <chrono>
#include <cstdio>
#include <cstring>

#include "nasch.h"

static int fail(const char* what, int rc) {
    std::fprintf(stderr, "nasch_traffic: %s: %s (%d)\n", what, nasch_strerror(rc), rc);
    return 1;
}

int main(int argc, char** argv) {
    if (argc < 2) {
        std::fprintf(stderr, "usage: %s file.ini [--agent] [--stream] [--onestep]\n", argv[0]);
        return 2;
    }
    nasch_ini ini;
    int rc = nasch_ini_read(argv[1], &ini);
    if (rc) return fail(argv[1], rc);
    nasch_opts o;
    nasch_default_opts(&o);
    for (int i = 2; i < argc; ++i) {
        if (!std::strcmp(argv[i], "--agent")) o.rep = NASCH_REP_AGENT;
        else if (!std::strcmp(argv[i], "--stream")) o.rng = NASCH_RNG_STREAM;
        else if (!std::strcmp(argv[i], "--onestep")) o.kernel = NASCH_KERNEL_ONESTEP;
        else {
            std::fprintf(stderr, "unknown option %s\n", argv[i]);
            return 2;
        }
    }
    nasch_sim* h = nullptr;
    rc = nasch_init(&h, ini.L, ini.N, ini.vmax, ini.p, ini.seed, &o);
    if (rc) return fail("nasch_init", rc);
    nasch_writer* w = nullptr;
    if (ini.per) {
        rc = nasch_writer_open(&w, ini.outputprefix, ini.L);
        if (rc) return fail("nasch_writer_open", rc);
        rc = nasch_writer_frame(w, h);
        if (rc) return fail("nasch_writer_frame", rc);
    }
    rc = nasch_reserve_log(h, ini.T);
    if (rc) return fail("nasch_reserve_log", rc);
    const auto t0 = std::chrono::steady_clock::now();
    uint64_t done = 0;
    while (done < ini.T) {
        const uint64_t n = ini.per ? (ini.per < ini.T - done ? ini.per : ini.T - done) : ini.T;
        rc = nasch_step_n(h, n);
        if (rc) return fail("nasch_step_n", rc);
        done += n;
        if (w && done % ini.per == 0) {
            rc = nasch_writer_frame(w, h);
            if (rc) return fail("nasch_writer_frame", rc);
        }
    }
    uint64_t last = 0;
    if (ini.T) {
        rc = nasch_flux(h, ini.T - 1, 1, &last);   // synchronises
        if (rc) return fail("nasch_flux", rc);
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (w) {
        rc = nasch_writer_close(w);
        if (rc) return fail("nasch_writer_close", rc);
    }
    std::printf("L=%llu N=%llu vmax=%u p=%g T=%llu seed=%llu per=%llu: %.6f s, %.4g cell-updates/s, F(T-1)=%llu\n",
                (unsigned long long)ini.L, (unsigned long long)ini.N, ini.vmax, ini.p,
                (unsigned long long)ini.T, (unsigned long long)ini.seed,
                (unsigned long long)ini.per, secs, secs > 0 ? (double)ini.L * ini.T / secs : 0.0,
                (unsigned long long)last);
    nasch_free(h);
    return 0;
}
