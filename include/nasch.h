/*
 * nasch.h -- C ABI of libnasch, the MI355X (gfx950) implementation of the
 * Nagel-Schreckenberg (NaSch) traffic model on a circular road.
 *
 * The operation (van Zon & Ponce, "Parallelizing a 1-Dim Nagel-Schreckenberg
 * Traffic Model", Handout section "The Nagel-Schreckenberg traffic model",
 * rules 1-4 and their summary system): every time step, every car
 *   1. speeds up by one if below vmax,
 *   2. slows to d-1 if the car in front is d cells ahead and v >= d,
 *   3. if v > 0, slows by one with probability p (a uniform r < p accepts),
 *   4. moves v cells forward on the ring of L cells (periodic boundary,
 *      Handout section "Starter Code").
 * All cars update synchronously from the state at the start of the step.
 *
 * Randomness.  The uniform r of rule 3 for the car that starts step t in cell
 * x is a 32-bit integer R(seed, replica, t, x), compared as R < thr with
 * thr = floor(p * 2^32).  R is built from Philox4x32-10 (Salmon et al., SC'11)
 * with key (seed mod 2^32, seed >> 32):
 *   bits 31..28 = bit (x mod 32) of output words 0..3 (word 0 on top) of
 *                 Philox(counter = (x div 32, t, replica, 1));
 *   bits 27..0  = output word 0 of Philox(counter = (x, t, replica, 2)) >> 4.
 * Results therefore do not depend on thread count, launch shape, temporal
 * block depth, representation or batch composition (the reproducibility the
 * paper demands in "Concepts Covered" and assignment item 1).
 *
 * Initial state (the paper asks for random positions but gives no method,
 * Handout "Starter Code"): car i < N starts in cell pi(i), where pi is a
 * 4-round balanced Feistel permutation on b bits (b = ceil(log2 L) rounded
 * up to even, >= 2), round function word 0 of Philox((half, round, replica,
 * 3)) masked to b/2 bits, restricted to [0, L) by cycle-walking.  Initial velocity: 0, or
 * floor(w * (vmax+1) / 2^32) with w = word 0 of Philox((x, 0, replica, 4)).
 *
 * Grid representation ("Concepts Covered"): one uint8 per cell, 0xFF = empty,
 * else the velocity of the car in the cell.  Agent representation: int32
 * positions x[N] in road order (cyclically sorted) and uint8 velocities v[N].
 * F(t) = sum of the velocities after step t (the flux of step t).
 *
 * Conventions for every entry point:
 *   - Return 0 on success or a negative NASCH_E* code; no exception crosses
 *     the ABI.  After NASCH_EDEVICE the HIP error code is kept in the handle
 *     (nasch_last_device_error).
 *   - Handles are owned by the library and released by the matching *_free /
 *     *_destroy call.  Every output pointer is caller-owned host memory of the
 *     stated size unless the name says "device".
 *   - Stepping calls are asynchronous on the handle's stream; calls that hand
 *     results to the host synchronise that stream first.
 *   - A handle must not be used from two threads at once; separate handles
 *     may be used concurrently.
 *   - The library uses the HIP device that is current when the handle is
 *     created.
 */
#ifndef NASCH_H
#define NASCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define NASCH_OK        0
#define NASCH_EINVAL   (-1)  /* an argument is out of range or inconsistent   */
#define NASCH_ENOMEM   (-2)  /* device or host allocation failed             */
#define NASCH_EDEVICE  (-3)  /* a HIP call failed; see nasch_last_device_error */
#define NASCH_ERANGE   (-4)  /* the step counter would reach 2^32            */
#define NASCH_ESTATE   (-5)  /* the handle is not in a state for this call    */
#define NASCH_EBUSY    (-6)  /* the request cannot be admitted right now      */
#define NASCH_ENOTFOUND (-7) /* no such replica / request                    */

/* ---- limits ------------------------------------------------------------ */
#define NASCH_MAX_VMAX  8u            /* the grid form's kernels (bit planes) are
                                         specialised for vmax <= 8: grid handles,
                                         batches, servers, device-buffer steps  */
#define NASCH_MAX_VMAX_AGENT 254u     /* the agent form takes any vmax up to 254
                                         (0xFF marks an empty cell)           */
#define NASCH_MAX_L     0x7FFFFFFFull /* L < 2^31: positions are int32         */

/* ---- option values ----------------------------------------------------- */
#define NASCH_REP_GRID   0u  /* uint8 per cell                            */
#define NASCH_REP_AGENT  1u  /* int32 x[N], uint8 v[N]                    */
#define NASCH_INIT_V_ZERO    0u
#define NASCH_INIT_V_UNIFORM 1u
#define NASCH_KERNEL_AUTO    0u /* autotuned: the temporal-blocked kernel, (k, q) chosen by timing */
#define NASCH_KERNEL_ONESTEP 1u /* one step per launch (no blocking); grid: on the byte form; agent: one-step launches of the k-step kernel */
#define NASCH_KERNEL_KSTEP   2u /* grid: k steps per launch, bit-sliced, k*vmax halo; agent: k steps per launch */
#define NASCH_RNG_KEYED      0u /* rule 3 draws R(seed, replica, t, x), see above */
#define NASCH_RNG_STREAM     1u /* agent form only: the paper's one shared stream, see below */
#define NASCH_BOUNDARY_RING  0u /* the circular road (periodic boundary)                    */
#define NASCH_BOUNDARY_OPEN  1u /* grid form only: an open road with entry and exit, below   */

typedef struct nasch_sim nasch_sim;

typedef struct {
    uint32_t replica;  /* Philox stream id (counter word 2); default 0; never a batch slot */
    uint32_t rep;      /* NASCH_REP_GRID or NASCH_REP_AGENT                                */
    uint32_t init_v;   /* NASCH_INIT_V_ZERO or NASCH_INIT_V_UNIFORM                         */
    uint32_t kernel;   /* NASCH_KERNEL_*                                                    */
    uint32_t k;        /* steps per launch for NASCH_KERNEL_KSTEP; 0 = default             */
    uint32_t q;        /* grid form: 32-cell words per lane of the bit-sliced kernel (1 to 4);
                          agent form: cars per lane of its k-step tiling (4 to 8), by default
                          chosen from the density so that the rule-3 blocks a wave's cars
                          start in take as few passes per car as possible; 0 = default       */
    uint32_t use_graph;/* 1: replay nasch_step_n launch sequences from a captured hipGraph */
    uint32_t rng;      /* NASCH_RNG_KEYED (default) or NASCH_RNG_STREAM (agent form only)   */
    void*    stream;   /* hipStream_t to run on; NULL = a stream owned by the handle        */
    uint32_t boundary; /* NASCH_BOUNDARY_RING (default) or NASCH_BOUNDARY_OPEN              */
    uint32_t reserved; /* must be 0                                                         */
    double   alpha;    /* open road: entry probability per step, 0 <= alpha <= 1            */
    double   beta;     /* open road: exit probability per step, 0 <= beta <= 1             */
} nasch_opts;

/*
 * NASCH_BOUNDARY_OPEN: the boundary-condition variation the paper suggests
 * (section "Variations"), which it does not specify further; this library's
 * reading.  Cars drive from cell 0 toward cell L-1 and nothing wraps.  At each
 * step t one gate draw G = Philox(counter = (0, t, replica, 5)) (same key as R)
 * decides both ends:
 *   - entry: if cell 0 is empty at the start of the step and word 0 of G is
 *     below floor(alpha 2^32), a car with v = 0 is in cell 0 after the step;
 *   - exit: unless word 1 of G is below floor(beta 2^32), a stopped car sits
 *     in cell L for the step (rule 2 sees it); otherwise the road ahead of the
 *     front car is free.  A car whose move ends at or past L leaves the road.
 * Rules 1-4 are otherwise those of the ring, with the same R(seed, replica,
 * t, x).  F(t) sums the velocities after rules 1-3 of every car that was on
 * the road at the start of the step, so a leaving car counts its whole move.
 * The car count changes; the initial state is the ring's (N cars placed on
 * [0, L)).  For vmax = 1 this is the totally asymmetric exclusion process with
 * parallel update (entry alpha, exit beta (1 - p), hop probability 1 - p).
 * Grid representation only (nasch_init returns NASCH_EINVAL for the agent
 * form); nasch_restore accepts any number of cars.
 */

/*
 * NASCH_RNG_STREAM reproduces the paper's own approach to random numbers
 * (Concepts Covered: one sequence shared by all threads, each thread jumping
 * ahead to its own numbers; Handout "IMPORTANT" box: a multiplicative linear
 * congruential generator): one minstd_rand stream, x <- 48271 x mod (2^31 - 1), seeded
 * with seed mod (2^31 - 1) (1 if that is 0).  Every car draws one number per
 * step in car order: car i (agent index, numbered from the lowest cell at
 * t = 0) at step t takes output number t N + i + 1 and slows iff
 * x < ceil(p (2^31 - 1)) (binary64).  GPU lanes jump ahead to their numbers
 * (a^n mod m by a table of powers).  The initial state is the same as in the
 * keyed mode.
 */

typedef struct {
    uint64_t L, N, t;
    uint32_t vmax, thr, replica, rep, init_v, kernel, k, q;
    uint64_t seed;
    uint64_t device_bytes; /* device memory held by the handle */
} nasch_info;

/* Fills *opts with the defaults (grid representation, v0 = 0, autotuned kernel). */
void nasch_default_opts(nasch_opts* opts);

/*
 * Create a simulation of N cars on a ring of L cells, initialised as described
 * above (t = 0).  Requires 1 <= L < 2^31, N <= L, 0 <= p < 1 (the range the
 * paper gives for p, Handout bullet list on drawing r), p not NaN, and
 * vmax <= 8 for the grid form (NASCH_MAX_VMAX) or vmax <= 254 for the agent
 * form (NASCH_MAX_VMAX_AGENT; the paper leaves vmax free).
 * opts may be NULL (defaults).  On success *out is a new handle; on failure
 * *out is NULL and nothing is leaked.
 */
int nasch_init(nasch_sim** out, uint64_t L, uint64_t N, uint32_t vmax, double p,
               uint64_t seed, const nasch_opts* opts);

/* Advance T >= 0 steps (rules 1-4, synchronous update), asynchronously on the
 * handle's stream.  F(t) for each step is kept on the device.  NASCH_ERANGE if
 * t + T would exceed 2^32 - 1 (nothing is enqueued then). */
int nasch_step_n(nasch_sim* h, uint64_t T);

/* Make room in the device flux log for `steps` more steps, so that the next
 * nasch_step_n calls covering them allocate nothing and do not synchronise. */
int nasch_reserve_log(nasch_sim* h, uint64_t steps);

/* As nasch_step_n, then waits; *ms receives the device time between two HIP
 * events recorded on the handle's stream around the enqueued launches. */
int nasch_timed_step_n(nasch_sim* h, uint64_t T, double* ms);

/* Copy F(t0), ..., F(t0 + count - 1) to out[count] (uint64).  Requires
 * t0 + count <= t.  Synchronises. */
int nasch_flux(nasch_sim* h, uint64_t t0, uint64_t count, uint64_t* out);

/* Copy the whole road in grid form (L bytes, 0xFF = empty, else v) to out and
 * the current step count to *t_out (either may be NULL).  The agent
 * representation is scattered to a grid on the device first.  Synchronises. */
int nasch_snapshot(nasch_sim* h, uint8_t* out, uint64_t* t_out);

/* Copy cells [start, start + len) mod L of the grid form to out[len].  Synchronises. */
int nasch_snapshot_range(nasch_sim* h, uint64_t start, uint64_t len, uint8_t* out);

/* Agent representation only: copy x[N] (int32, road order, cyclically
 * sorted) and v[N] (uint8).  Either may be NULL.  Synchronises. */
int nasch_agent_state(nasch_sim* h, int32_t* x, uint8_t* v);

/* Checkpoint restore: replace the state by grid[L] (host, 0xFF or a velocity
 * <= vmax per cell, exactly N cars) at step count t.  The flux of steps before
 * t is forgotten (nasch_flux then accepts t0 >= t only).  Continuing from a
 * restored snapshot gives the same results as the uninterrupted run, because
 * R depends only on (seed, replica, t, x).  Synchronises. */
int nasch_restore(nasch_sim* h, const uint8_t* grid, uint64_t t);

/* Checkpoint restore in the agent form, keeping car identity (which the
 * shared-stream mode needs): x[N] int32 positions in road order (cyclically
 * sorted, distinct, < L), v[N] <= vmax, at step count t.  Synchronises. */
int nasch_restore_agent(nasch_sim* h, const int32_t* x, const uint8_t* v, uint64_t t);

/* Choose the kernel and its tuning explicitly (values as in nasch_opts).
 * k = 0 or q = 0 keeps the current value.  Takes effect at the next step call. */
int nasch_set_tuning(nasch_sim* h, uint32_t kernel, uint32_t k, uint32_t q);

/* Time the candidate (k, q) settings on a scratch copy of the state (the
 * simulation itself does not advance) and keep the fastest.  Synchronises. */
int nasch_autotune(nasch_sim* h);

int nasch_get_info(const nasch_sim* h, nasch_info* info);

/* The HIP error (hipError_t value) behind the last NASCH_EDEVICE, or 0. */
int nasch_last_device_error(const nasch_sim* h);

/* The last HIP error any entry point met on the calling thread (also when no
 * handle was created, e.g. a failed nasch_init), or 0. */
int nasch_thread_last_device_error(void);

/* Release the handle and its device memory; NULL is accepted. */
void nasch_free(nasch_sim* h);

/* Static text for a status code. */
const char* nasch_strerror(int status);

/* ======================================================================= */
/* One step of a road held in caller-owned device memory: no handle and no   */
/* state in the library.  For callers that keep their roads in their own     */
/* device buffers (torch tensors, an arena of their own) instead of the      */
/* handle's.                                                                 */
/* ======================================================================= */

/*
 * Step t of the ring (rules 1-4 as above, synchronous update, the same R and
 * therefore the same result as step t of a handle holding this state) from
 * d_in to d_out.
 *   d_in   device, L bytes, grid form (0xFF = empty, else v <= vmax); read only.
 *          Other byte values give unspecified cells but no fault.
 *   d_out  device, L bytes; receives the road after the step.  Must not
 *          overlap d_in.  Both pointers 16-byte aligned.
 *   L, vmax, p, seed, replica   as in nasch_init (1 <= L < 2^31, vmax <= 8,
 *          0 <= p < 1); the car count is whatever d_in holds.
 *   t      the step's index (R depends on it); t <= 2^32 - 2.
 *   d_flux device uint64 (may be NULL): receives F(t).
 *   stream hipStream_t to run on (NULL = the null stream).
 * Asynchronous: enqueues the launches and returns.  The per-wave flux
 * partials are scratch allocated and freed on the stream (stream-ordered
 * allocation).  The caller owns every buffer.  Returns NASCH_EINVAL for bad
 * parameters, a NULL, misaligned or overlapping road, NASCH_ERANGE for
 * t > 2^32 - 2, NASCH_ENOMEM if the scratch cannot be allocated,
 * NASCH_EDEVICE if a launch fails (nasch_thread_last_device_error).
 */
int nasch_grid_step_device(const uint8_t* d_in, uint8_t* d_out, uint64_t L, uint32_t vmax,
                           double p, uint64_t seed, uint32_t replica, uint64_t t,
                           uint64_t* d_flux, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * step as nasch_grid_step_device, same arguments, layout, ownership and
 * errors, but it allocates nothing.  Its scratch (one uint32 flux partial per
 * block of eight 1984-cell tiles) is a static device array of 135301 words
 * (about 0.5 MiB) that each device the library runs on holds until the
 * process ends; every L the library accepts fits it (a launch needing more
 * would be NASCH_EINVAL).
 * All calls on one device share that array, so calls that overlap on one
 * device (different streams, or threads without ordering) race and must not
 * be issued; calls ordered on one stream are safe.  The array's contents
 * after a call are unspecified.  The first call on a device looks up the
 * array's device address (hipGetSymbolAddress) with that device current.
 */
int nasch_grid_step_device_noalloc(const uint8_t* d_in, uint8_t* d_out, uint64_t L,
                                   uint32_t vmax, double p, uint64_t seed, uint32_t replica,
                                   uint64_t t, uint64_t* d_flux, void* stream);

/* ======================================================================= */
/* Batched ensemble: many independent rings ("replicas") advanced together.  */
/* The paper suggests running parameter-study cases as embarrassingly       */
/* parallel jobs (section "Variations"); here every replica keeps its own   */
/* (L, N, vmax, p, seed, replica) and its results are identical to the same  */
/* simulation run alone through nasch_init / nasch_step_n.                   */
/* ======================================================================= */
typedef struct nasch_batch nasch_batch;

typedef struct {
    uint64_t L, N;
    uint32_t vmax;
    uint32_t init_v;   /* NASCH_INIT_V_* */
    double   p;
    uint64_t seed;
    uint32_t replica;  /* Philox stream id of this replica */
    uint32_t reserved; /* must be 0 */
    uint64_t warmup;   /* F(t) is summed for t >= warmup */
    uint32_t boundary; /* NASCH_BOUNDARY_RING or NASCH_BOUNDARY_OPEN (same for every replica) */
    uint32_t reserved2;/* must be 0 */
    double   alpha;    /* open road: entry probability per step, 0 <= alpha <= 1 */
    double   beta;     /* open road: exit probability per step, 0 <= beta <= 1 */
} nasch_replica;

typedef struct {
    void*    stream;    /* NULL = owned stream */
    uint32_t k;         /* steps per launch; 0 = default (autotune with nasch_batch_autotune) */
    uint32_t q;         /* words per lane; 0 = default */
    uint32_t use_graph; /* capture each nasch_batch_step_n launch sequence in a hipGraph */
    uint32_t keep_log;  /* also keep F(t) of every replica and step (R x T uint64 on device) */
    uint64_t log_steps; /* capacity of that log in steps (required if keep_log) */
} nasch_batch_opts;

void nasch_batch_default_opts(nasch_batch_opts* opts);

/* Create R >= 1 replicas (each validated as in nasch_init) in one device
 * arena, all at t = 0.  The replicas are all rings or all open roads
 * (NASCH_EINVAL otherwise); vmax, p and the gate probabilities may differ. */
int nasch_batch_init(nasch_batch** out, const nasch_replica* reps, uint32_t R,
                     const nasch_batch_opts* opts);

/* Put every replica back to its initial state at t = 0 (init kernels again)
 * and zero the flux sums and logs.  Synchronises. */
int nasch_batch_reset(nasch_batch* b);

/* Advance every replica by T steps.  Each launch runs k steps of every tile of
 * every replica; the launches are the same kernels a single simulation uses. */
int nasch_batch_step_n(nasch_batch* b, uint64_t T);
int nasch_batch_timed_step_n(nasch_batch* b, uint64_t T, double* ms);

/* out[R]: sum of F(t) over warmup <= t < current step, per replica.  Synchronises. */
int nasch_batch_flux_sums(nasch_batch* b, uint64_t* out);

/* F(t0 .. t0+count-1) of replica r (needs keep_log).  Synchronises. */
int nasch_batch_flux(nasch_batch* b, uint32_t r, uint64_t t0, uint64_t count, uint64_t* out);

/* Grid of replica r (L_r bytes) and the step count.  Synchronises. */
int nasch_batch_snapshot(nasch_batch* b, uint32_t r, uint8_t* out, uint64_t* t_out);

/* Checkpoint of the whole batch: every replica's grid, back to back in replica
 * order (replica r's L_r bytes start at L_0 + ... + L_{r-1}; out holds the sum
 * of the L_r), and the step count.  out is caller-owned host memory; one
 * conversion launch and one copy.  Synchronises.  NASCH_EINVAL for a NULL out. */
int nasch_batch_snapshot_all(nasch_batch* b, uint8_t* out, uint64_t* t_out);

/* Resume from a checkpoint (the model state is the grid, so this is what
 * checkpoint and resume of an ensemble need; see nasch_restore for one ring):
 * every replica's grid from `grids`, laid out as nasch_batch_snapshot_all writes
 * it (host memory, caller-owned, read before the call returns), and the step
 * counter set to t for all replicas.  Each cell must be 0xFF or at most the
 * replica's vmax, and a ring's car count must equal its N (an open road's may
 * differ).  The flux sums and the flux log are cleared.  Synchronises.
 * NASCH_EINVAL for a bad grid (the batch is then unchanged), NASCH_ERANGE for
 * t >= 2^32, NASCH_ENOMEM if the staging copy cannot be allocated. */
int nasch_batch_restore(nasch_batch* b, const uint8_t* grids, uint64_t t);

/* Choose (k, q) for this batch by timing candidates on a scratch copy of the
 * arena (the replicas do not advance); *k_out / *q_out may be NULL. */
int nasch_batch_autotune(nasch_batch* b, uint32_t* k_out, uint32_t* q_out);
int nasch_batch_set_tuning(nasch_batch* b, uint32_t k, uint32_t q);
int nasch_batch_last_device_error(const nasch_batch* b);
void nasch_batch_free(nasch_batch* b);

/* ======================================================================= */
/* Serving: simulations submitted one by one, admitted onto the GPU while    */
/* others run (continuous batching), state resident on the device.           */
/* ======================================================================= */
typedef struct nasch_server nasch_server;

typedef struct {
    uint64_t hbm_budget;  /* device bytes the server may hold for simulations; 0 = 1/2 of free memory */
    uint32_t max_slots;   /* simulations on the device at once; 0 = 4096 */
    uint32_t k;           /* steps per launch; 0 = 32 */
    uint32_t q;           /* words per lane; 0 = 4 */
    uint32_t reserved;
    void*    stream;      /* NULL = owned stream */
} nasch_server_opts;

typedef struct {
    uint64_t L, N;
    uint32_t vmax, init_v;
    double   p;
    uint64_t seed;
    uint32_t replica, reserved;
    uint64_t T;           /* steps to run */
    uint64_t* flux_out;   /* optional caller buffer of T uint64: F(0..T-1); must stay valid until polled */
    uint8_t*  grid_out;   /* optional caller buffer of L bytes: final grid */
} nasch_request;

typedef struct {
    uint64_t id;
    int32_t  status;      /* NASCH_OK or an error code */
    uint32_t reserved;
    uint64_t flux_sum;    /* sum of F(t), 0 <= t < T */
    double   t_submit, t_admit, t_done;  /* seconds on the server's monotonic clock */
} nasch_result;

void nasch_server_default_opts(nasch_server_opts* opts);
/* Start the server and its scheduling thread. */
int nasch_server_create(nasch_server** out, const nasch_server_opts* opts);
/* Queue a request (validated as nasch_init, 1 <= T < 2^32); its footprint,
 * ceil256(L) + 2 * ceil256(4 (vmax + 1) ceil(L / 32)) + ceil256(8 T) bytes
 * (the byte grid, two bit-plane copies of the road and the flux log, each
 * rounded up to 256 bytes), must fit hbm_budget.  *id receives its id.  Never
 * blocks on the GPU; the request waits in arrival order until it fits. */
int nasch_server_submit(nasch_server* s, const nasch_request* req, uint64_t* id);
/* Move up to max finished results to out; *n receives the count.  If
 * wait_ms > 0, waits up to that long for at least one. */
int nasch_server_poll(nasch_server* s, nasch_result* out, uint32_t max, uint32_t* n,
                      uint32_t wait_ms);
/* Cancel a queued or running request; its result is reported with NASCH_ESTATE. */
int nasch_server_cancel(nasch_server* s, uint64_t id);
/* Counters: pending, running, finished; device bytes in use; launches. */
int nasch_server_stats(nasch_server* s, uint64_t* pending, uint64_t* running, uint64_t* done,
                       uint64_t* bytes_in_use, uint64_t* launches);
/* Monotonic clock of the server in seconds (same clock as nasch_result). */
double nasch_server_now(nasch_server* s);
/* Liveness of the scheduling thread, for a watchdog: *since receives the
 * seconds since it last finished a burst of launches or picked up new work (0
 * when no request is queued or running) and *live the requests queued or
 * running.  A value that keeps growing while requests are live means a launch
 * has not returned; the server cannot abort a kernel, so a caller that sees
 * this stops submitting and reports.  Either pointer may be NULL. */
int nasch_server_health(nasch_server* s, double* since, uint64_t* live);
/* Stop the scheduling thread and release everything; unfinished requests are dropped. */
void nasch_server_destroy(nasch_server* s);

/* ======================================================================= */
/* Parameter file and output of the paper's starter code (Handout, "Starter */
/* Code"): a plain-text file of `key = value` lines (L, T, N, p, vmax, seed  */
/* required; outputprefix, per optional; '#' or ';' start a comment), and    */
/* three numpy files <prefix>-dens.npy (uint8 [frames, L]: 1 where a car is), */
/* <prefix>-velo.npy (uint8 [frames, L]: the car's velocity, else 0) and     */
/* <prefix>-time.npy (int64 [frames]: the step of each frame).              */
/* ======================================================================= */
typedef struct {
    uint64_t L, T, N;
    double   p;
    uint32_t vmax, reserved;
    uint64_t seed, per;         /* per = 0: no output */
    char     outputprefix[256]; /* default "traffic" */
} nasch_ini;

/* Parse a parameter file; NASCH_EINVAL on a missing required key, a malformed
 * value or parameters nasch_init would reject. */
int nasch_ini_read(const char* path, nasch_ini* out);

typedef struct nasch_writer nasch_writer;

/* Create the three output files for a road of L cells (overwriting them). */
int nasch_writer_open(nasch_writer** out, const char* prefix, uint64_t L);
/* Append the simulation's current road as one frame.  The device-to-host copy
 * is enqueued on the simulation's stream into a pinned staging buffer and the
 * call returns; a writer thread converts and writes it while the simulation
 * continues (it blocks only when all staging buffers are in flight). */
int nasch_writer_frame(nasch_writer* w, nasch_sim* h);
/* Append a frame from a host grid (L bytes, 0xFF = empty) at step t. */
int nasch_writer_frame_host(nasch_writer* w, const uint8_t* grid, uint64_t t);
/* Write every pending frame, finish the headers and close the files. */
int nasch_writer_close(nasch_writer* w);

#ifdef __cplusplus
}
#endif
#endif /* NASCH_H */
