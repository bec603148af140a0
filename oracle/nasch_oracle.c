/*
 * nasch_oracle.c -- plain serial CPU oracle for the Nagel-Schreckenberg (NaSch)
 * time step on a circular road.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library.  Only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant generator with the HIP
 * path: every routine below is written out again from its published definition.
 *
 * What it follows (paper: "Parallelizing a 1-Dim Nagel-Schreckenberg Traffic
 * Model", van Zon & Ponce, EduHPC-23):
 *   - the four update rules and their summary system (Handout, section "The
 *     Nagel-Schreckenberg traffic model", rules 1-4 and the cases equation);
 *   - the acceptance test "r < p accepts, r >= p rejects" for rule 3 (same
 *     section, the bullet list on drawing random numbers);
 *   - the grid and agent representations (section "Concepts Covered"; Handout
 *     "IMPORTANT" box);
 *   - periodic boundary conditions, no cars entering or leaving (Handout,
 *     "Starter Code");
 *   - one reproducible random sequence, independent of the thread count
 *     (section "Concepts Covered"; Handout assignment item 1).
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - the update is synchronous: every car reads the state at the start of the
 *     step (the parallel update of Nagel & Schreckenberg 1992);
 *   - rule 3 lowers v by one, never below zero (the cases equation is garbled,
 *     the prose says "if v > 0");
 *   - d is the forward distance to the next car mod L; one car alone has d = L;
 *   - the uniform r in [0,1) of rule 3 is a 32-bit integer R compared with
 *     thr = floor(p * 2^32), drawn from a counter-based generator keyed by
 *     (seed, replica, step t, cell x where the car starts the step);
 *   - the random initial placement is a keyed Feistel permutation with
 *     cycle-walking; initial velocities are 0 or uniform in 0..vmax;
 *   - the flux of step t is F(t) = sum of the velocities after the step.
 *
 * Every function is plain and serial.  The only parallel construct is the
 * OpenMP loop of oracle_run_grid, the all-core twin used for large CPU runs; it
 * executes the very same per-car body, so its result cannot depend on the
 * number of threads (checked by the tests).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EMPTY 0xFFu

/* Tags that separate the independent random streams (counter word 3). */
#define TAG_SLOW_HI 1u  /* rule 3, top 4 bits of R, one block per 32 cells */
#define TAG_SLOW_LO 2u  /* rule 3, low 28 bits of R, one block per cell     */
#define TAG_PLACE   3u  /* initial placement, Feistel round function        */
#define TAG_VEL0    4u  /* initial velocities                               */

/* ------------------------------------------------------------------------- */
/* Philox4x32-10: Salmon, Moraes, Dror & Shaw, "Parallel Random Numbers: As   */
/* Easy as 1, 2, 3", SC'11, section 3 (the Philox S-box and key schedule).    */
/* Ten rounds; each round multiplies counter words 0 and 2 by the two Philox */
/* constants, and the key is bumped by the two Weyl constants between rounds.*/
/* ------------------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t prod0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                   uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------- */
/* The 32-bit uniform R(seed, replica, t, x) of rule 3.                       */
/*   bits 31..28: bit (x mod 32) of words 0,1,2,3 (word 0 is the top bit) of  */
/*                Philox((x div 32, t, replica, TAG_SLOW_HI), seed);          */
/*   bits 27..0 : word 0 of Philox((x, t, replica, TAG_SLOW_LO), seed) >> 4.  */
/* Every bit comes from a distinct output bit of the generator, so R is       */
/* uniform on [0, 2^32).                                                      */
/* ------------------------------------------------------------------------- */
uint32_t oracle_rand32(uint64_t seed, uint32_t replica, uint32_t t, uint32_t x)
{
    uint32_t blk[4], cell[4];
    philox(x >> 5, t, replica, TAG_SLOW_HI, seed, blk);
    philox(x, t, replica, TAG_SLOW_LO, seed, cell);
    uint32_t hi4 = 0;
    for (int j = 0; j < 4; j++)
        hi4 |= ((blk[j] >> (x & 31u)) & 1u) << (3 - j);
    uint32_t lo28 = cell[0] >> 4;
    return (hi4 << 28) | lo28;
}

/* thr = floor(p * 2^32); the product is exact in binary64. */
uint32_t oracle_threshold(double p)
{
    return (uint32_t)floor(p * 4294967296.0);
}

/* ------------------------------------------------------------------------- */
/* Initial placement: N distinct cells out of L.                              */
/* A balanced 4-round Feistel network on b bits (b = ceil(log2 L) rounded up  */
/* to even, at least 2) is a permutation of [0, 2^b); cycle-walking (Black &  */
/* Rogaway, "Ciphers with Arbitrary Finite Domains", CT-RSA 2002) restricts   */
/* it to a permutation of [0, L).  Car i starts at perm(i), i < N.            */
/* ------------------------------------------------------------------------- */
static unsigned feistel_bits(uint64_t L)
{
    unsigned b = 0;
    while (((uint64_t)1 << b) < L) b++;
    if (b & 1u) b++;
    if (b < 2) b = 2;
    return b;
}

static uint32_t feistel_round(uint32_t half, uint32_t round, uint32_t replica,
                              uint64_t seed, uint32_t mask)
{
    uint32_t o[4];
    philox(half, round, replica, TAG_PLACE, seed, o);
    return o[0] & mask;
}

static uint64_t feistel_forward(uint64_t i, unsigned b, uint32_t replica, uint64_t seed)
{
    unsigned h = b / 2;
    uint32_t mask = (uint32_t)(((uint64_t)1 << h) - 1);
    uint32_t left = (uint32_t)(i >> h) & mask, right = (uint32_t)i & mask;
    for (uint32_t j = 0; j < 4; j++) {
        uint32_t f = feistel_round(right, j, replica, seed, mask);
        uint32_t new_left = right;
        uint32_t new_right = left ^ f;
        left = new_left; right = new_right;
    }
    return ((uint64_t)left << h) | right;
}

static uint64_t feistel_inverse(uint64_t y, unsigned b, uint32_t replica, uint64_t seed)
{
    unsigned h = b / 2;
    uint32_t mask = (uint32_t)(((uint64_t)1 << h) - 1);
    uint32_t left = (uint32_t)(y >> h) & mask, right = (uint32_t)y & mask;
    for (int j = 3; j >= 0; j--) {
        /* forward round j mapped (l, r) -> (r, l ^ F_j(r)) */
        uint32_t old_right = left;
        uint32_t old_left = right ^ feistel_round(old_right, (uint32_t)j, replica, seed, mask);
        left = old_left; right = old_right;
    }
    return ((uint64_t)left << h) | right;
}

uint64_t oracle_place(uint64_t i, uint64_t L, uint32_t replica, uint64_t seed)
{
    unsigned b = feistel_bits(L);
    uint64_t y = feistel_forward(i, b, replica, seed);
    while (y >= L) y = feistel_forward(y, b, replica, seed);
    return y;
}

uint64_t oracle_place_inverse(uint64_t y, uint64_t L, uint32_t replica, uint64_t seed)
{
    unsigned b = feistel_bits(L);
    uint64_t z = feistel_inverse(y, b, replica, seed);
    while (z >= L) z = feistel_inverse(z, b, replica, seed);
    return z;
}

/* Initial velocity of the car that starts in cell x: 0, or uniform in
 * 0..vmax as floor(u * (vmax + 1) / 2^32) with u a 32-bit Philox word. */
uint32_t oracle_initial_velocity(uint32_t x, uint32_t vmax, uint32_t init_v,
                                 uint32_t replica, uint64_t seed)
{
    if (!init_v) return 0;
    uint32_t o[4];
    philox(x, 0, replica, TAG_VEL0, seed, o);
    return (uint32_t)(((uint64_t)o[0] * (uint64_t)(vmax + 1)) >> 32);
}

/* Grid at t = 0: EMPTY everywhere, v0 at the N placed cells. */
void oracle_init_grid(uint64_t L, uint64_t N, uint32_t vmax, uint32_t init_v,
                      uint32_t replica, uint64_t seed, uint8_t *g)
{
    memset(g, EMPTY, L);
    for (uint64_t i = 0; i < N; i++) {
        uint64_t x = oracle_place(i, L, replica, seed);
        g[x] = (uint8_t)oracle_initial_velocity((uint32_t)x, vmax, init_v, replica, seed);
    }
}

/* Cells [a, a+w) (mod L) of the grid at t = 0, through the inverse
 * permutation: cell y holds a car iff its preimage is below N. */
void oracle_init_window(uint64_t L, uint64_t N, uint32_t vmax, uint32_t init_v,
                        uint32_t replica, uint64_t seed, uint64_t a, uint64_t w,
                        uint8_t *out)
{
    for (uint64_t i = 0; i < w; i++) {
        uint64_t y = (a + i) % L;
        uint64_t z = oracle_place_inverse(y, L, replica, seed);
        out[i] = (z < N) ? (uint8_t)oracle_initial_velocity((uint32_t)y, vmax, init_v,
                                                             replica, seed)
                         : (uint8_t)EMPTY;
    }
}

/* ------------------------------------------------------------------------- */
/* The paper's own random numbers (Concepts Covered; Handout "IMPORTANT" box):  */
/* one multiplicative linear congruential stream shared by all cars.  Here it */
/* is the C++ minstd_rand engine, x <- 48271 x mod (2^31 - 1), seeded with    */
/* seed mod m (1 if that is 0).  Every car draws one number per step, in car  */
/* order: car i at step t uses output number t N + i + 1 of the stream.  The  */
/* uniform r = x / m is below p iff x < ceil(p m) (binary64).                  */
/* ------------------------------------------------------------------------- */
#define MLCG_A 48271u
#define MLCG_M 2147483647u

uint32_t oracle_mlcg_seed(uint64_t seed)
{
    uint32_t x0 = (uint32_t)(seed % MLCG_M);
    return x0 ? x0 : 1u;
}

uint32_t oracle_mlcg_next(uint32_t x)
{
    return (uint32_t)(((uint64_t)MLCG_A * x) % MLCG_M);
}

uint32_t oracle_mlcg_threshold(double p)
{
    return (uint32_t)ceil(p * 2147483647.0);
}

/* ------------------------------------------------------------------------- */
/* One car, rules 1-4.  v is the car's velocity at the start of step t, d its */
/* distance to the car in front.  Returns the velocity after the step; the    */
/* car then advances by that many cells.                                      */
/* ------------------------------------------------------------------------- */
static uint32_t nasch_rules(uint32_t v, uint64_t d, uint32_t vmax, uint32_t thr,
                            uint64_t seed, uint32_t replica, uint32_t t, uint32_t x)
{
    /* rule 1: speed up if below vmax */
    if (v < vmax) v = v + 1;
    /* rule 2: the car in front is d away; if v >= d, slow to d - 1 */
    if ((uint64_t)v >= d) v = (uint32_t)(d - 1);
    /* rule 3: if v > 0, with probability p slow by one (accept iff r < p) */
    if (v > 0 && oracle_rand32(seed, replica, t, x) < thr) v = v - 1;
    /* rule 4 is the move x <- x + v, done by the caller */
    return v;
}

/* Grid representation, one synchronous step t.  gin and gout are L cells
 * each (EMPTY or the velocity of the car in the cell).  Returns F(t). */
uint64_t oracle_step_grid(uint64_t L, uint32_t vmax, uint32_t thr, uint64_t seed,
                          uint32_t replica, uint32_t t, const uint8_t *gin, uint8_t *gout,
                          int nthreads)
{
    uint64_t flux = 0;
    memset(gout, EMPTY, L);
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) reduction(+ : flux) num_threads(nthreads)
#else
    (void)nthreads;
#endif
    for (int64_t xs = 0; xs < (int64_t)L; xs++) {
        uint64_t x = (uint64_t)xs;
        if (gin[x] == EMPTY) continue;
        /* distance to the next car ahead.  Only d <= vmax can change v
         * (rule 2 needs v >= d and v <= vmax), so the scan stops at vmax + 1;
         * on a ring shorter than that it meets the car itself at d = L. */
        uint64_t d = 1;
        while (d <= vmax && gin[(x + d) % L] == EMPTY) d++;
        uint32_t v = nasch_rules(gin[x], d, vmax, thr, seed, replica, t, (uint32_t)x);
        gout[(x + v) % L] = (uint8_t)v;
        flux += v;
    }
    return flux;
}

/* T steps from step t0 in the grid representation; g is updated in place,
 * flux[s] = F(t0 + s).  nthreads > 1 runs the OpenMP twin. */
int oracle_run_grid(uint64_t L, uint32_t vmax, double p, uint64_t seed, uint32_t replica,
                    uint64_t t0, uint64_t T, uint8_t *g, uint64_t *flux, int nthreads)
{
    uint32_t thr = oracle_threshold(p);
    uint8_t *tmp = (uint8_t *)malloc(L ? L : 1);
    if (!tmp) return -1;
    for (uint64_t s = 0; s < T; s++) {
        uint64_t f = oracle_step_grid(L, vmax, thr, seed, replica, (uint32_t)(t0 + s), g, tmp,
                                      nthreads);
        if (flux) flux[s] = f;
        memcpy(g, tmp, L);
    }
    free(tmp);
    return 0;
}

/* Agent representation, one synchronous step t: two vectors x[N], v[N] of
 * the cars in road order (x cyclically sorted).  d = (x[i+1] - x[i]) mod L,
 * or L for a car alone.  Returns F(t). */
uint64_t oracle_step_agent(uint64_t L, uint64_t N, uint32_t vmax, uint32_t thr, uint64_t seed,
                           uint32_t replica, uint32_t t, const int32_t *x, const uint8_t *v,
                           int32_t *xout, uint8_t *vout)
{
    uint64_t flux = 0;
    for (uint64_t i = 0; i < N; i++) {
        uint64_t d;
        if (N == 1) d = L;
        else d = ((uint64_t)x[(i + 1) % N] + L - (uint64_t)x[i]) % L;
        uint32_t vn = nasch_rules(v[i], d, vmax, thr, seed, replica, t, (uint32_t)x[i]);
        xout[i] = (int32_t)(((uint64_t)x[i] + vn) % L);
        vout[i] = (uint8_t)vn;
        flux += vn;
    }
    return flux;
}

/* Agent representation with the shared stream: *state is the stream state after
 * the draws of steps before t0 (oracle_mlcg_seed(seed) at t = 0); it is
 * advanced by N draws per step, strictly one after another. */
int oracle_run_agent_mlcg(uint64_t L, uint64_t N, uint32_t vmax, double p, uint32_t *state,
                          uint64_t T, int32_t *x, uint8_t *v, uint64_t *flux)
{
    uint32_t thr = oracle_mlcg_threshold(p);
    int32_t *xt = (int32_t *)malloc((N ? N : 1) * sizeof(int32_t));
    uint8_t *vt = (uint8_t *)malloc(N ? N : 1);
    if (!xt || !vt) { free(xt); free(vt); return -1; }
    for (uint64_t s = 0; s < T; s++) {
        uint64_t f = 0;
        for (uint64_t i = 0; i < N; i++) {
            uint64_t d;
            if (N == 1) d = L;
            else d = ((uint64_t)x[(i + 1) % N] + L - (uint64_t)x[i]) % L;
            uint32_t vn = v[i];
            /* rule 1 */
            if (vn < vmax) vn = vn + 1;
            /* rule 2 */
            if ((uint64_t)vn >= d) vn = (uint32_t)(d - 1);
            /* rule 3: this car's number of the shared stream */
            *state = oracle_mlcg_next(*state);
            if (vn > 0 && *state < thr) vn = vn - 1;
            /* rule 4 */
            xt[i] = (int32_t)(((uint64_t)x[i] + vn) % L);
            vt[i] = (uint8_t)vn;
            f += vn;
        }
        if (flux) flux[s] = f;
        memcpy(x, xt, N * sizeof(int32_t));
        memcpy(v, vt, N);
    }
    free(xt); free(vt);
    return 0;
}

int oracle_run_agent(uint64_t L, uint64_t N, uint32_t vmax, double p, uint64_t seed,
                     uint32_t replica, uint64_t t0, uint64_t T, int32_t *x, uint8_t *v,
                     uint64_t *flux)
{
    uint32_t thr = oracle_threshold(p);
    int32_t *xt = (int32_t *)malloc((N ? N : 1) * sizeof(int32_t));
    uint8_t *vt = (uint8_t *)malloc(N ? N : 1);
    if (!xt || !vt) { free(xt); free(vt); return -1; }
    for (uint64_t s = 0; s < T; s++) {
        uint64_t f = oracle_step_agent(L, N, vmax, thr, seed, replica, (uint32_t)(t0 + s), x, v,
                                       xt, vt);
        if (flux) flux[s] = f;
        memcpy(x, xt, N * sizeof(int32_t));
        memcpy(v, vt, N);
    }
    free(xt); free(vt);
    return 0;
}

/* Agent vectors of a grid: the occupied cells in ascending order. */
uint64_t oracle_grid_to_agent(uint64_t L, const uint8_t *g, int32_t *x, uint8_t *v)
{
    uint64_t n = 0;
    for (uint64_t c = 0; c < L; c++)
        if (g[c] != EMPTY) { x[n] = (int32_t)c; v[n] = g[c]; n++; }
    return n;
}

/* ------------------------------------------------------------------------- */
/* Final state of a window of a large ring, without simulating the ring.      */
/* A cell after one step depends only on the cells within vmax of it (the car */
/* that lands there started at most vmax behind and looked at most vmax       */
/* ahead of its start).  So cells [a, a+w) at step t0+T follow from cells     */
/* [a - T*vmax, a + w + T*vmax) at step t0.  The segment is stepped as an     */
/* open road whose outside is empty; the wrong values this puts at its ends   */
/* travel inward by at most vmax cells per step and never reach the window.   */
/* seg holds w + 2*T*vmax cells on entry (the state at t0 starting at ring    */
/* cell a - T*vmax mod L) and is overwritten; out receives w cells.           */
/* ------------------------------------------------------------------------- */
int oracle_advance_segment(uint64_t L, uint32_t vmax, double p, uint64_t seed,
                           uint32_t replica, uint64_t t0, uint64_t T, uint64_t a, uint64_t w,
                           uint8_t *seg, uint8_t *out)
{
    uint32_t thr = oracle_threshold(p);
    uint64_t R = T * (uint64_t)vmax;
    uint64_t S = w + 2 * R;
    uint64_t s0 = (a % L + L - (R % L)) % L; /* ring cell of seg[0] */
    uint8_t *tmp = (uint8_t *)malloc(S ? S : 1);
    if (!tmp) return -1;
    for (uint64_t s = 0; s < T; s++) {
        uint32_t t = (uint32_t)(t0 + s);
        memset(tmp, EMPTY, S);
        for (uint64_t c = 0; c < S; c++) {
            if (seg[c] == EMPTY) continue;
            uint64_t d = 1;
            while (d <= vmax && (c + d >= S || seg[c + d] == EMPTY)) d++;
            uint32_t xring = (uint32_t)((s0 + c) % L);
            uint32_t v = nasch_rules(seg[c], d, vmax, thr, seed, replica, t, xring);
            if (c + v < S) tmp[c + v] = (uint8_t)v;
        }
        memcpy(seg, tmp, S);
    }
    memcpy(out, seg + R, w);
    free(tmp);
    return 0;
}

/* Cells [a, a+w) of the ring after T steps from the initial state. */
int oracle_window_from_init(uint64_t L, uint64_t N, uint32_t vmax, double p, uint64_t seed,
                            uint32_t replica, uint32_t init_v, uint64_t T, uint64_t a,
                            uint64_t w, uint8_t *out)
{
    uint64_t R = T * (uint64_t)vmax;
    if (w + 2 * R >= L) {
        /* the cone covers the ring: simulate all of it */
        uint8_t *g = (uint8_t *)malloc(L);
        if (!g) return -1;
        oracle_init_grid(L, N, vmax, init_v, replica, seed, g);
        if (oracle_run_grid(L, vmax, p, seed, replica, 0, T, g, NULL, 1)) { free(g); return -1; }
        for (uint64_t i = 0; i < w; i++) out[i] = g[(a + i) % L];
        free(g);
        return 0;
    }
    uint64_t S = w + 2 * R;
    uint8_t *seg = (uint8_t *)malloc(S);
    if (!seg) return -1;
    uint64_t s0 = (a % L + L - (R % L)) % L;
    oracle_init_window(L, N, vmax, init_v, replica, seed, s0, S, seg);
    int rc = oracle_advance_segment(L, vmax, p, seed, replica, 0, T, a, w, seg, out);
    free(seg);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Open road (the paper's "Variations": change the boundary conditions).      */
/* Readings, since the paper gives no details:                                */
/*   - the road is cells 0 .. L-1 and cars drive toward L-1; nothing wraps;   */
/*   - at each step t one gate draw G = Philox((0, t, replica, 5)) decides   */
/*     the ends: a car enters iff word 0 < floor(alpha 2^32), the exit is   */
/*     open iff word 1 < floor(beta 2^32) (alpha = 1 or beta = 1: always);   */
/*   - a closed exit acts as a stopped car in cell L for that step, an open  */
/*     exit as an empty road beyond L-1; rules 1-3 are otherwise unchanged,  */
/*     and a car whose move ends at or beyond L leaves the road;             */
/*   - the entering car appears in cell 0 with v = 0 at the end of the step, */
/*     provided cell 0 was empty at its start (no car can move into cell 0); */
/*   - F(t) sums the velocities after rules 1-3 of every car that was on the */
/*     road at the start of the step, so a leaving car counts its whole move. */
/* For vmax = 1 this is the totally asymmetric exclusion process with        */
/* parallel update: entry alpha, exit beta (1 - p), hop probability 1 - p.   */
/* ------------------------------------------------------------------------- */
#define TAG_GATE 5u

/* floor(a 2^32) for 0 <= a <= 1, in [0, 2^32]: exact, since a * 2^32 only
 * changes the exponent of a binary64 number. */
uint64_t oracle_gate_threshold(double a)
{
    return (uint64_t)floor(ldexp(a, 32));
}

/* The two gate words of step t. */
void oracle_gate_words(uint64_t seed, uint32_t replica, uint32_t t, uint32_t *in_word,
                       uint32_t *out_word)
{
    uint32_t o[4];
    philox(0u, t, replica, TAG_GATE, seed, o);
    *in_word = o[0];
    *out_word = o[1];
}

/* One synchronous step t of cells [lo, lo+n) of an open road of L cells.
 * With lo = 0 and n = L this is the whole road.  A sub-range (for light-cone
 * windows) keeps the real boundary only at the ends it shares with the road:
 * a cut end takes no car in and treats what lies beyond as empty road, so
 * only cells far enough from it are exact after several steps.  Returns F(t);
 * *entered and *left (may be NULL) count the car that came in and the cars
 * that went out of the road in this step. */
uint64_t oracle_step_open(uint64_t L, uint64_t lo, uint64_t n, uint32_t vmax, uint32_t thr,
                          uint64_t thr_in, uint64_t thr_out, uint64_t seed, uint32_t replica,
                          uint32_t t, const uint8_t *gin, uint8_t *gout, uint64_t *entered,
                          uint64_t *left)
{
    uint32_t in_word, out_word;
    oracle_gate_words(seed, replica, t, &in_word, &out_word);
    int at_entry = (lo == 0);
    int at_exit = (lo + n == L);
    int enter = at_entry && (uint64_t)in_word < thr_in;
    int exit_closed = at_exit && !((uint64_t)out_word < thr_out);
    uint64_t flux = 0, went = 0, came = 0;
    memset(gout, EMPTY, n);
    for (uint64_t i = 0; i < n; i++) {
        if (gin[i] == EMPTY) continue;
        /* distance to what is in front: the next car within vmax cells, else
         * the closed exit (a stopped car in cell L), else nothing (vmax + 1
         * is as good as infinity for rule 2) */
        uint64_t d = 1;
        while (d <= vmax && i + d < n && gin[i + d] == EMPTY) d++;
        if (d <= vmax && i + d >= n) {           /* ran off the end of the cells */
            if (exit_closed && i + d == n) {
                /* cell L holds the stopped car: d is its distance */
            } else {
                d = (uint64_t)vmax + 1;
            }
        }
        uint32_t v = nasch_rules(gin[i], d, vmax, thr, seed, replica, t, (uint32_t)(lo + i));
        flux += v;
        if (i + v < n) gout[i + v] = (uint8_t)v;
        else if (at_exit) went++;             /* rule 4 took it past cell L-1 */
    }
    if (enter && gin[0] == EMPTY) {
        gout[0] = 0;
        came = 1;
    }
    if (entered) *entered = came;
    if (left) *left = went;
    return flux;
}

/* T steps from step t0 of cells [lo, lo+n) of an open road (see
 * oracle_step_open); g is updated in place; flux[s], entered[s] and left[s]
 * (each may be NULL) receive step t0 + s. */
int oracle_run_open(uint64_t L, uint64_t lo, uint64_t n, uint32_t vmax, double p, double alpha,
                    double beta, uint64_t seed, uint32_t replica, uint64_t t0, uint64_t T,
                    uint8_t *g, uint64_t *flux, uint64_t *entered, uint64_t *left)
{
    uint32_t thr = oracle_threshold(p);
    uint64_t thr_in = oracle_gate_threshold(alpha), thr_out = oracle_gate_threshold(beta);
    uint8_t *tmp = (uint8_t *)malloc(n ? n : 1);
    if (!tmp) return -1;
    for (uint64_t s = 0; s < T; s++) {
        uint64_t e = 0, l = 0;
        uint64_t f = oracle_step_open(L, lo, n, vmax, thr, thr_in, thr_out, seed, replica,
                                      (uint32_t)(t0 + s), g, tmp, &e, &l);
        if (flux) flux[s] = f;
        if (entered) entered[s] = e;
        if (left) left[s] = l;
        memcpy(g, tmp, n);
    }
    free(tmp);
    return 0;
}

/* Cells [a, a+w) of an open road after T steps from its initial state (the
 * same placement as the ring), evaluated on the light cone: the cells
 * [a - T vmax, a + w + T vmax) clipped to the road, run as a sub-range. */
int oracle_open_window_from_init(uint64_t L, uint64_t N, uint32_t vmax, double p, double alpha,
                                 double beta, uint64_t seed, uint32_t replica, uint32_t init_v,
                                 uint64_t T, uint64_t a, uint64_t w, uint8_t *out)
{
    uint64_t r = T * (uint64_t)vmax;
    uint64_t lo = a > r ? a - r : 0;
    uint64_t hi = a + w + r < L ? a + w + r : L;
    uint64_t n = hi - lo;
    uint8_t *g = (uint8_t *)malloc(n ? n : 1);
    if (!g) return -1;
    oracle_init_window(L, N, vmax, init_v, replica, seed, lo, n, g);
    if (oracle_run_open(L, lo, n, vmax, p, alpha, beta, seed, replica, 0, T, g, NULL, NULL,
                        NULL)) {
        free(g);
        return -1;
    }
    memcpy(out, g + (a - lo), w);
    free(g);
    return 0;
}

int oracle_num_threads_available(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* FNV-1a, 64-bit (Fowler, Noll & Vo): offset basis 14695981039346656037,    */
/* prime 2^40 + 2^8 + 0xb3.  Each byte is XORed in, then the hash is          */
/* multiplied by the prime mod 2^64.  A checksum of a whole final state for   */
/* the full-size parity records: h is the running hash (the offset basis to   */
/* start), and the result is the hash after the n further bytes.             */
/* ------------------------------------------------------------------------- */
uint64_t oracle_fnv1a64(const uint8_t *bytes, uint64_t n, uint64_t h)
{
    for (uint64_t i = 0; i < n; i++) {
        h ^= bytes[i];
        h *= 1099511628211ull;
    }
    return h;
}
