"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a published known-answer vector,
a textbook automaton, a closed form of the deterministic model, an exact
Markov-chain result computed by brute force, an exact expectation, or an
invariant of the update rules (Handout, "The Nagel-Schreckenberg traffic
model", rules 1-4).  A plausible slip in the oracle (a dropped rule, a wrong
sign or index, rules 2 and 3 swapped, a sequential instead of a synchronous
update, the acceptance test of rule 3 reversed) fails at least one of them.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

EMPTY = 0xFF
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- PRNG
def test_philox_known_answers(orc):
    """Philox4x32-10 reproduces the published known-answer vectors."""
    n = 0
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(s, 16) for s in line.replace("->", " ").split()]
            ctr, key, want = w[0:4], w[4:6], w[6:10]
            assert list(orc.philox4x32_10(ctr, key)) == want
            n += 1
    assert n == 3


@pytest.mark.parametrize("p", [0.0, 0.13, 0.25, 0.5, 0.2, 1e-9, 0.999999, 1 - 2**-53])
def test_threshold_is_floor_p_times_2_32(orc, p):
    """thr = floor(p * 2^32) exactly (exact rational arithmetic)."""
    want = math.floor(Fraction(p) * 2**32)
    assert orc.threshold(p) == want
    assert 0 <= want < 2**32


def test_rand32_uniform_and_acceptance_rate(orc):
    """R is uniform on 32 bits: the top nibble and the low bits are flat, and
    the fraction with R < floor(p 2^32) is p within 5 sigma."""
    n = 40000
    rs = np.array([orc.rand32(12345, 3, t, x) for t in range(4) for x in range(n // 4)],
                  dtype=np.uint64)
    top = (rs >> 28).astype(np.int64)
    counts = np.bincount(top, minlength=16)
    chi2 = ((counts - n / 16) ** 2 / (n / 16)).sum()
    assert chi2 < 50  # 15 dof, p ~ 1e-5
    low = ((rs >> 4) & 0xF).astype(np.int64)
    counts = np.bincount(low, minlength=16)
    assert ((counts - n / 16) ** 2 / (n / 16)).sum() < 50
    for p in (0.13, 0.5, 0.0625 + 0.001):
        thr = orc.threshold(p)
        frac = float((rs < thr).mean())
        sigma = math.sqrt(p * (1 - p) / n)
        assert abs(frac - p) < 5 * sigma, (p, frac)


def test_rand32_depends_on_every_key_field(orc):
    base = orc.rand32(1, 0, 0, 0)
    assert orc.rand32(2, 0, 0, 0) != base
    assert orc.rand32(1 << 40, 0, 0, 0) != orc.rand32(0, 0, 0, 0)
    assert orc.rand32(1, 1, 0, 0) != base
    assert orc.rand32(1, 0, 1, 0) != base
    assert orc.rand32(1, 0, 0, 1) != base
    # neighbours inside one 32-cell block differ in their low bits
    assert len({orc.rand32(1, 0, 0, x) for x in range(32)}) == 32


# --------------------------------------------------------------------------- init
@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 16, 17, 63, 64, 65, 1000, 1024, 1025])
def test_placement_is_a_permutation(orc, L):
    """Cycle-walked Feistel placement is a bijection of [0, L) with an inverse."""
    img = [orc.place(i, L, 0, 99) for i in range(L)]
    assert sorted(img) == list(range(L))
    for i, y in enumerate(img):
        assert orc.place_inverse(y, L, 0, 99) == i


def test_init_grid_exact_count_and_window(orc):
    for (L, N, vmax, init_v) in [(1000, 200, 5, 0), (1000, 200, 5, 1), (37, 37, 3, 1),
                                 (50, 0, 2, 1), (4096, 1000, 8, 1)]:
        g = orc.init_grid(L, N, vmax, seed=5, init_v=init_v)
        occ = g != EMPTY
        assert occ.sum() == N
        assert g[occ].max(initial=0) <= vmax
        if not init_v:
            assert (g[occ] == 0).all()
        w = orc.init_window(L, N, vmax, 5, a=L - 7, w=L + 14, init_v=init_v)
        assert np.array_equal(w, np.concatenate([g[L - 7:], g, g[:7]]))


def test_init_occupancy_uniform_over_seeds(orc):
    """Each cell is occupied with probability N/L (chi-square over 2000 seeds)."""
    L, N, S = 64, 16, 2000
    hits = np.zeros(L)
    for s in range(S):
        hits += orc.init_grid(L, N, 1, seed=s) != EMPTY
    exp = S * N / L
    chi2 = ((hits - exp) ** 2 / exp).sum()
    assert chi2 < 120  # 63 dof


def test_initial_velocity_uniform(orc):
    vmax = 5
    vs = np.array([orc.initial_velocity(x, vmax, 1, 0, 7) for x in range(30000)])
    counts = np.bincount(vs, minlength=vmax + 1)
    assert counts.size == vmax + 1
    exp = vs.size / (vmax + 1)
    assert ((counts - exp) ** 2 / exp).sum() < 30
    assert orc.initial_velocity(3, vmax, 0, 0, 7) == 0


# --------------------------------------------------------------------------- rules
def _rule184(occ):
    """Wolfram's elementary cellular automaton rule 184 on a ring."""
    left, right = np.roll(occ, 1), np.roll(occ, -1)
    code = 4 * left + 2 * occ + right
    return (184 >> code) & 1


@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 11])
def test_vmax1_p0_is_rule_184_exhaustive(orc, L):
    """vmax = 1 and p = 0 is the traffic automaton rule 184: every ring
    configuration of L <= 11 cells, every initial velocity in {0, 1}."""
    for bits in range(1 << L):
        occ = np.array([(bits >> i) & 1 for i in range(L)], dtype=np.int64)
        for vbits in (0, (1 << L) - 1):
            g = np.where(occ == 1, np.array([(vbits >> i) & 1 for i in range(L)]), EMPTY)
            g = g.astype(np.uint8)
            out, f = orc.step_grid(g, 1, 0.0, seed=1, t=0)
            assert np.array_equal((out != EMPTY).astype(np.int64), _rule184(occ)), (L, bits)
            # velocity 1 exactly where a car arrived from the left
            moved = (np.roll(occ, 1) == 1) & (occ == 0)
            assert np.array_equal(out == 1, moved)
            assert f == int(moved.sum())


def _random_grid(rng, L, N, vmax):
    g = np.full(L, EMPTY, np.uint8)
    cells = rng.choice(L, size=N, replace=False)
    g[cells] = rng.integers(0, vmax + 1, size=N)
    return g


@pytest.mark.parametrize("L,N,vmax", [(1000, 200, 5), (1000, 100, 5), (500, 300, 2),
                                      (37, 5, 3), (97, 40, 8), (200, 1, 5), (64, 63, 4),
                                      (10, 10, 3), (300, 30, 1)])
def test_p0_stationary_flux_closed_form(orc, L, N, vmax):
    """Without rule 3 the stationary flux per step is min(N vmax, L - N):
    free flow moves every car vmax, a jam moves every car its whole gap."""
    rng = np.random.default_rng(L * 131 + N)
    g = _random_grid(rng, L, N, vmax)
    W = max(2 * L, 1000)
    _, flux = orc.run_grid(g, vmax, 0.0, seed=3, T=W + L)
    assert set(flux[W:].tolist()) == {min(N * vmax, L - N)}


def test_p0_stationary_patterns(orc):
    """Free flow: the state is rotated by vmax each step.  Jam: every car's
    gap becomes the gap of the car ahead (the gap sequence moves back by one)."""
    rng = np.random.default_rng(4)
    L, vmax = 600, 5
    g = _random_grid(rng, L, 80, vmax)          # 80*6 <= 600: free flow
    g, _ = orc.run_grid(g, vmax, 0.0, 1, 2000)
    g2, _ = orc.step_grid(g, vmax, 0.0, 1, 2000)
    assert np.array_equal(g2, np.roll(g, vmax))
    assert set(g[g != EMPTY].tolist()) == {vmax}
    g = _random_grid(rng, L, 250, vmax)         # 250*5 > 350: jammed
    g, _ = orc.run_grid(g, vmax, 0.0, 1, 2000)
    x, v = orc.grid_to_agent(g)
    x2, v2, _ = orc.step_agent(L, x, v, vmax, 0.0, 1, 2000)
    gaps = (np.roll(x, -1) - x - 1) % L
    gaps2 = (np.roll(x2, -1) - x2 - 1) % L
    assert np.array_equal(v2, gaps)             # every car drives its full gap
    assert np.array_equal(np.roll(v, -1), gaps) # a gap is the velocity of the car ahead
    assert np.array_equal(gaps2, np.roll(gaps, -1))


@pytest.mark.parametrize("L,vmax,v0", [(1000, 5, 0), (1000, 5, 3), (4, 5, 0), (2, 3, 1),
                                       (1, 4, 0)])
def test_single_car_closed_form(orc, L, vmax, v0):
    """One car alone (d = L): v_t = min(v0 + t, vmax, L - 1) with p = 0."""
    g = np.full(L, EMPTY, np.uint8)
    g[0] = min(v0, L - 1) if L > 1 else 0
    v, x = int(g[0]), 0
    for t in range(30):
        g, f = orc.step_grid(g, vmax, 0.0, 1, t)
        v = min(v + 1, vmax, L - 1)
        x = (x + v) % L
        assert f == v and g[x] == v and (g != EMPTY).sum() == 1


def test_single_car_mean_velocity_is_vmax_minus_p(orc):
    """A free car drives vmax with probability 1 - p and vmax - 1 with
    probability p (rule 3 accepts iff r < p): mean vmax - p within 5 sigma."""
    L, vmax, p, T = 100000, 5, 0.13, 20000
    g = np.full(L, EMPTY, np.uint8)
    g[0] = vmax
    _, flux = orc.run_grid(g, vmax, p, seed=11, T=T)
    mean = flux.mean()
    sigma = math.sqrt(p * (1 - p) / T)
    assert abs(mean - (vmax - p)) < 5 * sigma, mean


def _exact_chain_flux(L, N, vmax, p):
    """Stationary mean flux of the synchronous model on a tiny ring, by
    enumerating every state and every set of cars that draw r < p.  The rules
    are written out here from their text, in agent coordinates."""
    states = []
    for pos in itertools.combinations(range(L), N):
        for vs in itertools.product(range(vmax + 1), repeat=N):
            states.append(tuple(zip(pos, vs)))
    index = {s: i for i, s in enumerate(states)}
    n = len(states)
    P = np.zeros((n, n))
    J = np.zeros(n)
    for s in states:
        for slow in itertools.product((False, True), repeat=N):
            prob, new, flow = 1.0, [], 0
            for i, (x, v) in enumerate(s):
                d = L if N == 1 else (s[(i + 1) % N][0] - x) % L
                if v < vmax:          # rule 1
                    v += 1
                if v >= d:            # rule 2
                    v = d - 1
                if v > 0:             # rule 3
                    prob *= p if slow[i] else 1 - p
                    v -= slow[i]
                elif slow[i]:
                    prob = 0.0
                new.append(((x + v) % L, v))   # rule 4
                flow += v
            if prob:
                P[index[s], index[tuple(sorted(new))]] += prob
                J[index[s]] += prob * flow
    w, V = np.linalg.eig(P.T)
    pi = np.real(V[:, np.argmin(abs(w - 1))])
    pi /= pi.sum()
    return float(pi @ J)


@pytest.mark.parametrize("L,N,vmax,p", [(6, 2, 2, 0.3), (7, 3, 3, 0.5), (8, 3, 2, 0.4)])
def test_long_run_flux_matches_exact_markov_chain(orc, L, N, vmax, p):
    """The oracle's time-averaged flux on a tiny ring equals the exact
    stationary flux of the Markov chain (rules 2 and 3 in the paper's order;
    the swapped order gives a flux 0.45 to 1.9 higher on these rings)."""
    exact = _exact_chain_flux(L, N, vmax, p)
    g = np.full(L, EMPTY, np.uint8)
    g[np.arange(N) * (L // N)] = 0
    T = 200000
    _, flux = orc.run_grid(g, vmax, p, seed=2024, T=T)
    batch = flux[1000:].astype(np.float64).reshape(-1, 1000).mean(axis=1)
    se = batch.std(ddof=1) / math.sqrt(batch.size)
    assert abs(batch.mean() - exact) < 5 * se + 1e-3, (batch.mean(), exact, se)


@pytest.mark.parametrize("rho,p", [(0.1, 0.13), (0.3, 0.5), (0.5, 0.13), (0.7, 0.5)])
def test_vmax1_flux_matches_exact_parallel_update_result(orc, rho, p):
    """vmax = 1: the infinite-ring flux of the parallel update is
    J = (1 - sqrt(1 - 4 (1-p) rho (1-rho))) / 2 (Schreckenberg, Schadschneider,
    Nagel & Ito, Phys. Rev. E 51, 2939 (1995)); a ring of 2e4 cells matches
    it within 1 %."""
    L = 20000
    N = int(rho * L)
    g = orc.init_grid(L, N, 1, seed=8)
    _, flux = orc.run_grid(g, 1, p, seed=8, T=3000)
    J = flux[1000:].mean() / L
    exact = 0.5 * (1 - math.sqrt(1 - 4 * (1 - p) * rho * (1 - rho)))
    assert abs(J / exact - 1) < 0.01, (J, exact)


@pytest.mark.parametrize("seed", range(6))
def test_invariants_every_step(orc, seed):
    """Car count and order are kept, 0 <= v <= vmax, each car moves exactly its
    new v and never past its gap, and the flux is the total displacement; the
    grid and agent forms agree step by step."""
    rng = np.random.default_rng(seed)
    L = int(rng.integers(20, 400))
    N = int(rng.integers(1, L))
    vmax = int(rng.integers(1, 9))
    p = float(rng.choice([0.0, 0.13, 0.5, 0.9]))
    g = _random_grid(rng, L, N, vmax)
    x, v = orc.grid_to_agent(g)
    for t in range(60):
        g2, fg = orc.step_grid(g, vmax, p, seed, t)
        x2, v2, fa = orc.step_agent(L, x, v, vmax, p, seed, t)
        assert (g2 != EMPTY).sum() == N
        assert v2.max() <= vmax
        gap = L - 1 if N == 1 else (np.roll(x, -1) - x - 1) % L
        disp = (x2 - x) % L
        assert np.array_equal(disp, v2) and (disp <= gap).all()
        assert fg == fa == int(disp.sum())
        if N >= 2:
            assert int((np.diff(x2) < 0).sum()) <= 1   # one cyclic descent at most
        assert np.array_equal(orc.agent_to_grid(L, x2, v2), g2)
        g, x, v = g2, x2, v2


def test_thread_count_does_not_change_results(orc):
    """The all-core twin gives the serial result for every thread count."""
    L, N, vmax, p = 20000, 5000, 5, 0.13
    g0 = orc.init_grid(L, N, vmax, seed=21, init_v=1)
    ref, fref = orc.run_grid(g0, vmax, p, 21, 200, nthreads=1)
    for nt in (2, 3, 8):
        g, f = orc.run_grid(g0, vmax, p, 21, 200, nthreads=nt)
        assert np.array_equal(g, ref) and np.array_equal(f, fref)


def test_light_cone_window_matches_full_ring(orc):
    L, N, vmax, p, T = 50000, 12000, 5, 0.13, 80
    g = orc.init_grid(L, N, vmax, seed=6, init_v=1)
    full, _ = orc.run_grid(g, vmax, p, 6, T)
    for a, w in [(0, 100), (49990, 30), (12345, 777)]:
        win = orc.window_from_init(L, N, vmax, p, 6, T, a, w, init_v=1)
        assert np.array_equal(win, full[(a + np.arange(w)) % L])
    # a later start time: advance a segment cut from the full state at t0
    t0, T2 = T, 40
    a, w = 20000, 500
    R = T2 * vmax
    seg = full[(a - R + np.arange(w + 2 * R)) % L]
    out = orc.advance_segment(L, seg, vmax, p, 6, t0, T2, a, w)
    full2, _ = orc.run_grid(full, vmax, p, 6, T2, t0=t0)
    assert np.array_equal(out, full2[a:a + w])


# --------------------------------------------------------------------------- checksum
def test_fnv1a64_known_answers(orc):
    """The checksum of the full-size parity records is 64-bit FNV-1a: the
    published test vectors, and a hash continued over two pieces equals the
    hash of their concatenation."""
    with open(os.path.join(GOLDEN, "fnv1a64_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            text, want = line.rsplit(None, 1)
            data = np.frombuffer(text.strip('"').encode("ascii"), np.uint8)
            assert orc.fnv1a64(data) == int(want, 16)
    rng = np.random.default_rng(5)
    a = rng.integers(0, 256, 1000, dtype=np.uint8)
    assert orc.fnv1a64(a[600:], orc.fnv1a64(a[:600])) == orc.fnv1a64(a)
    assert orc.fnv1a64(np.array([1], np.uint64)) == orc.fnv1a64(np.array([1] + [0] * 7, np.uint8))


# --------------------------------------------------------------------------- shared stream
def test_minstd_rand_known_answer(orc):
    """The shared-stream generator is minstd_rand: its 10000th output from the
    default seed is the value the C++ standard requires."""
    with open(os.path.join(GOLDEN, "minstd_rand_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            seed, n, want = (int(v) for v in line.split())
            x = orc.mlcg_seed(seed)
            for _ in range(n):
                x = orc.mlcg_next(x)
            assert x == want


def test_mlcg_closed_form_state(orc):
    """x_n = x0 a^n mod m is the closed form of a multiplicative LCG: a stream
    started from that state (Python's exact modular power) continues exactly
    as the stream advanced draw by draw, so tests may start it far along."""
    m = 2**31 - 1
    x = orc.mlcg_seed(11)
    for _ in range(777):
        x = orc.mlcg_next(x)
    assert x == orc.mlcg_seed(11) * pow(48271, 777, m) % m
    rng = np.random.default_rng(4)
    L, N = 300, 70
    g = _random_grid(rng, L, N, 4)
    xs, vs = orc.grid_to_agent(g)
    a = orc.run_agent_mlcg(L, xs, vs, 4, 0.3, 11, 12, t0=9)
    b = orc.run_agent_mlcg(L, xs, vs, 4, 0.3, 11, 12,
                           state0=orc.mlcg_seed(11) * pow(48271, 9 * N, m) % m)
    for u, w in zip(a, b):
        assert np.array_equal(u, w)


def test_mlcg_threshold_is_ceil_p_m(orc):
    m = 2**31 - 1
    for p in (0.0, 0.13, 0.25, 0.5, 0.999):
        assert orc.mlcg_threshold(p) == math.ceil(Fraction(p) * m)
    assert orc.mlcg_seed(0) == 1 and orc.mlcg_seed(m) == 1 and orc.mlcg_seed(5) == 5


def test_stream_mode_without_rule3_equals_keyed_mode(orc):
    """With p = 0 no draw matters: the shared-stream agent run equals the keyed
    agent run step for step."""
    L, N, vmax = 3000, 700, 5
    g = orc.init_grid(L, N, vmax, seed=4, init_v=1)
    x, v = orc.grid_to_agent(g)
    xa, va, fa = orc.run_agent(L, x, v, vmax, 0.0, 4, 300)
    xb, vb, fb = orc.run_agent_mlcg(L, x, v, vmax, 0.0, 4, 300)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(fa, fb)


def test_stream_mode_invariants_and_rate(orc):
    """Invariants hold with the shared stream, and a free car drives vmax - p
    on average (the stream's numbers are uniform)."""
    L, vmax, p, T = 100000, 5, 0.13, 20000
    xs, vs, flux = orc.run_agent_mlcg(L, np.array([0]), np.array([vmax]), vmax, p, 3, T)
    mean = flux.mean()
    assert abs(mean - (vmax - p)) < 5 * math.sqrt(p * (1 - p) / T)
    rng = np.random.default_rng(2)
    L, N = 500, 120
    g = _random_grid(rng, L, N, vmax)
    x, v = orc.grid_to_agent(g)
    for t in range(30):
        x2, v2, f = orc.run_agent_mlcg(L, x, v, vmax, 0.3, 9, 1, t0=t)
        gap = (np.roll(x, -1) - x - 1) % L
        disp = (x2 - x) % L
        assert np.array_equal(disp, v2) and (disp <= gap).all() and int(f[0]) == int(disp.sum())
        assert len(set(x2.tolist())) == N
        x, v = x2, v2
