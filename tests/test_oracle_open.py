"""Pins of the open-road oracle (the boundary-condition variation of the paper's
"Variations" section) against facts that do not come from the oracle itself.

Readings of the variation, written out in the oracle: cars drive from cell 0
toward cell L-1; at step t one gate draw decides whether a car enters cell 0
(probability alpha, only if the cell was empty at the start of the step) and
whether the exit is closed (probability 1 - beta: a stopped car in cell L for
that step); a car whose move ends at or beyond L leaves; F(t) sums the
velocities of all cars that were on the road at the start of the step.

What fixes the expected values:
  - an exact Markov chain over every state of tiny roads, written here from the
    rule text in agent coordinates (catches a wrong gate probability, a wrong
    entry condition, a car entering with the wrong velocity, a mis-placed
    exit obstacle);
  - for vmax = 1 the model is the totally asymmetric exclusion process with
    parallel update, whose exact currents in the low-density, high-density and
    maximal-current phases are known (Evans, Rajewsky & Speer, J. Stat. Phys.
    95, 45 (1999); de Gier & Nienhuis, Phys. Rev. E 59, 4899 (1999));
  - the deterministic free-flow closed form for p = 0, beta = 1 (every car
    holds cell 0 for exactly one step and then accelerates undisturbed);
  - the absorbing states of alpha = 0 (the road drains) and beta = 0 (the road
    fills with stopped cars);
  - conservation and the per-car rules at every step;
  - away from the ends the open road is the ring (pinned separately) cell by
    cell, and a light-cone window equals the full road.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

EMPTY = 0xFF


# --------------------------------------------------------------------------- gate
@pytest.mark.parametrize("a", [0.0, 2.0 ** -33, 1e-9, 0.13, 0.5, 0.999999999, 1.0])
def test_gate_threshold_is_floor_a_times_2_32(orc, a):
    want = math.floor(Fraction(a) * 2 ** 32)
    assert orc.gate_threshold(a) == want
    assert 0 <= want <= 2 ** 32


def test_gate_words_rate(orc):
    """The two gate words are uniform: P(word < floor(a 2^32)) = a within 5 sigma."""
    T = 40000
    w = np.array([orc.gate_words(5, t) for t in range(T)], dtype=np.uint64)
    for a in (0.1, 0.5, 0.8):
        thr = orc.gate_threshold(a)
        for col in (0, 1):
            rate = float((w[:, col] < thr).mean())
            assert abs(rate - a) < 5 * math.sqrt(a * (1 - a) / T), (a, col, rate)
    assert not np.array_equal(w[:, 0], w[:, 1])


# --------------------------------------------------------------------------- exact chain
def _exact_open_chain(L, vmax, p, alpha, beta):
    """Stationary means of (F, entries, exits) on an open road of L cells, by
    enumerating every state, gate outcome and set of cars that draw r < p."""
    cells = [None] + list(range(vmax + 1))        # None = empty, else v
    states = list(itertools.product(cells, repeat=L))
    index = {s: i for i, s in enumerate(states)}
    n = len(states)
    P = np.zeros((n, n))
    EF, EIN, EOUT = np.zeros(n), np.zeros(n), np.zeros(n)
    for s in states:
        cars = [(x, v) for x, v in enumerate(s) if v is not None]
        for enter, closed in itertools.product((False, True), repeat=2):
            pg = (alpha if enter else 1 - alpha) * ((1 - beta) if closed else beta)
            if pg == 0.0:
                continue
            for slow in itertools.product((False, True), repeat=len(cars)):
                prob, new, flow, out = pg, [None] * L, 0, 0
                for i, (x, v) in enumerate(cars):
                    if i + 1 < len(cars):
                        d = cars[i + 1][0] - x            # the car in front
                    elif closed:
                        d = L - x                         # the stopped car in cell L
                    else:
                        d = vmax + 1                      # open road ahead
                    v = min(v + 1, vmax)                  # rule 1
                    v = min(v, d - 1)                     # rule 2
                    if v > 0:                             # rule 3
                        prob *= p if slow[i] else 1 - p
                        v -= slow[i]
                    elif slow[i]:
                        prob = 0.0
                    flow += v
                    if x + v < L:                         # rule 4
                        new[x + v] = v
                    else:
                        out += 1
                came = 0
                if enter and s[0] is None:
                    new[0] = 0
                    came = 1
                if prob:
                    j = index[tuple(new)]
                    P[index[s], j] += prob
                    EF[index[s]] += prob * flow
                    EIN[index[s]] += prob * came
                    EOUT[index[s]] += prob * out
    w, V = np.linalg.eig(P.T)
    pi = np.real(V[:, np.argmin(abs(w - 1))])
    pi /= pi.sum()
    return float(pi @ EF), float(pi @ EIN), float(pi @ EOUT)


@pytest.mark.parametrize("L,vmax,p,alpha,beta", [
    (3, 2, 0.3, 0.6, 0.4),
    (4, 1, 0.5, 0.3, 0.7),
    (3, 3, 0.13, 0.9, 0.2),
    (4, 2, 0.0, 0.5, 0.5),
    (2, 2, 0.25, 1.0, 0.6),
])
def test_long_run_means_match_exact_markov_chain(orc, L, vmax, p, alpha, beta):
    ef, ein, eout = _exact_open_chain(L, vmax, p, alpha, beta)
    assert abs(ein - eout) < 1e-9        # the chain itself conserves cars
    T = 200000
    g = np.full(L, EMPTY, np.uint8)
    _, flux, ent, lft = orc.run_open(g, vmax, p, alpha, beta, seed=77, T=T)
    for series, exact in ((flux, ef), (ent, ein), (lft, eout)):
        batch = series[1000:].astype(np.float64).reshape(-1, 1000).mean(axis=1)
        se = batch.std(ddof=1) / math.sqrt(batch.size)
        assert abs(batch.mean() - exact) < 5 * se + 1e-3, (batch.mean(), exact, se)


# --------------------------------------------------------------------------- vmax = 1: TASEP
def _tasep_current(alpha, beta_eff, q):
    """Exact bulk current of the parallel-update TASEP with entry alpha, exit
    beta_eff and hop probability q."""
    ac = 1 - math.sqrt(1 - q)
    if alpha <= beta_eff and alpha < ac:
        return alpha * (q - alpha) / (q - alpha ** 2)          # low density (and coexistence)
    if beta_eff < alpha and beta_eff < ac:
        return beta_eff * (q - beta_eff) / (q - beta_eff ** 2)  # high density
    return (1 - math.sqrt(1 - q)) / 2                           # maximal current


@pytest.mark.parametrize("alpha,beta,p,tol", [
    (0.2, 0.9, 0.25, 0.0),    # low density
    (0.9, 0.3, 0.25, 0.0),    # high density
    (0.6, 0.2, 0.13, 0.0),    # high density
    (0.3, 0.3, 0.0, 0.0),     # coexistence line (alpha = beta (1 - p))
    (0.9, 1.0, 0.25, 0.01),   # maximal current: 1/L finite-size excess allowed
])
def test_vmax1_current_is_parallel_tasep(orc, alpha, beta, p, tol):
    """vmax = 1: mean F / L is the TASEP current (every one of the L bonds,
    the exit included, carries it), with exit probability beta (1 - p) since
    a car at the exit still obeys rule 3."""
    L = 200
    q = 1 - p
    g = np.full(L, EMPTY, np.uint8)
    g, _, _, _ = orc.run_open(g, 1, p, alpha, beta, seed=7, T=20000)
    _, flux, ent, lft = orc.run_open(g, 1, p, alpha, beta, seed=7, T=200000, t0=20000)
    batch = flux.astype(np.float64).reshape(40, -1).mean(axis=1) / L
    J, se = batch.mean(), batch.std(ddof=1) / math.sqrt(batch.size)
    want = _tasep_current(alpha, beta * q, q)
    assert abs(J - want) < 5 * se + tol * want, (J, want, se)
    # the same current enters and leaves
    assert abs(ent.mean() - J) < 5 * se + tol * want + 1e-3
    assert abs(lft.mean() - J) < 5 * se + tol * want + 1e-3


# --------------------------------------------------------------------------- p = 0 closed forms
def _trajectory(vmax, L):
    """Ages a = 1, 2, ... of a car in free flow: (velocity min(a, vmax), start
    position X(a - 1)) while it starts the step on the road."""
    out, X, a = [], 0, 1
    while X < L:
        v = min(a, vmax)
        out.append((v, X))
        X += v
        a += 1
    return out


@pytest.mark.parametrize("vmax", [1, 2, 3, 5, 8])
def test_p0_alpha1_beta1_is_deterministic_free_flow(orc, vmax):
    """alpha = beta = 1, p = 0 from the empty road: a car enters at every even
    step (cell 0 is held for exactly one step), each car has v = min(age, vmax),
    and F(t) is the sum of min(a, vmax) over the ages a = t, t-2, ... >= 1 whose
    car still starts the step on the road."""
    L, T = 97, 400
    g = np.full(L, EMPTY, np.uint8)
    gT, flux, ent, lft = orc.run_open(g, vmax, 0.0, 1.0, 1.0, seed=3, T=T)
    traj = _trajectory(vmax, L)
    for t in range(T):
        assert ent[t] == (t % 2 == 0)
        want = sum(v for a, (v, _) in enumerate(traj, start=1) if a <= t and (t - a) % 2 == 0)
        assert flux[t] == want, (t, flux[t], want)
    assert lft.sum() == ent.sum() - int((gT != EMPTY).sum())


@pytest.mark.parametrize("vmax,alpha", [(1, 0.3), (3, 0.5), (5, 0.2), (8, 0.7)])
def test_p0_beta1_entry_rate_closed_form(orc, vmax, alpha):
    """p = 0, beta = 1: entries form a renewal process (one blocked step, then
    a geometric number of tries), rate alpha / (1 + alpha); every car makes the
    free-flow trajectory, so mean F = rate x (distance a car covers until it
    leaves)."""
    L, T = 60, 200000
    g = np.full(L, EMPTY, np.uint8)
    _, flux, ent, _ = orc.run_open(g, vmax, 0.0, alpha, 1.0, seed=9, T=T)
    rate = alpha / (1 + alpha)
    cover = sum(v for v, _ in _trajectory(vmax, L))
    mu, var = 1 + 1 / alpha, (1 - alpha) / alpha ** 2       # cycle length mean, variance
    se_rate = math.sqrt(var / mu ** 3 / T)
    assert abs(ent.mean() - rate) < 5 * se_rate
    assert abs(flux[1000:].mean() / cover - rate) < 5 * se_rate + 2e-3


def test_alpha0_drains_and_beta0_fills(orc):
    L, N, vmax = 300, 90, 5
    g0 = orc.init_grid(L, N, vmax, seed=4, init_v=1)
    g, flux, ent, lft = orc.run_open(g0, vmax, 0.3, 0.0, 0.7, seed=4, T=5000)
    assert (g == EMPTY).all() and ent.sum() == 0 and lft.sum() == N and flux[-1] == 0
    g, flux, ent, lft = orc.run_open(g0, vmax, 0.3, 0.6, 0.0, seed=4, T=20000)
    assert (g == 0).all(), "a closed exit fills the road with stopped cars"
    assert lft.sum() == 0 and ent.sum() == L - N and flux[-1] == 0


# --------------------------------------------------------------------------- per step
@pytest.mark.parametrize("seed", range(6))
def test_invariants_every_step(orc, seed):
    """Per step: cars in + entered - left = cars out; cars keep their order;
    each remaining car moves exactly its new v, which is at most
    min(v + 1, vmax) and below its gap; the cars that left are the front
    ones; a new car sits in cell 0 with v = 0 only if that cell was empty;
    F is the remaining cars' moves plus at least the distance of the leavers
    to L."""
    rng = np.random.default_rng(100 + seed)
    L = int(rng.integers(5, 300))
    vmax = int(rng.integers(0, 9))
    p = float(rng.choice([0.0, 0.13, 0.5]))
    alpha, beta = float(rng.choice([0.0, 0.4, 1.0])), float(rng.choice([0.0, 0.5, 1.0]))
    N = int(rng.integers(0, L + 1))
    g = orc.init_grid(L, N, vmax, seed=seed, init_v=1)
    for t in range(120):
        g2, f, e, l = orc.step_open(g, vmax, p, alpha, beta, seed, t)
        x, v = np.flatnonzero(g != EMPTY), g[g != EMPTY].astype(int)
        x2, v2 = np.flatnonzero(g2 != EMPTY), g2[g2 != EMPTY].astype(int)
        assert x2.size == x.size + e - l
        assert e in (0, 1) and (e == 0 or (g[0] == EMPTY and g2[0] == 0))
        if e:
            x2, v2 = x2[1:], v2[1:]
        stay = x.size - l
        assert np.array_equal(x2 - x[:stay], v2)
        assert (v2 <= np.minimum(v[:stay] + 1, vmax)).all()
        ahead = np.append(x[1:], L + vmax + 1)[:stay]
        assert (x[:stay] + v2 < ahead).all()
        assert (x[stay:] + vmax >= L).all()
        assert f >= v2.sum() + (L - x[stay:]).sum()
        assert f <= v2.sum() + vmax * l
        g = g2


# --------------------------------------------------------------------------- against the ring
def test_interior_equals_the_ring(orc):
    """Cells at least T vmax away from both ends never feel the boundaries:
    after T steps they equal the ring's cells (same placement, same draws)."""
    L, N, vmax, p, T = 5000, 1200, 5, 0.13, 60
    g0 = orc.init_grid(L, N, vmax, seed=12, init_v=1)
    ring, _ = orc.run_grid(g0, vmax, p, 12, T)
    road, _, _, _ = orc.run_open(g0, vmax, p, 0.5, 0.5, seed=12, T=T)
    r = T * vmax
    assert np.array_equal(road[r:L - r], ring[r:L - r])
    assert not np.array_equal(road[:r], ring[:r]) or not np.array_equal(road[L - r:], ring[L - r:])


def test_light_cone_window_matches_full_road(orc):
    L, N, vmax, p, T = 20000, 4000, 5, 0.13, 70
    alpha, beta = 0.45, 0.35
    g0 = orc.init_grid(L, N, vmax, seed=31, init_v=1)
    full, _, _, _ = orc.run_open(g0, vmax, p, alpha, beta, seed=31, T=T)
    for a, w in [(0, 100), (L - 40, 40), (7777, 555), (100, 300), (L - 500, 200)]:
        win = orc.open_window_from_init(L, N, vmax, p, alpha, beta, 31, T, a, w, init_v=1)
        assert np.array_equal(win, full[a:a + w]), (a, w)
