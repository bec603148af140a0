"""Seeded synthetic workloads shaped like the paper's (its reference case is 200 cars
on L = 1000, p = 0.13, vmax = 5).  Parameter draws only: nothing here computes
any part of the model.  Both the GPU library and the CPU oracle are driven from
these dictionaries.
"""
from __future__ import annotations

import math

import numpy as np

# The paper's reference test case (Figure 1 caption): 200 cars, L = 1000,
# p = 0.13, vmax = 5; T and the seed are chosen here.
REFERENCE = dict(L=1000, N=200, vmax=5, p=0.13, seed=1, replica=0, init_v=0, T=2000)

# One large ring (grid form), density 0.2, N = floor(0.2 L).
LARGE_RING = dict(L=2**30, N=int(math.floor(0.2 * 2**30)), vmax=5, p=0.13, seed=1, replica=0,
                  init_v=1, T=1000)

# Agent form: 2^26 cars on 2^28 cells.
AGENT_RING = dict(L=2**28, N=2**26, vmax=5, p=0.25, seed=1, replica=0, init_v=1, T=1000)

# The large ring's road opened at both ends: entry probability 0.3, exit 0.9.
OPEN_ROAD = dict(L=2**30, N=int(math.floor(0.2 * 2**30)), vmax=5, p=0.13, seed=1, replica=0,
                 init_v=1, T=1000, alpha=0.3, beta=0.9)


def ensemble(n_replicas: int = 4096, seed: int = 1, T: int = 5000, warmup: int = 1000,
             L_lo_exp: float = 3.0, L_hi_exp: float = 6.0) -> list[dict]:
    """Fundamental-diagram ensemble: replica r draws L log-uniform in
    [10^L_lo_exp, 10^L_hi_exp], density uniform in [0.05, 0.6], p from
    {0, 0.13, 0.25, 0.5}, vmax uniform in 1..8.  Every replica uses the
    ensemble seed with its own Philox stream id (replica = r)."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_replicas):
        u = rng.random()
        L = int(round(10 ** (L_lo_exp + (L_hi_exp - L_lo_exp) * u)))
        rho = float(rng.uniform(0.05, 0.6))
        p = float(rng.choice([0.0, 0.13, 0.25, 0.5]))
        vmax = int(rng.integers(1, 9))
        out.append(dict(L=L, N=int(math.floor(rho * L)), vmax=vmax, p=p, seed=seed, replica=r,
                        init_v=1, T=T, warmup=warmup, rho=rho))
    return out


def requests(n: int = 2000, seed: int = 7, L_exp=(3.0, 7.0), T_exp=(2.0, 4.0),
             rate: float = 100.0) -> list[dict]:
    """Serving stream: Poisson arrivals at `rate` per second; L log-uniform in
    [10^3, 10^7], density uniform in [0.05, 0.6], p uniform in [0, 0.5],
    vmax uniform in 1..8, T log-uniform in [10^2, 10^4], request seed 1000 + i."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        L = int(round(10 ** rng.uniform(*L_exp)))
        rho = float(rng.uniform(0.05, 0.6))
        p = float(rng.uniform(0.0, 0.5))
        vmax = int(rng.integers(1, 9))
        T = int(round(10 ** rng.uniform(*T_exp)))
        out.append(dict(arrival=t, L=L, N=int(math.floor(rho * L)), vmax=vmax, p=p,
                        seed=1000 + i, replica=0, init_v=1, T=T))
    return out


def open_ensemble(n_replicas: int = 4096, seed: int = 1, T: int = 5000, warmup: int = 1000):
    """The ensemble's roads opened at both ends, for a parameter study over the
    gates: entry and exit probabilities drawn uniformly from [0, 1]."""
    reps = ensemble(n_replicas, seed=seed, T=T, warmup=warmup)
    rng = np.random.default_rng(seed + 7919)
    for r in reps:
        r["boundary"] = "open"
        r["alpha"] = float(rng.random())
        r["beta"] = float(rng.random())
    return reps
