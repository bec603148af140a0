"""Write tests/golden/fullsize.json: checksums of the whole final state and the
whole flux log of the full-size one-road workloads, computed by the oracle
alone.

    python tests/golden/make_fullsize.py [workload ...] [--threads N]

Workloads (the sizes of the benchmark's one-road workloads):
  large_ring    grid form, L = 2^30, N = floor(0.2 L), vmax 5, p 0.13, seed 1,
                v0 uniform, T = 1000: the all-core OpenMP twin of the grid step
                (bit-identical to the serial oracle for every thread count,
                which the oracle's own tests check);
  agent_ring    L = 2^28, N = 2^26, vmax 5, p 0.25, seed 1, v0 uniform,
                T = 1000, keyed draws: the same twin (the final state of the
                agent form is the same grid by construction of the method);
  agent_stream  the agent ring with the shared minstd stream: the serial
                stream oracle, one draw after another;
  open_road     the large ring opened at both ends (alpha 0.3, beta 0.9):
                the serial open-road oracle (hours on one core);
  ensemble      the benchmark's 4096-replica ensemble (T = 5000, flux summed
                from t = 1000): the serial oracle per replica, replicas spread
                over worker processes.  The road checksum runs over every
                replica's final road back to back in replica order (the layout
                of a whole-batch snapshot), the flux checksum over the uint64
                flux sums of all replicas.

For each, the record holds the 64-bit FNV-1a of the final grid (L bytes,
0xFF = empty, else v) and of the flux log (T uint64, little-endian), plus the
car count, F(T-1) and the sum of the log as readable cross-checks.  Only
oracle/ is called; the workload parameters are read from the package's
workload module, which holds parameter draws and no model arithmetic.
Existing records of other workloads are kept.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import fcntl
import importlib.util
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402

OUT = os.path.join(HERE, "fullsize.json")


def _workloads():
    path = os.path.join(ROOT, "paper_2309_14311_amd", "workloads.py")
    spec = importlib.util.spec_from_file_location("nasch_workloads", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _record(cfg, grid, flux, how, seconds):
    occ = grid != oracle.EMPTY
    return {
        "L": cfg["L"], "N": cfg["N"], "vmax": cfg["vmax"], "p": cfg["p"], "seed": cfg["seed"],
        "replica": cfg["replica"], "init_v": cfg["init_v"], "T": cfg["T"],
        **({"alpha": cfg["alpha"], "beta": cfg["beta"]} if "alpha" in cfg else {}),
        "grid_fnv1a64": f"{oracle.fnv1a64(grid):016x}",
        "flux_fnv1a64": f"{oracle.fnv1a64(flux.astype('<u8')):016x}",
        "cars_final": int(occ.sum()),
        "flux_last": int(flux[-1]),
        "flux_sum": int(flux.astype(np.uint64).sum()),
        "oracle": how,
        "oracle_seconds": round(seconds, 1),
    }


def _ensemble_replica(r):
    """Final road and flux sum (t >= warm-up) of one ensemble replica."""
    g0 = oracle.init_grid(r["L"], r["N"], r["vmax"], r["seed"], replica=r["replica"],
                          init_v=r["init_v"])
    g, flux = oracle.run_grid(g0, r["vmax"], r["p"], r["seed"], r["T"], replica=r["replica"])
    return g.tobytes(), int(flux[r["warmup"]:].astype(np.uint64).sum())


def run_ensemble(wl, workers):
    t0 = time.time()
    reps = wl.ensemble(4096, seed=1, T=5000, warmup=1000)
    h = oracle.FNV64_OFFSET
    sums = np.zeros(len(reps), np.uint64)
    with cf.ProcessPoolExecutor(workers) as ex:
        for i, (g, fsum) in enumerate(ex.map(_ensemble_replica, reps, chunksize=4)):
            h = oracle.fnv1a64(np.frombuffer(g, np.uint8), h)
            sums[i] = fsum
    return {
        "replicas": len(reps), "seed": 1, "T": 5000, "warmup": 1000,
        "cells": int(sum(r["L"] for r in reps)),
        "grid_fnv1a64": f"{h:016x}",
        "flux_sums_fnv1a64": f"{oracle.fnv1a64(sums.astype('<u8')):016x}",
        "flux_sums_total": int(sums.sum()),
        "oracle": f"oracle.run_grid per replica, serial, {workers} worker processes",
        "oracle_seconds": round(time.time() - t0, 1),
    }


def run(name, wl, threads):
    t0 = time.time()
    if name == "ensemble":
        return run_ensemble(wl, threads)
    if name in ("large_ring", "agent_ring"):
        cfg = wl.LARGE_RING if name == "large_ring" else wl.AGENT_RING
        g = oracle.init_grid(cfg["L"], cfg["N"], cfg["vmax"], cfg["seed"],
                             replica=cfg["replica"], init_v=cfg["init_v"])
        g, flux = oracle.run_grid(g, cfg["vmax"], cfg["p"], cfg["seed"], cfg["T"],
                                  replica=cfg["replica"], nthreads=threads)
        how = f"oracle.run_grid, OpenMP twin, {threads} threads"
    elif name == "agent_stream":
        cfg = wl.AGENT_RING
        g0 = oracle.init_grid(cfg["L"], cfg["N"], cfg["vmax"], cfg["seed"],
                              replica=cfg["replica"], init_v=cfg["init_v"])
        x, v = oracle.grid_to_agent(g0)
        del g0
        x, v, flux = oracle.run_agent_mlcg(cfg["L"], x, v, cfg["vmax"], cfg["p"], cfg["seed"],
                                           cfg["T"])
        g = oracle.agent_to_grid(cfg["L"], x, v)
        how = "oracle.run_agent_mlcg, serial shared minstd stream"
    elif name == "open_road":
        cfg = wl.OPEN_ROAD
        g = oracle.init_grid(cfg["L"], cfg["N"], cfg["vmax"], cfg["seed"],
                             replica=cfg["replica"], init_v=cfg["init_v"])
        g, flux, _, _ = oracle.run_open(g, cfg["vmax"], cfg["p"], cfg["alpha"], cfg["beta"],
                                        cfg["seed"], cfg["T"], replica=cfg["replica"])
        how = "oracle.run_open, serial"
    else:
        raise SystemExit(f"unknown workload {name}")
    return _record(cfg, g, flux, how, time.time() - t0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="*",
                    default=["agent_ring", "large_ring", "agent_stream"])
    ap.add_argument("--threads", type=int, default=oracle.num_threads_available())
    args = ap.parse_args()
    wl = _workloads()
    for name in args.workloads:
        rec = run(name, wl, args.threads)
        # several runs of this script may finish at once: merge under a lock
        with open(OUT + ".lock", "w") as lk:
            fcntl.flock(lk, fcntl.LOCK_EX)
            data = {}
            if os.path.exists(OUT):
                with open(OUT) as f:
                    data = json.load(f)
            data[name] = rec
            with open(OUT + ".tmp", "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
                f.write("\n")
            os.replace(OUT + ".tmp", OUT)
        print(name, json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
