#!/usr/bin/env python
"""Benchmark of the NaSch hot path on one MI355X.

Default workload (the metric's): the fundamental-diagram ensemble, 4096 rings
with L log-uniform in [1e3, 1e6], density in [0.05, 0.6], p in {0, .13, .25, .5},
vmax in 1..8, T = 5000 steps (1000 warm-up), all advanced together by the
batched temporal-blocked grid kernel.  One benchmark step = one pass of the
whole hot path over that batch: initial placement, T time steps of every
replica, and the per-replica flux sums copied to the host.  Inputs are
resident in HBM when the timed region starts.

Besides the JSON line's `value` (batched cell-updates/s) it reports the same
work run as the plain one-replica-per-launch loop, the roofline of the
dominant kernel, and the CPU oracle timed on the host (`cpu_baseline`).

Other workloads (`--workload large_ring|agent|reference`) measure the single
large ring (k-step vs one-step), the agent form and the paper's reference case.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

try:
    _CPUS_AT_START = len(os.sched_getaffinity(0))
except (AttributeError, OSError):
    _CPUS_AT_START = os.cpu_count() or 1

HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
BYTES_PER_CELL_UPDATE = 2.0  # read 1 B + write 1 B of uint8 state per cell per step
# 32-bit vector ALU, lane-operations/s.  gfx950 issues a wave64 add, xor or
# three-input bitwise op (v_bitop3_b32) in 2 cycles per SIMD, the datapath of the
# published 157.3 TFLOP/s fp32 vector peak: 256 CU x 4 SIMD x 32 lanes x 2.4 GHz.
# Shifts, funnel shifts, byte permutes, popcounts, multiplies (v_mad_u64_u32),
# 64-bit adds and DPP lane moves take 4 cycles, half that rate
# (libnasch_probe measures both on the device, with the clock).
VALU_PEAK = 256 * 4 * 32 * 2.4e9
VALU_PEAK_4CYCLE = VALU_PEAK / 2
CSRC = os.path.join(ROOT, "paper_2309_14311_amd", "csrc")
# the sources the k-step kernel is compiled from
KSTEP_SRCS = [os.path.join(CSRC, f) for f in ("grid_kstep.hip", "grid_common.hpp",
                                               "bitplanes.hpp", "nasch_device.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_grid_kstep_ensemble.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_grid_kstep_ensemble.json")


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def kstep_ops_per_cell_update(vmax, p):
    """Algorithmic operations of the bit-sliced update, per cell-update: per 32-cell
    word and step, rules 1-2 take vmax funnel shifts, vmax - 1 ORs and vmax AND-NOTs
    (3 vmax - 1), rule 3 vmax selects, rule 4 vmax class masks, vmax shifts and
    vmax ORs, and F(t) vmax popcounts: 8 vmax in all (with the slow-mask AND).  When
    p > 0 the word's rule-3 block draw adds one Philox4x32-10 call (10 rounds of two
    32x32->64 multiplies and two three-input XORs: 40) and the 4-bit comparison (4).
    Tied cars (1 in 16 moving cars when p has bits below 2^-4) draw once more each;
    their number depends on the state, so they are not counted."""
    thr = int(p * 2.0 ** 32)
    return (8 * vmax + (44 if thr > 0 else 0)) / 32.0


def _src_hash(paths):
    """First 16 hex digits of the sha256 of the concatenated sources."""
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _profile_record(path, k, q):
    """The committed counter record of the k-step kernel at (k, q), if it was
    taken on the current kernel sources; else None."""
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_src_sha256_16") != _src_hash(KSTEP_SRCS):
        return None
    for r in rec.get("records", []):
        if r.get("k") == k and r.get("q") == q:
            return r
    return None


def _traffic(k, q, launch_cell_updates):
    """Counter-measured HBM bytes of one launch of the k-step kernel, scaled from
    the committed counter summary (bytes per cell-update at the same (k, q))."""
    r = _profile_record(TRAFFIC_FILE, k, q)
    return None if r is None else r["bytes_per_cell_update"] * launch_cell_updates


def _issued_valu(k, q, launch_cell_updates):
    """VALU lane-instructions one launch of the k-step kernel issues
    (SQ_INSTS_VALU x 64 from the committed counter summary, per cell-update)."""
    r = _profile_record(VALU_FILE, k, q)
    return None if r is None else r["valu_lane_instructions_per_cell_update"] * launch_cell_updates


def measure_valu():
    """The vector-ALU ceilings measured live (libnasch_probe): lane-ops/s of a
    2-cycle instruction (v_bitop3_b32) and of a 4-cycle one (v_alignbit_b32),
    each with the shader clock during its run."""
    from paper_2309_14311_amd import native
    out = {}
    for kind in ("bitop3", "alignbit"):
        r = native.probe_valu(kind, 4096, 4000)
        out[kind] = {"lane_ops_per_s": r["lane_ops_per_s"], "sclk_ghz": r["sclk_hz"] / 1e9,
                     "frac_of_derived": r["lane_ops_per_s"] / (
                         VALU_PEAK if kind == "bitop3" else VALU_PEAK_4CYCLE)}
    return out


def _host_info():
    """CPU model, sockets, physical cores and logical CPUs of the host."""
    model, cores = None, set()
    try:
        with open("/proc/cpuinfo") as f:
            pid = None
            for line in f:
                key, _, val = line.partition(":")
                key, val = key.strip(), val.strip()
                if key == "model name" and model is None:
                    model = val
                elif key == "physical id":
                    pid = val
                elif key == "core id":
                    cores.add((pid, val))
    except OSError:
        pass
    return {"cpu": model, "sockets": len({p for p, _ in cores}) or None,
            "physical_cores": len(cores) or None, "logical_cpus": os.cpu_count()}


def _cpu_threads():
    """Threads of the all-core oracle: one per physical core (no SMT), within the
    CPUs this process could use when it started (an OpenMP runtime that binds
    its threads narrows the affinity later)."""
    phys = _host_info()["physical_cores"] or os.cpu_count() or 1
    return max(1, min(phys, _CPUS_AT_START))


def _median_of_chunks(advance, cells, warm_s, chunk_s, repeats=3):
    """The oracle's step loop timed the way the CPU baseline protocol asks:
    untimed warm-up steps (1, 2, 4, ... at a time) until warm_s seconds have
    passed, which also gives the rate, then `repeats` consecutive chunks of
    timed steps, each sized for about chunk_s seconds at that rate.  Returns
    (median chunk rate in cell-updates/s, the chunk rates, warm-up steps, chunk
    steps).  advance(t0, steps) runs the sample."""
    t, n, spent, rate = 0, 1, 0.0, 0.0
    while spent < warm_s:
        t0 = time.perf_counter()
        advance(t, n)
        dt = time.perf_counter() - t0
        spent += dt
        rate = cells * n / max(dt, 1e-9)
        t += n
        n *= 2
    chunk = max(1, int(round(rate * chunk_s / cells)))
    warm, rates = t, []
    for _ in range(repeats):
        t0 = time.perf_counter()
        advance(t, chunk)
        rates.append(cells * chunk / (time.perf_counter() - t0))
        t += chunk
    return float(np.median(rates)), rates, warm, chunk


def _ordinal(m):
    """1st, 2nd, 3rd, 4th, ..., 11th, 12th, 13th, ..., 21st, ..."""
    suffix = "th" if m % 100 in (11, 12, 13) else {1: "st", 2: "nd", 3: "rd"}.get(m % 10, "th")
    return f"{m}{suffix}"


def _stratified(reps, target_cells):
    """Every m-th replica in order of L (all sizes represented), m chosen so the
    sample holds about target_cells cells."""
    order = sorted(range(len(reps)), key=lambda i: reps[i]["L"])
    total = sum(r["L"] for r in reps)
    m = min(len(order), max(1, int(round(total / max(1.0, target_cells)))))
    return [reps[i] for i in order[m // 2::m]], m


def cpu_baseline_ensemble(reps, T, budget_s=15.0):
    """The oracle on a bounded, L-stratified sample of the ensemble: the all-core
    OpenMP twin on one thread per physical core (OMP_PLACES=cores,
    OMP_PROC_BIND=spread), warm-up steps for about a fifth of the time budget,
    then the median rate of 3 timed chunks of steps, each about a quarter of it
    (the reported value); the serial oracle the same way on a smaller sample.  The sample's rate stands for the whole workload, whose
    time is extrapolated from it (labelled as such)."""
    import oracle
    threads = _cpu_threads()
    total = sum(r["L"] for r in reps)

    def run(sample, nthreads, warm, chunk):
        grids = [oracle.init_grid(r["L"], r["N"], r["vmax"], r["seed"], replica=r["replica"],
                                  init_v=r["init_v"]) for r in sample]

        def advance(t0, steps):
            for i, r in enumerate(sample):
                if r.get("boundary") == "open":
                    grids[i] = oracle.run_open(grids[i], r["vmax"], r["p"], r["alpha"],
                                               r["beta"], r["seed"], steps, t0=t0,
                                               replica=r["replica"])[0]
                else:
                    grids[i] = oracle.run_grid(grids[i], r["vmax"], r["p"], r["seed"], steps,
                                               t0=t0, replica=r["replica"], nthreads=nthreads)[0]
        cells = sum(r["L"] for r in sample)
        return _median_of_chunks(advance, cells, warm, chunk), cells

    # the sample: about 20 steps of it per timed chunk at a rate typical of such
    # hosts (1e8 cell-updates/s per core); a fifth of the budget warms up, each
    # of the 3 chunks takes about a quarter
    is_open = any(r.get("boundary") == "open" for r in reps)
    nthreads = 1 if is_open else threads
    sample, m = _stratified(reps, 1.0e8 * nthreads * budget_s / 4 / 20)
    (value, rates, warm, chunk), cells = run(sample, nthreads, budget_s / 5, budget_s / 4)
    s_sample, s_m = _stratified(reps, 1.0e8 * budget_s / 8 / 20)
    (s_value, s_rates, s_warm, s_chunk), s_cells = run(s_sample, 1, budget_s / 10, budget_s / 8)

    def desc(mm, smp, c, w, ch, rr):
        return (f"every {_ordinal(mm)} of {len(reps)} replicas in order of L ({len(smp)}, {c:.3g} "
                f"cells): {w} warm-up steps, then median of 3 chunks of {ch} steps "
                f"(chunk rates {', '.join(f'{x:.3g}' for x in rr)})")
    return {"value": value, "unit": "cell-updates/s", "cores": nthreads, "kind": "oracle",
            "sample": desc(m, sample, cells, warm, chunk, rates),
            "omp": {"OMP_PLACES": os.environ.get("OMP_PLACES"),
                    "OMP_PROC_BIND": os.environ.get("OMP_PROC_BIND"), "threads": nthreads},
            "extrapolated_full_workload_s": total * T / value, "extrapolated": True,
            "serial": {"value": s_value, "unit": "cell-updates/s", "cores": 1,
                       "sample": desc(s_m, s_sample, s_cells, s_warm, s_chunk, s_rates),
                       "extrapolated_full_workload_s": total * T / s_value,
                       "extrapolated": True},
            "host": _host_info()}


def cpu_baseline_single(cfg, T, budget_s=15.0, rng="keyed", max_cells=1 << 22):
    """The oracle on a bounded sample of a one-road workload: a road of at most
    max_cells cells with the workload's density, vmax, p and seed.  After a
    warm-up chunk, the median of 3 timed chunks on one thread per physical core
    (the reported value), then the same serially.  The keyed grid oracle stands
    for both representations (they give identical results); an open road and
    the shared stream have only serial oracles.  The full workload's time is
    extrapolated from the rate (labelled as such)."""
    import oracle
    L = min(cfg["L"], max_cells)
    N = int(round(cfg["N"] * L / cfg["L"]))
    g0 = oracle.init_grid(L, N, cfg["vmax"], cfg["seed"], init_v=cfg["init_v"])
    is_open = "alpha" in cfg
    stream = rng == "stream"
    threads = 1 if (is_open or stream) else _cpu_threads()

    def measure(nthreads, budget):
        state = {"g": g0}
        if stream:
            state["x"], state["v"] = oracle.grid_to_agent(g0)

        def advance(t0, steps):
            if is_open:
                state["g"] = oracle.run_open(state["g"], cfg["vmax"], cfg["p"], cfg["alpha"],
                                             cfg["beta"], cfg["seed"], steps, t0=t0)[0]
            elif stream:
                # the chunk continues the stream from its state after t0 N draws
                m = (1 << 31) - 1
                st = oracle.mlcg_seed(cfg["seed"]) * pow(48271, t0 * N, m) % m
                state["x"], state["v"], _ = oracle.run_agent_mlcg(
                    L, state["x"], state["v"], cfg["vmax"], cfg["p"], cfg["seed"], steps,
                    state0=st)
            else:
                state["g"] = oracle.run_grid(state["g"], cfg["vmax"], cfg["p"], cfg["seed"],
                                             steps, t0=t0, nthreads=nthreads)[0]
        rate, rates, warm, chunk = _median_of_chunks(advance, L, budget / 5, budget / 4)
        return rate, (f"L = {L}, N = {N}: {warm} warm-up steps, then median of 3 chunks of "
                      f"{chunk} steps (chunk rates {', '.join(f'{x:.3g}' for x in rates)})")

    value, smp = measure(threads, budget_s)
    s_value, s_smp = measure(1, budget_s / 2)
    return {"value": value, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": smp,
            "omp": {"OMP_PLACES": os.environ.get("OMP_PLACES"),
                    "OMP_PROC_BIND": os.environ.get("OMP_PROC_BIND"), "threads": threads},
            "extrapolated_full_workload_s": cfg["L"] * T / value, "extrapolated": True,
            "serial": {"value": s_value, "unit": "cell-updates/s", "cores": 1, "sample": s_smp,
                       "extrapolated_full_workload_s": cfg["L"] * T / s_value,
                       "extrapolated": True},
            "host": _host_info()}


def _cpu_baseline(job):
    """Run a CPU baseline in a child process of its own: the OpenMP runtime
    there starts with OMP_PLACES=cores and OMP_PROC_BIND=spread and every CPU
    of the process, which this process (torch's own OpenMP runtime binds its
    main thread once those variables are set) could not offer."""
    import subprocess
    env = dict(os.environ, OMP_PLACES="cores", OMP_PROC_BIND="spread",
               OMP_NUM_THREADS=str(_cpu_threads()))
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                        json.dumps(job)], capture_output=True, text=True, env=env, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"CPU baseline child failed:\n{r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def bench_ensemble(args):
    import torch
    from paper_2309_14311_amd import Batch, Sim, workloads

    make = workloads.open_ensemble if args.workload == "open_ensemble" else workloads.ensemble
    reps = make(args.replicas, seed=1, T=args.T, warmup=args.warmup_steps)
    cells = sum(r["L"] for r in reps)
    _log(f"ensemble: {len(reps)} replicas, sum L = {cells:.4g}, T = {args.T}")
    b = Batch(reps, use_graph=True)
    if args.k and args.q:
        b.set_tuning(args.k, args.q)
        k, q = args.k, args.q
        _log(f"fixed k={k} q={q}")
    else:
        k, q = b.autotune()
        _log(f"autotuned k={k} q={q}")
    launches = (args.T + k - 1) // k

    def one_pass():
        b.reset()
        ms = b.timed_step(args.T)
        sums = b.flux_sums()
        return ms, sums

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ms = []
    for _ in range(args.steps):
        ms, sums = one_pass()
        step_ms.append(ms)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    cell_updates = cells * args.T
    value = cell_updates / (ms_per_step * 1e-3)
    kernel_ms = float(np.mean(step_ms)) / launches      # average k-step launch
    achieved = BYTES_PER_CELL_UPDATE * cell_updates / launches / (kernel_ms * 1e-3)
    # the kernel is bound by VALU issue: its roofline counts the algorithmic
    # operations per launch (averaged like the bytes above) against the
    # vector-ALU peak
    ops_per_cu = sum(r["L"] * kstep_ops_per_cell_update(r["vmax"], r["p"]) for r in reps) / cells
    ops_achieved = ops_per_cu * cell_updates / launches / (kernel_ms * 1e-3)
    is_open = args.workload == "open_ensemble"
    # counters cover the ring kernel
    traffic = None if is_open else _traffic(k, q, cells * k)
    issued = None if is_open else _issued_valu(k, q, cells * k)
    probe = measure_valu()

    extra = {"batched_kernel_cups": cell_updates / (np.mean(step_ms) * 1e-3),
             "k": k, "q": q, "launches_per_pass": launches,
             "mean_flux_per_cell": float(np.sum(sums)) / max(1, sum(
                 r["L"] * (args.T - r["warmup"]) for r in reps))}

    # the plain loop: one replica per launch sequence, the same kernel, one stream
    if not args.no_plain:
        sample = reps[::args.plain_stride]
        stream = torch.cuda.Stream()
        sims = [Sim(r["L"], r["N"], r["vmax"], r["p"], r["seed"], replica=r["replica"],
                    init_v=r["init_v"], stream=stream, use_graph=True,
                    boundary=r.get("boundary", "ring"), alpha=r.get("alpha", 0.0),
                    beta=r.get("beta", 0.0)) for r in sample]
        for s in sims:
            s.reserve_log(2 * args.plain_T)
            s.step(args.plain_T)          # warm-up: captures each sim's launch graph
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for s in sims:
            s.step(args.plain_T)
        e1.record(stream)
        e1.synchronize()
        plain_ms = e0.elapsed_time(e1)
        plain_cells = sum(r["L"] for r in sample) * args.plain_T
        extra["plain_cups"] = plain_cells / (plain_ms * 1e-3)
        extra["plain_sample"] = f"every {_ordinal(args.plain_stride)} replica ({len(sample)}), " \
                                f"{args.plain_T} steps each"
        extra["batched_over_plain"] = extra["batched_kernel_cups"] / extra["plain_cups"]
        for s in sims:
            s.close()
    b.close()
    line = {
        "metric": "cell-updates/s and % HBM roofline, batched vs plain on 1 GPU, bit-exact",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": ("batched open-road ensemble (alpha, beta U[0,1]): " if is_open
                                else "batched ensemble: ") + f"{len(reps)} rings, L log-uniform "
                               f"[1e3,1e6], rho U[0.05,0.6], p in {{0,.13,.25,.5}}, vmax U{{1..8}}, "
                               f"T={args.T} ({args.warmup_steps} warm-up)",
                   "cells": cells, "T": args.T},
        # the whole pass's cell-updates priced at the one-step kernel's 2 B each:
        # a cell-update equivalent, not bytes that crossed HBM (see roofline.traffic)
        "cell_update_equiv_hbm_frac": value * BYTES_PER_CELL_UPDATE / HBM_PEAK,
        "roofline": {"bound": "alu", "achieved": ops_achieved / 1e12, "peak": VALU_PEAK / 1e12,
                     "unit": "TOP/s", "frac": ops_achieved / VALU_PEAK, "traffic": traffic,
                     "kernel": f"grid_kstep_mixed_kernel<{q}, {'true' if is_open else 'false'}>",
                     "kernel_ms": kernel_ms, "ops_per_cell_update": ops_per_cu,
                     "issued_valu_lane_instr_per_s": None if issued is None
                     else issued / (kernel_ms * 1e-3),
                     "issued_frac": None if issued is None
                     else issued / (kernel_ms * 1e-3) / VALU_PEAK,
                     "probe": probe,
                     "hbm_counter_GBps": None if traffic is None
                     else traffic / (kernel_ms * 1e-3) / 1e9,
                     "hbm_counter_frac": None if traffic is None
                     else traffic / (kernel_ms * 1e-3) / HBM_PEAK,
                     "cell_update_equiv_GBps": achieved / 1e9,
                     "cell_update_equiv_frac": achieved / HBM_PEAK},
        "extra": extra,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = _cpu_baseline(dict(
            kind="ensemble", open=is_open, replicas=args.replicas, T=args.T,
            warmup=args.warmup_steps, budget=args.cpu_budget))
    return line


def bench_serving(args):
    """Continuous batching: Poisson arrivals of requests (L log-uniform in
    [1e3, 1e7], density U[0.05, 0.6], p U[0, 0.5], vmax U{1..8}, T log-uniform
    in [1e2, 1e4]) at a fraction of the capacity measured on a short ensemble
    run; reports p50/p99 latency (arrival to result on the host) and the
    aggregate cell-updates/s over the whole stream."""
    import threading
    import torch
    from paper_2309_14311_amd import Batch, Server, workloads
    # capacity: cell-updates/s of the batched kernel on an ensemble shaped like the requests
    cal = workloads.requests(512, seed=99, rate=1.0)
    b = Batch([dict(r, warmup=0) for r in cal], k=32, q=4, use_graph=True)
    b.step(64)
    ms = b.timed_step(256)
    cap_cups = sum(r["L"] for r in cal) * 256 / (ms * 1e-3)
    b.close()
    mean_work = float(np.mean([r["L"] * r["T"] for r in workloads.requests(20000, seed=98)]))
    rate = args.rate_frac * cap_cups / mean_work
    reqs = workloads.requests(args.requests, seed=7, rate=rate)
    _log(f"serving: capacity {cap_cups:.3g} cell-updates/s, mean work {mean_work:.3g}, "
         f"rate {rate:.1f}/s x {len(reqs)} requests")
    srv = Server(k=32, q=4)
    results = {}
    submitted = {}
    t0 = time.perf_counter()
    s0 = srv.now()

    def producer():
        for r in reqs:
            delay = r["arrival"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            rid = srv.submit(r["L"], r["N"], r["vmax"], r["p"], r["seed"], r["T"],
                             init_v=r["init_v"], want_flux=False)
            submitted[rid] = r

    th = threading.Thread(target=producer)
    th.start()
    while len(results) < len(reqs):
        for res in srv.poll(max_results=1024, wait_ms=20):
            results[res["id"]] = res
    th.join()
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    lat = np.array([r["t_done"] - r["t_submit"] for r in results.values()])
    first = min(r["t_submit"] for r in results.values())
    last = max(r["t_done"] for r in results.values())
    work = sum(r["L"] * r["T"] for r in reqs)
    bad = sum(1 for r in results.values() if r["status"] != 0)
    value = work / (last - first)
    # latency per decade of L
    bands = {}
    for lo in (1e3, 1e4, 1e5, 1e6):
        sel = np.array([r["t_done"] - r["t_submit"] for rid, r in results.items()
                        if lo <= submitted[rid]["L"] < lo * 10 or (lo == 1e6 and
                                                                   submitted[rid]["L"] >= 1e7)])
        if sel.size:
            bands[f"L_{lo:.0e}"] = {"n": int(sel.size), "p50_s": float(np.percentile(sel, 50)),
                                    "p99_s": float(np.percentile(sel, 99))}
    # untimed tail: every 50th request's flux sum against the oracle (the
    # all-core twin), within a CPU budget; requests of more than 5e9
    # cell-updates are left to the unit tests
    import oracle
    checked, mismatched, spent = 0, 0, 0.0
    threads = _cpu_threads()
    for i, (rid, r) in enumerate(sorted(submitted.items())):
        if i % 50 or r["L"] * r["T"] > 5e9 or spent > args.cpu_budget * 2:
            continue
        t0 = time.perf_counter()
        g0 = oracle.init_grid(r["L"], r["N"], r["vmax"], r["seed"], replica=r["replica"],
                              init_v=r["init_v"])
        _, f = oracle.run_grid(g0, r["vmax"], r["p"], r["seed"], r["T"], replica=r["replica"],
                               nthreads=threads)
        spent += time.perf_counter() - t0
        checked += 1
        if results[rid]["status"] != 0 or int(f.sum()) != int(results[rid]["flux_sum"]):
            mismatched += 1
    return {
        "metric": "cell-updates/s and % HBM roofline, batched vs plain on 1 GPU, bit-exact",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": len(reqs),
        "warmup": 0, "ms_per_step": (last - first) * 1e3 / len(reqs),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson arrivals at {args.rate_frac} x capacity "
                               f"({rate:.1f} requests/s), {len(reqs)} requests"},
        "cell_update_equiv_hbm_frac": value * BYTES_PER_CELL_UPDATE / HBM_PEAK,
        "extra": {"latency_p50_s": float(np.percentile(lat, 50)),
                  "latency_p99_s": float(np.percentile(lat, 99)),
                  "latency_mean_s": float(lat.mean()), "latency_by_L": bands, "failed": bad,
                  "oracle_checked": checked, "oracle_mismatches": mismatched,
                  "oracle_check": "every 50th request of at most 5e9 cell-updates, flux sum "
                                  "over all T steps against the oracle's all-core twin",
                  "capacity_cups": cap_cups, "rate_per_s": rate, "launches": st["launches"],
                  "makespan_s": last - first, "server_clock_origin": s0},
    }


def bench_valu_probe(args):
    """The vector-ALU ceiling: sustained lane-ops/s of every instruction kind the
    step kernels use (libnasch_probe), with the shader clock of each run, against
    the unit-count peaks (2-cycle and 4-cycle issue)."""
    from paper_2309_14311_amd import native
    kinds = {}
    for kind in native.PROBE_KINDS:
        r = native.probe_valu(kind, 4096, 4000)
        per_cycle = r["lane_ops_per_s"] / r["sclk_hz"] / 256 / 64
        kinds[kind] = {"lane_ops_per_s": r["lane_ops_per_s"], "sclk_ghz": r["sclk_hz"] / 1e9,
                       "wave_instr_per_cycle_per_cu": per_cycle,
                       "issue_cycles": 2 if per_cycle > 1.25 else 4}
    best = max(v["lane_ops_per_s"] for v in kinds.values())
    return {
        "metric": "vector-ALU lane-ops/s by instruction kind", "value": best,
        "unit": "lane-ops/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "VALU probe: 4096 blocks x 256 lanes, 8 independent chains of "
                               "one instruction kind per lane"},
        "peak_2cycle": VALU_PEAK, "peak_4cycle": VALU_PEAK_4CYCLE, "kinds": kinds,
    }


def bench_single(args, cfg, rep, kernels):
    """One ring: value = k-step (autotuned) CUPS; the one-step kernel beside it."""
    import torch
    from paper_2309_14311_amd import Sim
    rng = getattr(args, "rng", "keyed") if rep == "agent" else "keyed"
    road = {}
    if "alpha" in cfg:
        road = dict(boundary="open", alpha=cfg["alpha"], beta=cfg["beta"])
    s = Sim(cfg["L"], cfg["N"], cfg["vmax"], cfg["p"], cfg["seed"], rep=rep,
            init_v=cfg["init_v"], use_graph=True, rng=rng, **road)
    if args.k and args.q:
        s.set_tuning("kstep", args.k, args.q)   # q: words per lane (grid) or cars per lane (agent)
    else:
        s.autotune()
    info = s.info()
    T = cfg["T"] if args.T_single is None else args.T_single
    res = {}
    for kern in kernels:
        s.set_tuning(kern, info["k"], info["q"])
        for _ in range(args.warmup):
            s.timed_step(T)
        ms = [s.timed_step(T) for _ in range(args.steps)]
        res[kern] = cfg["L"] * T / (np.mean(ms) * 1e-3)
    torch.cuda.synchronize()
    s.close()
    value = res["kstep"]
    # algorithmic bytes per cell-update: the grid reads and writes each cell's
    # byte; the agent form reads and writes x (4 B) and v (1 B) of each car
    bpcu = BYTES_PER_CELL_UPDATE if rep == "grid" else 10.0 * cfg["N"] / cfg["L"]
    if "onestep" in res:
        # one step per launch moves all of them every step: HBM-bound
        res["onestep_hbm_frac"] = res["onestep"] * bpcu / HBM_PEAK
    ms_T = {kern: cfg["L"] * T / res[kern] * 1e3 for kern in kernels}
    if rep == "grid" and cfg["L"] >= 1 << 24:
        # achievable HBM bandwidth, bytes read + written over 1 GiB, timed with
        # events: the runtime's device-to-device copy, and an elementwise
        # read-modify-write kernel (the faster of the two here)
        n = 1 << 30
        a = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        c = torch.empty_like(a)

        def rate(fn):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(5):
                fn()
            e1.record()
            e1.synchronize()
            return 2.0 * n * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9

        res["copy_GBps"] = rate(lambda: c.copy_(a))
        res["stream_rw_GBps"] = rate(lambda: torch.add(a.view(torch.float32), 1.0,
                                                        out=c.view(torch.float32)))
        del a, c
        torch.cuda.empty_cache()
        # the bit-sliced kernel without temporal blocking (k = 1): the one-step
        # path whose bound is HBM at 2 B per cell-update
        s = Sim(cfg["L"], cfg["N"], cfg["vmax"], cfg["p"], cfg["seed"], rep=rep,
                init_v=cfg["init_v"], use_graph=True, kernel="kstep", k=1, q=1, **road)
        s.timed_step(min(T, 64))
        ms = [s.timed_step(T) for _ in range(args.steps)]
        res["kstep_k1"] = cfg["L"] * T / (np.mean(ms) * 1e-3)
        res["kstep_k1_hbm_frac"] = res["kstep_k1"] * BYTES_PER_CELL_UPDATE / HBM_PEAK
        torch.cuda.synchronize()
        s.close()
    line = {
        "metric": "cell-updates/s and % HBM roofline, batched vs plain on 1 GPU, bit-exact",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": cfg["L"] * T / value * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": (f"open road alpha={cfg['alpha']} beta={cfg['beta']}" if road
                                else f"{rep} ring") +
                               f" L={cfg['L']} N={cfg['N']} vmax={cfg['vmax']} "
                               f"p={cfg['p']} T={T}" + (" shared-stream rng" if rng == "stream"
                                                        else ""),
                   "k": info["k"], "q": info["q"]},
        # the k-step rate priced at the one-step kernel's algorithmic bytes: a
        # cell-update equivalent, not bytes that crossed HBM
        "cell_update_equiv_hbm_frac": value * bpcu / HBM_PEAK,
        "bytes_per_cell_update": bpcu,
        "extra": {(k if k.endswith(("frac", "GBps")) else f"{k}_cups"): v for k, v in res.items()},
    }
    line["extra"].update({f"{kern}_ms_for_T": v for kern, v in ms_T.items()})
    if rep == "grid" and not road:
        # the k-step kernel is bound by vector-ALU issue (see the ensemble)
        ops = kstep_ops_per_cell_update(cfg["vmax"], cfg["p"]) * value
        line["roofline"] = {"bound": "alu", "achieved": ops / 1e12, "peak": VALU_PEAK / 1e12,
                            "unit": "TOP/s", "frac": ops / VALU_PEAK, "traffic": None,
                            "kernel": f"grid_kstep_kernel<{cfg['vmax']}, {info['q']}, false>"}
        if "onestep" in res:
            line["roofline_onestep"] = {
                "bound": "hbm", "achieved": res["onestep"] * bpcu / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": res["onestep"] * bpcu / HBM_PEAK, "traffic": None,
                "kernel": f"grid_onestep_kernel<{cfg['vmax']}, 1, false>"}
    if not args.no_cpu:
        line["cpu_baseline"] = _cpu_baseline(dict(kind="single", cfg=cfg, T=T,
                                                  budget=args.cpu_budget, rng=rng))
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ensemble",
                    choices=["ensemble", "large_ring", "agent", "reference", "serving",
                             "open_road", "open_ensemble", "valu_probe"])
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate-frac", type=float, default=0.5)
    ap.add_argument("--replicas", type=int, default=4096)
    ap.add_argument("--T", type=int, default=5000)
    ap.add_argument("--warmup-steps", type=int, default=1000)
    ap.add_argument("--T-single", type=int, default=None)
    ap.add_argument("--k", type=int, default=0,
                    help="steps per launch (0: autotune; one-road workloads use --k and --q "
                         "only when both are given)")
    ap.add_argument("--q", type=int, default=0,
                    help="words per lane of the grid kernel, or cars per lane of the agent "
                         "k-step kernel (0: autotune / by density)")
    ap.add_argument("--plain-stride", type=int, default=8)
    ap.add_argument("--plain-T", type=int, default=1000)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rng", default="keyed", choices=["keyed", "stream"],
                    help="rule-3 numbers of the agent workload: keyed draws or the shared "
                         "minstd stream")
    ap.add_argument("--cpu-baseline-child", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_child:
        # the CPU baseline's own process (see _cpu_baseline): no torch, no GPU
        job = json.loads(args.cpu_baseline_child)
        from paper_2309_14311_amd import workloads
        if job["kind"] == "ensemble":
            make = workloads.open_ensemble if job["open"] else workloads.ensemble
            reps = make(job["replicas"], seed=1, T=job["T"], warmup=job["warmup"])
            out = cpu_baseline_ensemble(reps, job["T"], budget_s=job["budget"])
        else:
            out = cpu_baseline_single(job["cfg"], job["T"], budget_s=job["budget"],
                                      rng=job["rng"])
        print(json.dumps(out), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the NaSch hot path here is measured per GPU "
              "(--gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    from paper_2309_14311_amd import workloads
    if args.workload in ("ensemble", "open_ensemble"):
        line = bench_ensemble(args)
    elif args.workload == "serving":
        line = bench_serving(args)
    elif args.workload == "valu_probe":
        line = bench_valu_probe(args)
    elif args.workload == "large_ring":
        line = bench_single(args, workloads.LARGE_RING, "grid", ["kstep", "onestep"])
    elif args.workload == "open_road":
        line = bench_single(args, workloads.OPEN_ROAD, "grid", ["kstep", "onestep"])
    elif args.workload == "agent":
        line = bench_single(args, workloads.AGENT_RING, "agent", ["kstep", "onestep"])
    else:
        line = bench_single(args, workloads.REFERENCE, "grid", ["kstep", "onestep"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
