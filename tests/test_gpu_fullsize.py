"""Parity at the full workload sizes, in the launch configuration the benchmark
times:
  - the whole final road and the whole flux log against the oracle, through
    64-bit FNV-1a checksums that tests/golden/make_fullsize.py computed with
    the oracle alone (the all-core twin of the grid step, or the serial stream
    run) and stored in tests/golden/fullsize.json;
  - sampled windows of the final road against the oracle's light-cone
    evaluation (a cell after T steps depends only on cells within T*vmax);
  - the temporal-blocked, one-step and agent paths agree on the whole state;
  - properties of the flux log that hold at any size: F(T-1) is the sum of the
    final velocities, and F(t) <= min(N vmax, L - N) (no car exceeds vmax or
    its gap, and the gaps add up to L - N).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2309_14311_amd import Batch, Sim, workloads

pytestmark = pytest.mark.gpu
EMPTY = 0xFF
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "fullsize.json")) as _f:
    GOLDEN = json.load(_f)


def _assert_golden(name, cfg, grid, flux):
    """The whole final road and flux log equal the oracle's (by checksum)."""
    g = GOLDEN[name]
    for key in ("L", "N", "vmax", "p", "seed", "replica", "init_v", "T"):
        assert g[key] == cfg[key], (name, key)
    assert f"{oracle.fnv1a64(grid):016x}" == g["grid_fnv1a64"], f"{name}: final road differs"
    assert int(flux[-1]) == g["flux_last"] and int(flux.sum()) == g["flux_sum"]
    assert f"{oracle.fnv1a64(flux.astype('<u8')):016x}" == g["flux_fnv1a64"], \
        f"{name}: flux log differs"


def _windows(L, n, w, seed):
    rng = np.random.default_rng(seed)
    starts = [0, L - w // 2, L // 2] + [int(x) for x in rng.integers(0, L, size=n)]
    return [(s % L, w) for s in starts]


def _check_windows(sim_range, cfg, T, windows):
    for a, w in windows:
        want = oracle.window_from_init(cfg["L"], cfg["N"], cfg["vmax"], cfg["p"], cfg["seed"], T,
                                       a, w, replica=cfg["replica"], init_v=cfg["init_v"])
        got = sim_range(a, w)
        np.testing.assert_array_equal(got, want, err_msg=f"window at {a}")


def _flux_properties(flux, final_grid, N, vmax):
    L = final_grid.size
    assert int(flux.max()) <= min(N * vmax, L - N)
    occ = final_grid != EMPTY
    assert int(occ.sum()) == N
    assert int(final_grid[occ].astype(np.int64).sum()) == int(flux[-1])


def test_large_ring_kstep_onestep_and_oracle_windows():
    cfg = workloads.LARGE_RING
    L, N, T = cfg["L"], cfg["N"], cfg["T"]
    a = Sim(L, N, cfg["vmax"], cfg["p"], cfg["seed"], init_v=cfg["init_v"], use_graph=True)
    a.autotune()
    a.step(T)
    _check_windows(a.snapshot_range, cfg, T, _windows(L, 5, 192, 1))
    ga, _ = a.snapshot()
    fa = a.flux(0, T)
    a.close()
    _flux_properties(fa, ga, N, cfg["vmax"])
    _assert_golden("large_ring", cfg, ga, fa)
    b = Sim(L, N, cfg["vmax"], cfg["p"], cfg["seed"], init_v=cfg["init_v"], kernel="onestep",
            use_graph=True)
    b.step(T)
    gb, _ = b.snapshot()
    fb = b.flux(0, T)
    b.close()
    _assert_golden("large_ring", cfg, gb, fb)


def test_open_road_kstep_onestep_and_oracle_windows():
    """The 2^30-cell open road: windows at both ends (where cars enter and
    leave) and inside against the oracle's light cone; k-step (autotuned, as
    benchmarked) and one-step agree on the whole road and the flux log; the
    last step's flux covers the final velocities plus at most vmax^2 for the
    cars that left in it."""
    cfg = workloads.OPEN_ROAD
    L, N, T, vmax = cfg["L"], cfg["N"], cfg["T"], cfg["vmax"]
    kw = dict(init_v=cfg["init_v"], boundary="open", alpha=cfg["alpha"], beta=cfg["beta"])
    a = Sim(L, N, vmax, cfg["p"], cfg["seed"], use_graph=True, **kw)
    a.autotune()
    a.step(T)
    for s0, w in [(0, 512), (L - 512, 512), (L // 2, 192), (123456789, 192), (L - 6000, 300)]:
        want = oracle.open_window_from_init(L, N, vmax, cfg["p"], cfg["alpha"], cfg["beta"],
                                            cfg["seed"], T, s0, w, init_v=cfg["init_v"])
        np.testing.assert_array_equal(a.snapshot_range(s0, w), want, err_msg=f"window at {s0}")
    ga, _ = a.snapshot()
    fa = a.flux(0, T)
    a.close()
    b = Sim(L, N, vmax, cfg["p"], cfg["seed"], kernel="onestep", **kw)
    b.step(T)
    gb, _ = b.snapshot()
    np.testing.assert_array_equal(b.flux(0, T), fa)
    b.close()
    assert np.array_equal(ga, gb)
    occ = ga != EMPTY
    extra = int(fa[-1]) - int(ga[occ].astype(np.int64).sum())
    assert 0 <= extra <= vmax * vmax


def test_maximum_length_ring():
    """L = 2^31 - 1, the largest ring the library accepts: odd, so the word
    that wraps the ring end is unaligned.  Windows at both ends, across the
    wrap and inside match the oracle's light cone after two k-step launches;
    the one-step kernel gives the same road and flux log."""
    L, vmax, p, seed, T = 2**31 - 1, 5, 0.13, 7, 40
    N = int(0.2 * L)
    cfg = dict(L=L, N=N, vmax=vmax, p=p, seed=seed, replica=0, init_v=1)
    a = Sim(L, N, vmax, p, seed, init_v=1, kernel="kstep", k=32, q=4)
    a.step(T)
    _check_windows(a.snapshot_range, cfg, T,
                   [(0, 256), (L - 256, 256), (L - 100, 200), (L // 3, 160), (1234567891, 96)])
    ga, _ = a.snapshot()
    fa = a.flux(0, T)
    a.close()
    _flux_properties(fa, ga, N, vmax)
    b = Sim(L, N, vmax, p, seed, init_v=1, kernel="onestep")
    b.step(T)
    gb, _ = b.snapshot()
    np.testing.assert_array_equal(b.flux(0, T), fa)
    b.close()
    assert np.array_equal(ga, gb)


def test_agent_ring_equals_grid_and_oracle_windows():
    cfg = workloads.AGENT_RING
    L, N, T = cfg["L"], cfg["N"], cfg["T"]
    a = Sim(L, N, cfg["vmax"], cfg["p"], cfg["seed"], rep="agent", init_v=cfg["init_v"],
            use_graph=True)
    a.autotune()
    a.step(T)
    _check_windows(a.snapshot_range, cfg, T, _windows(L, 4, 160, 2))
    ga, _ = a.snapshot()
    fa = a.flux(0, T)
    x, v = a.agent_state()
    a.close()
    assert int((np.diff(x) < 0).sum()) <= 1          # order kept: one cyclic descent
    _flux_properties(fa, ga, N, cfg["vmax"])
    _assert_golden("agent_ring", cfg, ga, fa)
    b = Sim(L, N, cfg["vmax"], cfg["p"], cfg["seed"], rep="agent", init_v=cfg["init_v"],
            kernel="onestep", use_graph=True)
    b.step(T)
    gb, _ = b.snapshot()
    fb = b.flux(0, T)
    b.close()
    _assert_golden("agent_ring", cfg, gb, fb)
    g = Sim(L, N, cfg["vmax"], cfg["p"], cfg["seed"], init_v=cfg["init_v"])
    g.step(T)
    gg, _ = g.snapshot()
    np.testing.assert_array_equal(g.flux(0, T), fa)
    g.close()
    assert np.array_equal(ga, gg)


@pytest.mark.parametrize("kernel", ["kstep", "onestep"])
def test_agent_ring_shared_stream_whole_state(kernel):
    """The agent ring with the paper's shared minstd stream (car numbers up to
    1000 N = 6.7e10), as the benchmark's --rng stream run: the whole final road
    and flux log equal the serial stream oracle's."""
    cfg = workloads.AGENT_RING
    L, N, T = cfg["L"], cfg["N"], cfg["T"]
    a = Sim(L, N, cfg["vmax"], cfg["p"], cfg["seed"], rep="agent", rng="stream",
            init_v=cfg["init_v"], use_graph=True, kernel=kernel)
    if kernel == "kstep":
        a.autotune()
    a.step(T)
    ga, _ = a.snapshot()
    fa = a.flux(0, T)
    a.close()
    _assert_golden("agent_stream", cfg, ga, fa)


def test_ensemble_in_bench_configuration():
    """The 4096-replica ensemble as the benchmark runs it (graph replay, autotuned
    (k, q), reset between passes): every replica's final road and flux sum
    against the oracle's (by checksum, over two passes); the smallest replicas,
    a median-size one and the largest one against the oracle in full (the
    largest on the oracle's all-core twin), a sample of the rest against the
    same replica run alone."""
    reps = workloads.ensemble(4096, seed=1, T=5000, warmup=1000)
    g = GOLDEN["ensemble"]
    assert (g["replicas"], g["seed"], g["T"], g["warmup"]) == (4096, 1, 5000, 1000)
    assert g["cells"] == sum(r["L"] for r in reps)
    b = Batch(reps, use_graph=True)
    b.autotune()
    for _ in range(2):
        b.reset()
        b.step(5000)
        sums = b.flux_sums()
        grids, t = b.snapshot_all()
        assert t == 5000
        assert f"{oracle.fnv1a64(grids):016x}" == g["grid_fnv1a64"], "final roads differ"
        assert int(sums.astype(np.uint64).sum()) == g["flux_sums_total"]
        assert f"{oracle.fnv1a64(sums.astype('<u8')):016x}" == g["flux_sums_fnv1a64"], \
            "flux sums differ"
        del grids
    order = np.argsort([r["L"] for r in reps])
    nthreads = min(16, oracle.num_threads_available())
    for i in list(order[:12]) + [order[len(order) // 2], order[-1]]:
        r = reps[i]
        g0 = oracle.init_grid(r["L"], r["N"], r["vmax"], r["seed"], replica=r["replica"],
                              init_v=r["init_v"])
        g, flux = oracle.run_grid(g0, r["vmax"], r["p"], r["seed"], 5000, replica=r["replica"],
                                  nthreads=nthreads)
        np.testing.assert_array_equal(b.snapshot(i)[0], g, err_msg=f"replica {i} L={r['L']}")
        assert int(sums[i]) == int(flux[1000:].sum())
    for i in order[::400]:
        r = reps[i]
        s = Sim(r["L"], r["N"], r["vmax"], r["p"], r["seed"], replica=r["replica"],
                init_v=r["init_v"])
        s.step(5000)
        np.testing.assert_array_equal(b.snapshot(i)[0], s.snapshot()[0])
        assert int(sums[i]) == int(s.flux(1000, 4000).sum())
        s.close()
    b.close()
