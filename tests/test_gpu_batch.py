"""GPU parity of the batched ensemble: every replica equals the oracle and equals
itself run alone; results do not depend on (k, q), graph replay or reset."""
import numpy as np
import pytest

import oracle
from paper_2309_14311_amd import Batch, NaschError, Sim, workloads

pytestmark = pytest.mark.gpu


def _small_ensemble(n=48, seed=3, T=300, warmup=100):
    return workloads.ensemble(n, seed=seed, T=T, warmup=warmup, L_lo_exp=1.0, L_hi_exp=4.3)


def _oracle_replica(r, T):
    g0 = oracle.init_grid(r["L"], r["N"], r["vmax"], r["seed"], replica=r["replica"],
                          init_v=r["init_v"])
    return oracle.run_grid(g0, r["vmax"], r["p"], r["seed"], T, replica=r["replica"])


def test_every_replica_matches_oracle_with_logs():
    reps = _small_ensemble()
    T = 300
    b = Batch(reps, keep_log=True, log_steps=T)
    b.step(T)
    sums = b.flux_sums()
    for i, r in enumerate(reps):
        g, flux = _oracle_replica(r, T)
        got, t = b.snapshot(i)
        assert t == T
        np.testing.assert_array_equal(got, g, err_msg=f"replica {i} {r}")
        np.testing.assert_array_equal(b.flux(i, 0, T), flux)
        assert int(sums[i]) == int(flux[r["warmup"]:].sum())
    b.close()


@pytest.mark.parametrize("k,q", [(1, 1), (5, 2), (16, 4), (32, 4), (64, 4), (24, 1)])
def test_tuning_and_graph_do_not_change_results(k, q):
    reps = _small_ensemble(32, seed=9)
    T = 257
    ref = Batch(reps)
    ref.step(T)
    want = ref.flux_sums()
    want_g = [ref.snapshot(i)[0] for i in range(len(reps))]
    ref.close()
    for use_graph in (False, True):
        b = Batch(reps, k=k, q=q, use_graph=use_graph)
        for chunk in (100, 57, 100):
            b.step(chunk)
        np.testing.assert_array_equal(b.flux_sums(), want)
        for i in range(len(reps)):
            np.testing.assert_array_equal(b.snapshot(i)[0], want_g[i])
        b.close()


def test_replica_in_batch_equals_replica_alone():
    """A replica's result does not depend on the other replicas of the launch."""
    reps = workloads.ensemble(64, seed=5, T=400, warmup=100, L_lo_exp=3.0, L_hi_exp=5.5)
    b = Batch(reps, use_graph=True)
    b.step(400)
    sums = b.flux_sums()
    for i in range(0, 64, 7):
        r = reps[i]
        s = Sim(r["L"], r["N"], r["vmax"], r["p"], r["seed"], replica=r["replica"],
                init_v=r["init_v"])
        s.step(400)
        g, _ = s.snapshot()
        np.testing.assert_array_equal(b.snapshot(i)[0], g)
        assert int(sums[i]) == int(s.flux(r["warmup"], 400 - r["warmup"]).sum())
        s.close()
    b.close()


def test_reset_and_autotune_reproduce():
    reps = _small_ensemble(24, seed=11)
    b = Batch(reps, use_graph=True)
    b.step(200)
    first = b.flux_sums().copy()
    k, q = b.autotune()
    assert k > 0 and q in (1, 2, 3, 4)
    b.reset()
    b.step(200)
    np.testing.assert_array_equal(b.flux_sums(), first)
    b.close()


def test_batch_rejects_bad_replicas():
    with pytest.raises(NaschError):
        Batch([dict(L=10, N=11, vmax=5, p=0.1, seed=1)])
    with pytest.raises(NaschError):
        Batch([dict(L=10, N=5, vmax=5, p=1.5, seed=1)])


def _open_ensemble(n, seed):
    """Open roads for a parameter study: the small ensemble's roads with entry
    and exit probabilities drawn over [0, 1], the extremes included."""
    rng = np.random.default_rng(seed)
    reps = _small_ensemble(n, seed=seed)
    for i, r in enumerate(reps):
        r["boundary"] = "open"
        r["alpha"] = float(rng.choice([0.0, 1.0, rng.random()]))
        r["beta"] = float(rng.choice([0.0, 1.0, rng.random()]))
    return reps


@pytest.mark.parametrize("k,q", [(16, 2), (7, 1), (32, 4)])
def test_open_road_ensemble_matches_oracle(k, q):
    """A batch of open roads (mixed vmax, p, alpha, beta, ragged and tiny L):
    every replica's log, flux sum and final road equal the oracle's."""
    reps = _open_ensemble(40, seed=21)
    T = 220
    b = Batch(reps, k=k, q=q, keep_log=True, log_steps=T, use_graph=True)
    try:
        b.step(100)
        b.step(T - 100)
        sums = b.flux_sums()
        for i, r in enumerate(reps):
            g0 = oracle.init_grid(r["L"], r["N"], r["vmax"], r["seed"], replica=r["replica"],
                                  init_v=r["init_v"])
            g, flux, _, _ = oracle.run_open(g0, r["vmax"], r["p"], r["alpha"], r["beta"],
                                            r["seed"], T, replica=r["replica"])
            got, t = b.snapshot(i)
            assert t == T
            np.testing.assert_array_equal(got, g, err_msg=f"replica {i} {r}")
            np.testing.assert_array_equal(b.flux(i, 0, T), flux)
            assert int(sums[i]) == int(flux[r["warmup"]:].sum())
    finally:
        b.close()


def test_open_and_ring_replicas_do_not_mix():
    reps = _small_ensemble(4, seed=2)
    reps[1].update(boundary="open", alpha=0.5, beta=0.5)
    with pytest.raises(NaschError):
        Batch(reps)
    bad = _open_ensemble(3, seed=4)
    bad[2]["alpha"] = float("nan")
    with pytest.raises(NaschError):
        Batch(bad)


def test_every_state_of_a_tiny_ring_in_one_batch():
    """Every grid state of a ring of L = 8 cells with vmax = 3 (5^8 = 390625
    states, each cell empty or a car with v = 0..3) as the replicas of one
    batch, restored in one call: after 40 steps (launches of 16, 16 and 8) every
    replica's grid and flux sum equal the oracle's.  The ring is far shorter
    than the k vmax halo, so every segment holds many periodic images; p = 0.3
    has bits below its top nibble, so tied draws are refined too."""
    import itertools
    L, vmax, p, seed, T = 8, 3, 0.3, 77, 40
    states = np.array(list(itertools.product(range(vmax + 2), repeat=L)), np.uint8)
    states[states == vmax + 1] = 0xFF
    cars = (states != 0xFF).sum(axis=1)
    reps = [dict(L=L, N=int(n), vmax=vmax, p=p, seed=seed, replica=i) for i, n in enumerate(cars)]
    b = Batch(reps, k=16, q=2, use_graph=True)
    try:
        b.restore(states.reshape(-1), 0)
        b.step(T)
        got, t = b.snapshot_all()
        assert t == T
        got = got.reshape(-1, L)
        sums = b.flux_sums()
    finally:
        b.close()
    bad = []
    for i in range(len(reps)):
        g, flux = oracle.run_grid(states[i], vmax, p, seed, T, replica=i)
        if not np.array_equal(got[i], g) or int(sums[i]) != int(flux.sum()):
            bad.append(i)
            if len(bad) >= 5:
                break
    assert not bad, f"replicas {bad}: first state {states[bad[0]]}"


def test_batch_checkpoint_and_resume():
    """snapshot_all at t = 150, restore into a fresh batch, 100 more steps:
    grids and the flux of those steps equal the uninterrupted run's."""
    reps = _small_ensemble(24, seed=13)
    for r in reps:
        r["warmup"] = 0
    a = Batch(reps, keep_log=True, log_steps=250)
    try:
        a.step(150)
        snap, t = a.snapshot_all()
        assert t == 150
        mid_sums = a.flux_sums().copy()
        a.step(100)
        want, _ = a.snapshot_all()
        want_sums = a.flux_sums() - mid_sums
        want_log = [a.flux(i, 150, 100) for i in range(len(reps))]
    finally:
        a.close()
    b = Batch(reps, keep_log=True, log_steps=250, use_graph=True)
    try:
        b.restore(snap, 150)
        b.step(100)
        got, t = b.snapshot_all()
        assert t == 250
        np.testing.assert_array_equal(got, want)
        np.testing.assert_array_equal(b.flux_sums(), want_sums)
        for i in range(len(reps)):
            np.testing.assert_array_equal(b.flux(i, 150, 100), want_log[i])
        # the per-replica snapshot agrees with the whole-batch one
        off = 0
        for i, r in enumerate(reps):
            np.testing.assert_array_equal(b.snapshot(i)[0], got[off:off + r["L"]])
            off += r["L"]
    finally:
        b.close()


def test_batch_restore_rejects_bad_grids():
    reps = [dict(L=40, N=10, vmax=3, p=0.2, seed=1, replica=i) for i in range(3)]
    b = Batch(reps)
    try:
        good, _ = b.snapshot_all()
        for bad in (np.where(good == 0xFF, 0xFF, 4).astype(np.uint8),    # v > vmax
                    np.full_like(good, 0xFF)):                            # car count != N
            with pytest.raises(NaschError):
                b.restore(bad, 5)
        with pytest.raises(NaschError):
            b.restore(good, 2**32)
        b.restore(good, 7)    # a good checkpoint still restores
        assert b.snapshot_all()[1] == 7
    finally:
        b.close()
