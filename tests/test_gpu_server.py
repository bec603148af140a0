"""GPU tests of the serving loop: every result equals the oracle, a request gives
the same result alone and in the mix, requests queue when the HBM budget is
small, cancellation and invalid requests."""
import time

import numpy as np
import pytest

import oracle
from paper_2309_14311_amd import NaschError, Server, Sim, workloads

pytestmark = pytest.mark.gpu


def _footprint(r):
    """Device bytes of one request's slot, as nasch_server_submit documents it."""
    c256 = lambda n: (n + 255) // 256 * 256
    return c256(r["L"]) + 2 * c256(4 * (r["vmax"] + 1) * ((r["L"] + 31) // 32)) + c256(8 * r["T"])


def _oracle(r):
    g0 = oracle.init_grid(r["L"], r["N"], r["vmax"], r["seed"], replica=r["replica"],
                          init_v=r["init_v"])
    return oracle.run_grid(g0, r["vmax"], r["p"], r["seed"], r["T"], replica=r["replica"])


def _drain(srv, n, timeout=120.0):
    out = {}
    deadline = time.time() + timeout
    while len(out) < n and time.time() < deadline:
        for res in srv.poll(wait_ms=50):
            out[res["id"]] = res
    assert len(out) == n, f"only {len(out)} of {n} results"
    return out


def test_results_match_oracle():
    reqs = workloads.requests(40, seed=3, L_exp=(1.5, 4.0), T_exp=(1.0, 2.7))
    srv = Server(k=16)
    ids = [srv.submit(r["L"], r["N"], r["vmax"], r["p"], r["seed"], r["T"], init_v=r["init_v"],
                      want_grid=True) for r in reqs]
    res = _drain(srv, len(ids))
    for rid, r in zip(ids, reqs):
        g, flux = _oracle(r)
        got = res[rid]
        assert got["status"] == 0
        np.testing.assert_array_equal(got["flux"], flux)
        np.testing.assert_array_equal(got["grid"], g)
        assert got["flux_sum"] == int(flux.sum())
        assert got["t_submit"] <= got["t_admit"] <= got["t_done"]
    srv.close()


def test_alone_equals_in_mix_and_queueing_under_small_budget():
    reqs = workloads.requests(60, seed=4, L_exp=(3.0, 5.0), T_exp=(1.5, 3.0))
    # budget fits a few requests only: the rest must wait, not fail
    budget = 6 * max(_footprint(r) for r in reqs)
    srv = Server(k=32, hbm_budget=budget)
    ids = [srv.submit(r["L"], r["N"], r["vmax"], r["p"], r["seed"], r["T"], init_v=r["init_v"],
                      want_grid=True) for r in reqs]
    saw_pending = srv.stats()["pending"] > 0
    res = _drain(srv, len(ids))
    assert saw_pending
    st = srv.stats()
    assert st["done"] == len(reqs) and st["bytes_in_use"] == 0 and st["running"] == 0
    srv.close()
    for rid, r in list(zip(ids, reqs))[::6]:
        s = Sim(r["L"], r["N"], r["vmax"], r["p"], r["seed"], init_v=r["init_v"])
        s.step(r["T"])
        g, _ = s.snapshot()
        np.testing.assert_array_equal(res[rid]["grid"], g)
        np.testing.assert_array_equal(res[rid]["flux"], s.flux(0, r["T"]))
        s.close()


def test_rings_of_very_different_sizes_in_one_arena():
    """Rings of 10^3 to 2 x 10^5 cells, submitted together, share the launches:
    each equals the oracle in its flux log and final grid."""
    reqs = workloads.requests(24, seed=11, L_exp=(3.0, 5.8), T_exp=(2.0, 3.0))
    assert min(r["L"] for r in reqs) < 2000 and max(r["L"] for r in reqs) > 150000
    srv = Server(k=32)
    ids = [srv.submit(r["L"], r["N"], r["vmax"], r["p"], r["seed"], r["T"], init_v=r["init_v"],
                      want_grid=True) for r in reqs]
    res = _drain(srv, len(ids))
    srv.close()
    for rid, r in zip(ids, reqs):
        g, flux = _oracle(r)
        assert res[rid]["status"] == 0
        np.testing.assert_array_equal(res[rid]["flux"], flux)
        np.testing.assert_array_equal(res[rid]["grid"], g)


def test_cancel_and_invalid_requests():
    srv = Server(k=32)
    with pytest.raises(NaschError):
        srv.submit(100, 200, 5, 0.1, 1, 10)        # N > L
    with pytest.raises(NaschError):
        srv.submit(100, 20, 5, 0.1, 1, 0)          # T = 0
    big = srv.submit(2_000_000, 400_000, 5, 0.2, 1, 20000, want_flux=True)
    small = srv.submit(1000, 200, 5, 0.13, 1, 50)
    # a small ring (the second chain of launches) with many steps, cancelled
    # while that chain runs
    long_small = srv.submit(5000, 1000, 5, 0.2, 2, 400_000, want_flux=True)
    srv.cancel(big)
    time.sleep(0.05)
    srv.cancel(long_small)
    res = _drain(srv, 3)
    assert res[small]["status"] == 0
    assert res[big]["status"] == -5
    assert res[long_small]["status"] == -5
    assert srv.stats()["bytes_in_use"] == 0   # released as each result is queued
    srv.close()


def test_health_for_a_watchdog():
    """While a long request runs, the seconds since the scheduling thread last
    finished a burst stay far below the request's run time and the live count
    covers it; once the server is idle both are zero."""
    srv = Server(k=32)
    assert srv.health() == {"since_progress_s": 0.0, "live": 0}
    rid = srv.submit(10_000_000, 2_000_000, 5, 0.2, 1, 100_000)
    worst, saw_live, res = 0.0, False, []
    deadline = time.time() + 60
    while not res and time.time() < deadline:
        h = srv.health()
        worst = max(worst, h["since_progress_s"])
        saw_live = saw_live or h["live"] >= 1
        res = srv.poll(wait_ms=5)
    assert res and res[0]["id"] == rid and res[0]["status"] == 0
    assert saw_live and worst < 0.5
    deadline = time.time() + 5
    while srv.health()["live"] and time.time() < deadline:
        time.sleep(0.01)
    assert srv.health() == {"since_progress_s": 0.0, "live": 0}
    srv.close()
