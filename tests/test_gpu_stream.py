"""GPU parity of the shared-stream mode (the paper's one generator for all
cars, reached by jump-ahead on the GPU) against the oracle, which runs the
stream strictly serially."""
import numpy as np
import pytest

import oracle
from paper_2309_14311_amd import NaschError, Sim

pytestmark = pytest.mark.gpu


def _oracle(L, N, vmax, p, seed, T, init_v=1):
    g0 = oracle.init_grid(L, N, vmax, seed, init_v=init_v)
    x, v = oracle.grid_to_agent(g0)
    return oracle.run_agent_mlcg(L, x, v, vmax, p, seed, T)


@pytest.mark.parametrize("kernel,k", [("onestep", 0), ("kstep", 1), ("kstep", 7), ("kstep", 32),
                                      ("kstep", 100)])
@pytest.mark.parametrize("L,N", [(1000, 200), (30011, 9000), (40, 3), (5000, 513)])
def test_stream_mode_matches_serial_oracle(kernel, k, L, N):
    vmax, p, seed, T = 5, 0.13, 77, 150
    xo, vo, fo = _oracle(L, N, vmax, p, seed, T)
    s = Sim(L, N, vmax, p, seed, rep="agent", rng="stream", init_v=1, kernel=kernel,
            k=k if k else 0)
    s.step(T)
    x, v = s.agent_state()
    np.testing.assert_array_equal(x, xo)
    np.testing.assert_array_equal(v, vo)
    np.testing.assert_array_equal(s.flux(0, T), fo)
    s.close()


def test_stream_mode_restore_agent_resumes_exactly():
    L, N, vmax, p, seed = 20000, 5000, 5, 0.25, 5
    a = Sim(L, N, vmax, p, seed, rep="agent", rng="stream", init_v=1)
    a.step(120)
    xm, vm = a.agent_state()
    a.step(80)
    xe, ve = a.agent_state()
    b = Sim(L, N, vmax, p, seed + 1, rep="agent", rng="stream")
    with pytest.raises(NaschError):
        b.restore_agent(xm[::-1].copy(), vm, 120)   # not in road order
    b2 = Sim(L, N, vmax, p, seed, rep="agent", rng="stream")
    b2.restore_agent(xm, vm, 120)
    b2.step(80)
    x, v = b2.agent_state()
    np.testing.assert_array_equal(x, xe)
    np.testing.assert_array_equal(v, ve)
    for s in (a, b, b2):
        s.close()


def test_stream_mode_only_in_agent_form():
    with pytest.raises(NaschError):
        Sim(1000, 100, 5, 0.1, 1, rep="grid", rng="stream")


@pytest.fixture(scope="module")
def far_stream_case():
    """2^24 + 2^20 cars on 2^26 cells restored at step 2^32 - 60: their numbers
    n = t N + i + 1 lie near 2^56, so the device's jump-ahead reads the
    digits of n up to 16^14.  The oracle starts from the generator state
    x0 a^(t N) mod m, computed with Python's exact modular power (the state
    after t N draws of the stream), and then draws serially."""
    L, N, vmax, p, seed, t0, T = 1 << 26, (1 << 24) + (1 << 20), 5, 0.13, 9, (1 << 32) - 60, 50
    g0 = oracle.init_grid(L, N, vmax, seed, init_v=1)
    x0, v0 = oracle.grid_to_agent(g0)
    m = (1 << 31) - 1
    state = oracle.mlcg_seed(seed) * pow(48271, t0 * N, m) % m
    assert (t0 + T) * N >= 16 ** 14
    want = oracle.run_agent_mlcg(L, x0, v0, vmax, p, seed, T, state0=state)
    return dict(L=L, N=N, vmax=vmax, p=p, seed=seed, t0=t0, T=T, x0=x0, v0=v0, want=want)


@pytest.mark.parametrize("kernel,k", [("kstep", 16), ("onestep", 0)])
def test_stream_mode_far_into_the_stream(far_stream_case, kernel, k):
    c = far_stream_case
    s = Sim(c["L"], c["N"], c["vmax"], c["p"], c["seed"], rep="agent", rng="stream",
            kernel=kernel, k=k)
    s.restore_agent(c["x0"], c["v0"], c["t0"])
    s.step(c["T"])
    x, v = s.agent_state()
    xo, vo, fo = c["want"]
    np.testing.assert_array_equal(x, xo)
    np.testing.assert_array_equal(v, vo)
    np.testing.assert_array_equal(s.flux(c["t0"], c["T"]), fo)
    s.close()


@pytest.mark.parametrize("vmax", [9, 254])
@pytest.mark.parametrize("kernel,k", [("onestep", 0), ("kstep", 16)])
def test_stream_mode_any_vmax(vmax, kernel, k):
    """The shared stream with vmax beyond the grid form's 8 (the agent form
    takes any vmax up to 254), against the serial oracle."""
    L, N, p, seed, T = 20011, 400, 0.3, 9, 80
    xo, vo, fo = _oracle(L, N, vmax, p, seed, T)
    s = Sim(L, N, vmax, p, seed, rep="agent", rng="stream", init_v=1, kernel=kernel, k=k)
    s.step(T)
    x, v = s.agent_state()
    np.testing.assert_array_equal(x, xo)
    np.testing.assert_array_equal(v, vo)
    np.testing.assert_array_equal(s.flux(0, T), fo)
    s.close()
