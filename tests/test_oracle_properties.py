"""Property-based checks of the oracle's step (Sec. "Conservation Law", Sec. "Boundary
Conditions"): on random small grids, models, time steps and films, one converged step conserves mass,
commutes with the reflections x -> L - x and y -> L - y (and with the transpose on square
grids), and leaves a flat film unchanged bit for bit."""
import numpy as np
import pytest
from hypothesis import HealthCheck, assume, given, settings
from hypothesis import strategies as st

MODELS = st.sampled_from(["power32", "power43", "power93", "linear", "nlc", "polymer"])


def make(orc, kind):
    if kind.startswith("power"):
        return orc.Model(kappa=10.0, b=0.1, n=float(kind[5]), m=float(kind[6])), 1.0
    if kind == "linear":
        return orc.Model(kind=orc.LINEAR, c0=1.0, c1=1.0), 1.0
    if kind == "nlc":
        return orc.Model.nlc(), 0.5
    return orc.Model.polymer(), 3.9


@settings(max_examples=300, derandomize=True, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(kind=MODELS, nx=st.integers(3, 11), ny=st.integers(3, 11), theta=st.sampled_from([0.5, 1.0]),
       dtf=st.floats(0.01, 1.0), dsf=st.floats(0.5, 2.0), seed=st.integers(0, 2 ** 31 - 1))
def test_step_invariants(orc, kind, nx, ny, theta, dtf, dsf, seed):
    M, h0 = make(orc, kind)
    f0, _, f1, _ = orc.coeffs(M, h0)
    ds = dsf * np.pi / np.sqrt(abs(f1) / (2 * f0) + 1e-3) / 4
    dt = dtf * ds ** 4 / f0 * 0.1
    u = h0 * (1.0 + 0.05 * np.random.default_rng(seed).uniform(-1, 1, (ny, nx)))
    S = orc.Scheme(theta=theta, tol=1e-13, max_newton=5000)
    v, res = orc.step(M, S, u, ds, dt)
    # the largest steps drawn can leave the Newton iteration's basin (Fig. FlowChartTime would
    # shrink dt); the invariants concern converged steps
    assume(res.status == orc.OK)
    # mass
    assert abs(v.sum() - u.sum()) <= 1e-13 * u.sum()
    # reflections
    vx, rx = orc.step(M, S, u[:, ::-1], ds, dt)
    vy, ry = orc.step(M, S, u[::-1, :], ds, dt)
    assert rx.status == orc.OK and ry.status == orc.OK
    scale = np.max(np.abs(v - u)) + 1e-300
    assert np.max(np.abs(vx[:, ::-1] - v)) <= 1e-9 * scale + 1e-14 * h0
    assert np.max(np.abs(vy[::-1, :] - v)) <= 1e-9 * scale + 1e-14 * h0
    if nx == ny:
        vt, rt = orc.step(M, S, u.T.copy(), ds, dt)
        assert rt.status == orc.OK
        assert np.max(np.abs(vt.T - v)) <= 1e-9 * scale + 1e-14 * h0
    # a flat film is a steady state
    flat = np.full((ny, nx), h0)
    w, rw = orc.step(M, S, flat, ds, dt)
    assert rw.status == orc.OK and np.array_equal(w, flat)
