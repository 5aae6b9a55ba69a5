"""Parity at the full workload sizes, in the launch configuration bench.py times.

* 2048^2 spinodal and nucleation films (L = 64 lambda_m, adaptive dt from 0.1 with
  K = 10): the first accepted steps, every cell, dt schedule and rejections.
* 8192^2 film (L = 256 lambda_m, dt = 0.2): one full Newton iteration, every cell, and
  the reduction record; the whole first accepted step (every Newton iteration of it)
  against the oracle's step, every cell.
* 2048^2 nucleation film near the pre-rupture horizon: from the GPU state at which min h
  first falls below 0.6, the oracle replays the next 20 accepted steps with the GPU's dt
  and iteration counts; every cell to 1e-10.
* 16384^2 film: one Newton iteration (largest size exercised).
* 2048^2 spinodal over many steps on the GPU alone: mass to 1e-12, positivity.
"""
import numpy as np
import pytest
import torch

from paper_1806_10550_amd import synth
from paper_1806_10550_amd.lib import Grid

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

ADAPT = dict(tol=1e-10, max_newton=10, adaptive=1, dt_min=1e-6, dt_max=1.0, dt_shrink=0.5, dt_grow=1.1,
             grow_after=5)


@pytest.fixture(scope="module", autouse=True)
def threads(orc):
    import os
    orc.set_threads(len(os.sched_getaffinity(0)))


@pytest.mark.parametrize("name", ["spinodal2048", "nucleation2048"])
def test_2048_first_steps_match_oracle(orc, name):
    cfg = synth.CONFIGS[name]
    h0 = cfg.film()
    g = Grid(cfg.n, cfg.n, cfg.ds)
    g.set_model(10.0, 0.1, 3, 2)
    g.set_scheme(**ADAPT)
    h = torch.from_numpy(h0).to(DEV)
    g.bind(h)
    nsteps = 4
    _, log = g.advance(nsteps, cfg.dt, log=True)
    M = orc.Model()
    S = orc.Scheme(theta=1.0, **ADAPT)
    u, dt, succ = h0, cfg.dt, 0
    for s in range(nsteps):
        u, res = orc.step(M, S, u, cfg.ds, dt, succ)
        assert res.status == orc.OK
        assert log[s]["dt_used"] == res.dt_used and log[s]["rejections"] == res.rejections
        assert log[s]["newton_iters"] == res.newton_iters
        dt, succ = res.dt_next, res.successes
    got = h.cpu().numpy()
    assert np.max(np.abs(got - u) / u) <= 1e-10


def test_8192_newton_iteration_matches_oracle(orc):
    cfg = synth.CONFIGS["large8192"]
    h0 = cfg.film()
    g = Grid(cfg.n, cfg.n, cfg.ds)
    g.set_model(10.0, 0.1, 3, 2)
    g.set_scheme(theta=1.0, tol=1e-10)
    un = torch.from_numpy(h0).to(DEV)
    out = torch.empty_like(un)
    e, r, flags = g.newton_iteration(un, un, out, cfg.dt)
    ref, e_ref, r_ref = orc.adi_iteration(orc.Model(), h0, h0, cfg.ds, cfg.dt, 1.0)
    got = out.cpu().numpy()
    v = ref - h0
    assert flags == 0
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(v))
    assert e == pytest.approx(e_ref, rel=1e-9)
    assert r == pytest.approx(r_ref, rel=1e-9)


def test_8192_first_accepted_step_matches_oracle(orc):
    """The whole first step of the 8192^2 workload (fixed dt = 0.2, tol 1e-10) from the noise
    film: the rough initial noise needs the most Newton iterations of the run. Same
    iteration count as the oracle's step (Fig. FlowChartTime with a fixed dt) and every cell
    to 1e-10 relative."""
    cfg = synth.CONFIGS["large8192"]
    h0 = cfg.film()
    g = Grid(cfg.n, cfg.n, cfg.ds)
    g.set_model(10.0, 0.1, 3, 2)
    g.set_scheme(theta=1.0, tol=cfg.tol, max_newton=5000, adaptive=0)
    h = torch.from_numpy(h0).to(DEV)
    g.bind(h)
    res = g.step(cfg.dt)
    got = h.cpu().numpy()
    del h
    g.close()
    torch.cuda.empty_cache()
    ref, r = orc.step(orc.Model(), orc.Scheme(theta=1.0, tol=cfg.tol, max_newton=5000, adaptive=0), h0, cfg.ds,
                      cfg.dt)
    assert r.status == orc.OK and res.info["status"] == 0
    assert res.info["newton_iters"] == r.newton_iters, (res.info["newton_iters"], r.newton_iters)
    assert res.info["newton_iters"] >= 6
    assert np.max(np.abs(got - ref) / ref) <= 1e-10


def test_2048_near_horizon_window_matches_oracle_replay(orc):
    """The 2048^2 nucleation film (Gaussian depression of depth 0.3 over noise, adaptive dt
    from 0.1 with K = 10) run on the GPU until min h first falls below 0.6, where the
    depression has deepened by a factor of about 1.5 on its way to rupture. From that state
    the oracle replays the next 20 accepted steps with the GPU's dt and Newton iteration
    count per step (A10); h agrees to 1e-10 relative after every 5 steps, and the oracle's
    own test takes the GPU's accept decision at all but at most two knife edges."""
    cfg = synth.CONFIGS["nucleation2048"]
    g = Grid(cfg.n, cfg.n, cfg.ds)
    g.set_model(10.0, 0.1, 3, 2)
    g.set_scheme(**ADAPT)
    g.set_diagnostics(True)
    h = torch.from_numpy(cfg.film()).to(DEV)
    g.bind(h)
    dt, steps = cfg.dt, 0
    while True:
        dt, log = g.advance(1, dt, log=True)
        steps += 1
        assert steps < 3000
        if log[0]["hmin"] < 0.6:
            break
    start = h.cpu().numpy()
    logs, snaps = [], {}
    for _ in range(4):
        dt, log = g.advance(5, dt, log=True)
        logs += log
        snaps[len(logs)] = h.cpu().numpy()
    g.close()
    M = orc.Model()
    u, disagree = start, 0
    for s, x in enumerate(logs):
        uk = u
        for k in range(x["newton_iters"]):
            uk, e, _ = orc.adi_iteration(M, u, uk, cfg.ds, x["dt_used"], 1.0)
            if (e < ADAPT["tol"]) != (k == x["newton_iters"] - 1):
                disagree += 1
        u = uk
        if s + 1 in snaps:
            rel = np.max(np.abs(snaps[s + 1] - u) / u)
            assert rel <= 1e-10, (steps, s + 1, rel)
    assert disagree <= 2, disagree
    assert min(x["hmin"] for x in logs) < 0.6


def test_16384_newton_iteration_matches_oracle(orc):
    """Largest size exercised: 16384^2 (2.1 GB per field), L = 512 lambda_m; one Newton
    iteration of the bench's launch configuration against the oracle."""
    n = 16384
    ds = 512 * synth.lambda_m(10.0) / n
    h0 = synth.noise_film(n, n, seed=7, amp=0.01)
    g = Grid(n, n, ds)
    g.set_model(10.0, 0.1, 3, 2)
    g.set_scheme(theta=1.0, tol=1e-10)
    un = torch.from_numpy(h0).to(DEV)
    out = torch.empty_like(un)
    e, r, flags = g.newton_iteration(un, un, out, 0.2)
    got = out.cpu().numpy()
    del out, un
    g.close()
    torch.cuda.empty_cache()
    ref, e_ref, r_ref = orc.adi_iteration(orc.Model(), h0, h0, ds, 0.2, 1.0)
    assert flags == 0
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref - h0))
    assert e == pytest.approx(e_ref, rel=1e-9)
    assert r == pytest.approx(r_ref, rel=1e-9)


def test_2048_long_run_mass_and_positivity():
    cfg = synth.CONFIGS["spinodal2048"]
    h0 = cfg.film()
    g = Grid(cfg.n, cfg.n, cfg.ds)
    g.set_model(10.0, 0.1, 3, 2)
    g.set_scheme(**ADAPT)
    g.set_diagnostics(True)
    h = torch.from_numpy(h0).to(DEV)
    g.bind(h)
    m0, _ = g.mass()
    dt = cfg.dt
    for _ in range(4):
        dt, log = g.advance(50, dt, log=True)
        for x in log:
            assert abs(x["mass"] - m0) <= 1e-12 * m0
            assert x["hmin"] > 0.0
    assert torch.isfinite(h).all()


@pytest.mark.parametrize("name", ["spinodal2048", "nucleation2048"])
def test_2048_through_rupture(name):
    """The two 2048^2 films of the benchmark set, 2000 adaptive steps from dt = 0.1 (K = 10):
    every step is accepted in the end, mass is conserved to 1e-12 at every step, h stays
    positive, and the film reaches the precursor scale (min h < 0.2, b = 0.1): the run goes
    through rupture onset (t ~ 820 for the noise film, ~ 130 with the Gaussian depression)."""
    cfg = synth.CONFIGS[name]
    g = Grid(cfg.n, cfg.n, cfg.ds)
    g.set_model(10.0, 0.1, 3, 2)
    g.set_scheme(**ADAPT)
    g.set_diagnostics(True)
    h = torch.from_numpy(cfg.film()).to(DEV)
    g.bind(h)
    m0, _ = g.mass()
    dt, hmin = cfg.dt, 1.0
    for _ in range(40):
        dt, log = g.advance(50, dt, log=True)
        for x in log:
            assert abs(x["mass"] - m0) <= 1e-12 * m0
            assert x["hmin"] > 0.0
            hmin = min(hmin, x["hmin"])
    assert hmin < 0.2
    assert torch.isfinite(h).all()
