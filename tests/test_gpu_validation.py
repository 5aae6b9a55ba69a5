"""The paper's validation suite (Sec. "Validation": convergence, conservation of mass,
comparison to LSA) run on the GPU for the linear, NLC and polymer models: the GPU runs of
paper_1806_10550_amd.validate are compared with the same runs made here by the CPU oracle,
and the GPU's convergence orders, mass drift and growth rates are checked against what the
paper states (second order in time and space, mass conserved to rounding, growth rates on
the dispersion curve).

The oracle-side runs below are written independently of validate.py: only the inputs
(synth.wave_film) are shared.
"""
import math

import numpy as np
import pytest

from paper_1806_10550_amd import synth
from paper_1806_10550_amd import validate as V

pytestmark = pytest.mark.gpu
KINDS = ["linear", "nlc", "polymer"]


def omodel(orc, kind):
    if kind == "linear":
        return orc.Model(kind=orc.LINEAR, c0=1.0, c1=1.0)
    return getattr(orc.Model, kind)()


def o_lsa(orc, kind):
    h0 = V.MODELS[kind]
    f0, _, f1, _ = orc.coeffs(omodel(orc, kind), h0)
    return h0, f0, f1, math.sqrt(f1 / (2 * f0)), f1 * f1 / (4 * f0)


def o_run(orc, kind, u, ds, dt, nsteps, tol):
    S = orc.Scheme(theta=0.5, tol=tol, max_newton=5000)
    M = omodel(orc, kind)
    for _ in range(nsteps):
        u, res = orc.step(M, S, u, ds, dt)
        assert res.status == orc.OK
    return u


@pytest.mark.parametrize("kind", KINDS)
def test_lsa_params_match_oracle(orc, kind):
    got = V.lsa_params(kind)
    ref = o_lsa(orc, kind)
    assert got == pytest.approx(ref, rel=1e-14)


@pytest.mark.parametrize("kind", KINDS)
def test_temporal_convergence_matches_oracle(orc, kind):
    """80 x 80 cells (a full and a ragged tile), dt_i = 2^-i dt0 for i = 0..3, tolerance
    1e-14: every level's solution equals the oracle's to 1e-13 H0."""
    sols, dt0 = V.temporal_solutions(kind, I0=80, levels=3)
    h0, _, _, qm, wm = o_lsa(orc, kind)
    assert dt0 == pytest.approx(1e-3 / wm, rel=1e-14)
    u0, ds = synth.wave_film(80, 6, qm, h0)
    for i, s in enumerate(sols):
        ref = o_run(orc, kind, u0, ds, dt0 / 2 ** i, 2 ** i, 1e-14)
        assert np.max(np.abs(s - ref)) <= 1e-13 * h0, i


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("tol", ["machine", "scaled"])
def test_temporal_order_two(kind, tol):
    """Paper's sizes (I0 = 256, six halvings): the trapezoidal rule converges at second
    order with tolerance 1e-14 (Fig. TimeConvergence, solid curves); with the tolerance
    max(dt^2, 1e-14) at least at second order (the coarse levels stop Newton early, which
    for the nonlinear models makes the error larger and the observed order higher, as the
    paper reports). The last two ratios are biased by the finite reference."""
    r = V.temporal(kind, I0=256, levels=6, tol_mode=tol)
    for o in r["orders"][:3]:
        if tol == "machine":
            assert 1.95 <= o <= 2.05, r["orders"]
        else:
            assert o >= 1.95, r["orders"]


@pytest.mark.parametrize("kind", KINDS)
def test_spatial_convergence_matches_oracle(orc, kind):
    """I = 36, 108, 324, one step of 1e-8 / omega_m: solutions equal the oracle's."""
    sols, dt = V.spatial_solutions(kind, I0=36, levels=3)
    h0, _, _, qm, wm = o_lsa(orc, kind)
    for k, s in enumerate(sols):
        u0, ds = synth.wave_film(36 * 3 ** k, 6, qm, h0)
        ref = o_run(orc, kind, u0, ds, dt, 1, 1e-14)
        assert np.max(np.abs(s - ref)) <= 1e-13 * h0, k


@pytest.mark.parametrize("kind", KINDS)
def test_spatial_order(kind):
    """I = 36 * 3^k up to 2916 (Fig. SpaceConvergence): second order for NLC and polymer
    at the finest levels. For the linear model at q = q_m the growth rate is stationary in
    the discrete wavenumber (d omega / d mu = f1 - 2 f0 mu = 0 at mu = q_m^2), so the
    O(ds^2) error of mu enters only squared and the observed order is four."""
    r = V.spatial(kind, I0=36, levels=5)
    o = r["orders"]
    if kind == "linear":
        assert o[0] >= 3.8 and o[1] >= 3.8, o
    else:
        assert 1.9 <= o[-1] <= 2.2 and 1.9 <= o[-2] <= 2.2, o


@pytest.mark.parametrize("kind", KINDS)
def test_mass_matches_oracle_and_is_conserved(orc, kind):
    """1000 steps of 1e-8 / omega_m on 108^2 (tolerance max(ds^2, 1e-14)): the GPU's mean
    thickness changes by at most 1e-13 relative (Fig. CoM), and its final state equals
    the oracle's."""
    r = V.mass(kind, "space", 1)
    assert r["max_abs"] <= 1e-13, r["rel_mass_change"]
    h0, _, _, qm, wm = o_lsa(orc, kind)
    u0, ds = synth.wave_film(108, 6, qm, h0)
    sols, rel = V._run(kind, u0, ds, r["dt"], 1000, max(ds * ds, 1e-14), sample_every=1000)
    ref = o_run(orc, kind, u0, ds, r["dt"], 1000, max(ds * ds, 1e-14))
    assert np.max(np.abs(sols - ref)) <= 1e-12 * h0
    assert abs(np.sum(ref) / np.sum(u0) - 1.0) <= 1e-13


@pytest.mark.parametrize("kind", KINDS)
def test_mass_time_family(kind):
    """I = 1024, 1000 steps of 1e-3 / omega_m (tolerance max(dt^2, 1e-14))."""
    r = V.mass(kind, "time", 0)
    assert r["max_abs"] <= 1e-13, r["rel_mass_change"]


def o_lsa_rate(orc, kind, frac, eps, axis, I=32):
    h0, f0, f1, qm, wm = o_lsa(orc, kind)
    q = frac * qm
    w = q * q * (f1 - f0 * q * q)
    T = math.log(1.3) / abs(w)
    u0, ds = synth.wave_film(I, 1, q, h0, eps if axis == "x" else 0.0, eps if axis == "y" else 0.0)
    M = omodel(orc, kind)
    S = orc.Scheme(theta=0.5, tol=1e-10, adaptive=1, max_newton=10, dt_min=1e-9, dt_max=1.0)
    u, t, dt, succ, steps = u0, 0.0, T / 100.0, 0, 0
    while t < T * (1.0 - 1e-14):
        u, res = orc.step(M, S, u, ds, min(dt, T - t), succ)
        assert res.status == orc.OK
        t += res.dt_used
        dt, succ = res.dt_next, res.successes
        steps += 1
    x = np.cos(q * ds * (np.arange(I) + 0.5))
    mode = np.outer(np.ones(I), x) if axis == "x" else np.outer(x, np.ones(I))
    amp = lambda v: float(np.sum((v - h0) * mode))
    return math.log(amp(u) / amp(u0)) / T, w, wm, steps


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("axis", ["x", "y"])
@pytest.mark.parametrize("eps", [0.1, 1e-3])
def test_lsa_growth_rates(orc, kind, axis, eps):
    """P = 1, I = 32 (Sec. "Comparison to LSA"): the GPU's growth rates equal the oracle's
    (same adaptive schedule); with a small perturbation they lie on the dispersion curve to
    1.2 % of omega_m (the O(ds^2) error of the 32-cell wavelength)."""
    for frac in (0.5, 1.0, 1.375):
        r = V.lsa_rate(kind, frac, eps, axis)
        ws, w, wm, steps = o_lsa_rate(orc, kind, frac, eps, axis)
        assert r["steps"] == steps
        assert r["omega_sim"] == pytest.approx(ws, rel=1e-8, abs=1e-10 * wm)
        assert r["omega_lsa"] == pytest.approx(w, rel=1e-13)
        if eps < 0.01:
            assert abs(r["omega_sim"] - w) <= 0.012 * wm, (frac, r)
