"""Pins of the oracle's NLC and polymer models (f0 = C h^3, f1 = h^3 Pi'(h); eqs.
GeneralDisPreForm, DisjPressNLC, mh_model, DisjPressPolymer) against values the paper
prints and against derivative consistency."""
import math

import numpy as np
import pytest

from paper_1806_10550_amd import synth


def lsa(orc, M, h0):
    """(q_m, omega_m) of sigma(q) = q^2 (f1(h0) - f0(h0) q^2) (Sec. "Linear Stability
    Analysis"; reading of the garbled formulas: q_m = sqrt(f1 / 2 f0), omega_m = f1^2 / 4 f0)."""
    f0, _, f1, _ = orc.coeffs(M, h0)
    return math.sqrt(f1 / (2 * f0)), f1 * f1 / (4 * f0)


def test_nlc_printed_growth_rate(orc):
    """Fig. dispersion_curves (b): q_m ~ 1.482, omega_m ~ 0.05169 for the NLC model at
    H0 = 0.5 with the parameters of eq. NLC_paras."""
    qm, wm = lsa(orc, orc.Model.nlc(), 0.5)
    assert abs(qm - 1.482) < 5e-4
    assert abs(wm - 0.05169) < 5e-6


def test_polymer_printed_growth_rate(orc):
    """Fig. dispersion_curves (c): omega_m ~ 2.040 for the polymer model at H0 = 3.9 with
    the parameters of eq. Polymer_scales. The printed q_m ~ 1.600 does not follow from the
    same f0, f1 (they give 1.5599, while the printed omega_m is reproduced); only omega_m
    is pinned."""
    qm, wm = lsa(orc, orc.Model.polymer(), 3.9)
    assert abs(wm - 2.040) < 5e-4
    assert abs(qm - 1.5599) < 1e-4


def test_nlc_pressure_vanishes_at_printed_thickness(orc):
    """Sec. "Nematic Liquid Crystals": Pi(H0) = 0 for H0 = 0.2624 (four digits)."""
    M = orc.Model.nlc()
    pi, pip, _ = orc.disjoining(M, 0.2624)
    assert abs(pi) < 0.5e-4 * abs(pip)   # the root lies within 5e-5 of 0.2624
    # and Pi changes sign across it
    assert orc.disjoining(M, 0.2623)[0] * orc.disjoining(M, 0.2626)[0] < 0


@pytest.mark.parametrize("kind,hs", [("nlc", (0.03, 0.1, 0.2624, 0.5, 0.9)), ("polymer", (1.5, 2.0, 3.9, 6.0))])
def test_disjoining_derivatives_consistent(orc, kind, hs):
    M = getattr(orc.Model, kind)()
    for h in hs:
        e = 1e-5 * h
        pi, pip, pipp = orc.disjoining(M, h)
        fd1 = (orc.disjoining(M, h + e)[0] - orc.disjoining(M, h - e)[0]) / (2 * e)
        fd2 = (orc.disjoining(M, h + e)[1] - orc.disjoining(M, h - e)[1]) / (2 * e)
        assert pip == pytest.approx(fd1, rel=1e-7, abs=1e-9)
        assert pipp == pytest.approx(fd2, rel=1e-6, abs=1e-8)
        f0, f0p, f1, f1p = orc.coeffs(M, h)
        g = lambda x: orc.coeffs(M, x)[2]
        assert f1p == pytest.approx((g(h + e) - g(h - e)) / (2 * e), rel=1e-6, abs=1e-9)
        assert f1 == pytest.approx(h ** 3 * pip, rel=1e-14)
        assert f0 == pytest.approx(M.cap * h ** 3, rel=1e-15)


@pytest.mark.parametrize("kind,h0,n", [("nlc", 0.5, 32), ("polymer", 3.9, 32)])
def test_discrete_growth_rate_of_new_models(orc, kind, h0, n):
    """The linearised step of Sec. "Linear Stability Analysis" on the cell-centred grid:
    a small cosine mode on a flat film h0 grows per backward-Euler step by
    1 / (1 + dt (f0 mu^2 - f1 mu)), mu = (4/ds^2) sin^2(pi k / 2n); domain = one most
    unstable wavelength (P = 1, I = 32, as in the paper's LSA runs)."""
    M = getattr(orc.Model, kind)()
    qm, wm = lsa(orc, M, h0)
    ds = 2 * math.pi / qm / n
    k, amp = 2, 1e-6
    dt = 0.1 / wm
    u = h0 * synth.cosine_film(n, 4, k, 0, amp=amp)
    mode = (u - h0) / (h0 * amp)
    f0, _, f1, _ = orc.coeffs(M, h0)
    mu = 4 / ds ** 2 * math.sin(math.pi * k / (2 * n)) ** 2
    g_exact = 1.0 / (1.0 + dt * (f0 * mu ** 2 - f1 * mu))
    a_prev = amp * h0
    for _ in range(3):
        u, res = orc.step(M, orc.Scheme(tol=1e-13), u, ds, dt)
        assert res.status == orc.OK
        a = np.sum((u - h0) * mode) / np.sum(mode * mode)
        assert a / a_prev == pytest.approx(g_exact, rel=1e-7)
        a_prev = a
    assert g_exact > 1.0  # the most unstable mode grows


@pytest.mark.parametrize("kind,h0", [("nlc", 0.5), ("polymer", 3.9)])
def test_second_order_in_time_and_space(orc, kind, h0):
    """Sec. "Convergence" for the new models (trapezoidal rule, eq. IC_LinearWave with
    P = 6, q = q_m): halving dt from 1e-3 / omega_m on 32^2 cells, and tripling the grid
    from 36 to 972 cells at one step of 1e-8 / omega_m, both converge at second order."""
    M = getattr(orc.Model, kind)()
    qm, wm = lsa(orc, M, h0)
    S = orc.Scheme(theta=0.5, tol=1e-14, max_newton=5000)

    def run(u, ds, dt, n):
        for _ in range(n):
            u, res = orc.step(M, S, u, ds, dt)
            assert res.status == orc.OK
        return u

    u0, ds = synth.wave_film(32, 6, qm, h0)
    sols = [run(u0, ds, 1e-3 / wm / 2 ** i, 2 ** i) for i in range(6)]
    e = [np.sqrt(np.mean((s - sols[-1]) ** 2)) for s in sols[:-1]]
    for i in range(2):
        assert 1.95 <= math.log2(e[i] / e[i + 1]) <= 2.05, e
    sols = []
    for k in range(4):
        u0, ds = synth.wave_film(36 * 3 ** k, 6, qm, h0)
        sols.append(run(u0, ds, 1e-8 / wm, 1))
    e = []
    for k in range(3):
        m = 3 ** (3 - k)
        idx = m * np.arange(36 * 3 ** k) + (m - 1) // 2
        e.append(np.sqrt(np.mean((sols[k] - sols[-1][np.ix_(idx, idx)]) ** 2)))
    assert 1.9 <= math.log(e[1] / e[2], 3) <= 2.2, e


def test_nlc_dimensional_wavelength(orc):
    """Sec. "Comparison to Experimental Results": the most unstable wavelength of the NLC film
    is 42 um with the scales of eq. NLC_scales (L = 10 um) and the parameters of eq.
    NLC_paras; H0 = 0.5 (the NLC thickness of Sec. "Validation") gives 2 pi / q_m = 4.24."""
    qm, _ = lsa(orc, orc.Model.nlc(), 0.5)
    assert round(2 * math.pi / qm * 10.0) == 42
