"""Pins of the radial-Fourier-transform oracle (App. "Radial Fourier Transform") against
closed forms: single Fourier modes, the transform of a Gaussian bump, exactly
piecewise-linear data, moving averages of linear data and the maxima of smooth curves."""
import math

import numpy as np
import pytest

from oracle import radial as R


def test_single_mode_lands_in_its_group():
    """zeta = A cos(2 pi k0 i / n): |F| / n^2 = A/2 at (+-k0, 0), 0 elsewhere; the group
    m = k0^2 (for k0 = 7 only (+-7, 0), (0, +-7)) averages to A/4."""
    n, k0, A, ds = 64, 7, 0.3, 0.5
    x = np.arange(n)
    h = 1.0 + A * np.cos(2 * np.pi * k0 * x / n)[None, :] * np.ones((n, 1))
    q, y, c = R.radial_spectrum(h, 1.0, ds, 0.0, 2 * math.pi * 20 / (n * ds))
    L = n * ds
    j = int(np.argmin(np.abs(q - 2 * math.pi * k0 / L)))
    assert c[j] == 4
    assert y[j] == pytest.approx(A / 4, rel=1e-12)
    assert np.max(np.abs(np.delete(y, j))) <= 1e-15


def test_gaussian_weights_and_sum_conservation():
    for sigma in (0.7, 1.0, 2.5):
        w = R.gaussian_weights(sigma)
        assert np.sum(w) == pytest.approx(1.0, rel=1e-15)
        r = (len(w) - 1) // 2
        assert w[r + 1] / w[r] == pytest.approx(math.exp(-1 / (2 * sigma * sigma)), rel=1e-14)
    a = np.random.default_rng(0).uniform(size=(32, 32))
    s = R.smooth(a, 1.5)
    assert np.sum(s) == pytest.approx(np.sum(a), rel=1e-13)  # periodic convolution keeps the sum
    d = np.zeros((32, 32))
    d[0, 0] = 1.0
    s = R.smooth(d, 1.0)
    w = R.gaussian_weights(1.0)
    assert s[1, 2] == pytest.approx(w[4 + 1] * w[4 + 2], rel=1e-14)
    assert s[-1, -3] == pytest.approx(w[4 - 1] * w[4 - 3], rel=1e-14)


def test_gaussian_bump_has_gaussian_radial_spectrum():
    """h = H0 + A exp(-r^2 / w^2) (w << L): the continuous transform is
    pi w^2 A exp(-q^2 w^2 / 4), so the radial data fall off as exp(-q^2 w^2 / 4)."""
    n, ds, w = 256, 0.25, 2.0
    c = (np.arange(n) + 0.5) * ds - n * ds / 2
    r2 = c[None, :] ** 2 + c[:, None] ** 2
    h = 1.0 + 0.1 * np.exp(-r2 / w ** 2)
    q, y, _ = R.radial_spectrum(h, 1.0, ds, 0.0, 3.0)
    ref = y[0] * np.exp(-(q ** 2 - q[0] ** 2) * w * w / 4)
    assert np.max(np.abs(y - ref)) <= 1e-9 * y[0]
    L = n * ds
    assert y[0] == pytest.approx(0.1 * math.pi * w * w / L ** 2 * math.exp(-q[0] ** 2 * w * w / 4), rel=1e-9)


def test_piecewise_fit_recovers_piecewise_linear_data():
    q = np.sort(np.random.default_rng(1).uniform(0.05, 4.9, 57))
    qmax = 5.0
    t = R.knots(q, qmax)
    assert len(t) == 6 and t[0] == 0 and t[-1] == qmax
    vals = np.array([0.0, 1.3, -0.4, 2.2, 0.7, 1.1])
    y = np.interp(q, t, vals)
    t2, a = R.piecewise_fit(q, y, qmax)
    assert np.array_equal(t, t2)
    assert np.max(np.abs(a - vals)) <= 1e-12
    # least squares: perturbing the fit never lowers the residual
    y2 = y + np.random.default_rng(2).normal(0, 0.1, len(q))
    _, a2 = R.piecewise_fit(q, y2, qmax)
    res = lambda aa: np.sum((np.interp(q, t, aa) - y2) ** 2)
    base = res(a2)
    for k in range(1, 6):
        for e in (1e-3, -1e-3):
            b = a2.copy()
            b[k] += e
            assert res(b) > base


def test_moving_average():
    x = np.linspace(0, 3, 50)
    v = 2.0 * x - 1.0
    for half in (1, 2, 3):
        m = R.moving_average(v, half)
        assert np.allclose(m[half:-half], v[half:-half], rtol=0, atol=1e-14)
    c = np.full(20, 0.7)
    assert np.allclose(R.moving_average(c, 3), c, rtol=0, atol=4e-16)
    assert R.moving_average(np.arange(5.0), 3)[0] == pytest.approx(np.mean([0, 1, 2, 3]))


def test_local_maxima_of_smooth_curves():
    """q^2 exp(-q) peaks at q = 2; sin has maxima at pi/2 + 2 pi k; minima are not reported."""
    x = np.linspace(0, 10, 400)
    p = R.local_maxima(x, x * x * np.exp(-x))
    assert len(p) == 1
    assert p[0][0] == pytest.approx(2.0, abs=2e-4)
    assert p[0][1] == pytest.approx(4 * math.exp(-2), rel=1e-4)
    x = np.linspace(0, 14, 400)
    p = R.local_maxima(x, np.sin(x))
    assert [round(v[0], 3) for v in p] == [round(math.pi / 2, 3), round(5 * math.pi / 2, 3)]


def test_ring_of_modes_peaks_at_its_wavenumber():
    """A film whose perturbation holds the modes |k| = 10 in several directions: the single
    maximum of the smoothed radial spectrum lies at q0 = 2 pi 10 / L (within the 400-point
    resolution)."""
    n, ds = 128, 0.3
    L = n * ds
    x = (np.arange(n) + 0.5) * ds
    X, Y = np.meshgrid(x, x)
    kk = [(10, 0), (0, 10), (6, 8), (8, 6)]
    h = 1.0 + sum(0.01 * np.cos(2 * np.pi * (a * X + b * Y) / L) for a, b in kk)
    q0 = 2 * math.pi * 10 / L
    peaks = R.dominant_wavenumbers(h, 1.0, ds, 1.0, 5 * q0 / 2)
    top = max(peaks, key=lambda p: p[1])
    assert abs(top[0] - q0) <= 0.05 * q0
