"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: exact invariants,
closed forms (DCT diagonalisation, linear stability), library routines (SciPy),
finite differences, brute-force dense Newton, convergence orders. The citations
refer to Lam, Cummings & Kondic, arXiv:1806.10550.
"""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.linalg

from paper_1806_10550_amd import synth

PL = dict(kappa=10.0, b=0.1, n=3.0, m=2.0)


def model(orc, **kw):
    p = dict(PL)
    p.update(kw)
    return orc.Model(**p)


# ---------------------------------------------------------------- model functions
def test_model_functions_match_definition(orc):
    """f1 = kappa h^3 f'(h) with f = (b/h)^n - (b/h)^m (eq. GeneralDisPreForm with the
    power-law part of eq. DisjPressNLC); derivatives checked by central differences of
    the defining expressions, f'(1) = 0.017 for b = 0.1, n = 3, m = 2."""
    M = model(orc)
    f = lambda h: (0.1 / h) ** 3 - (0.1 / h) ** 2
    for h in (0.15, 0.5, 1.0, 1.7, 3.0):
        f0, f0p, f1, f1p = orc.coeffs(M, h)
        d = 1e-5 * h
        fp = (f(h + d) - f(h - d)) / (2 * d)
        assert f0 == pytest.approx(h ** 3, rel=1e-15)
        scale = 10.0 * h ** 3 * (3 * 0.1 ** 3 / h ** 4 + 2 * 0.1 ** 2 / h ** 3)
        assert f1 == pytest.approx(10.0 * h ** 3 * fp, abs=1e-8 * scale)
        g = lambda x: orc.coeffs(M, x)[2]
        assert f1p == pytest.approx((g(h + d) - g(h - d)) / (2 * d), abs=1e-7 * scale / h)
        assert f0p == pytest.approx(3 * h * h, rel=1e-15)
    assert orc.coeffs(M, 1.0)[2] == pytest.approx(10.0 * 0.017, rel=1e-14)


# ---------------------------------------------------------------- P1 flat film
def test_flat_film_is_bit_exact(orc):
    """A flat film has zero flux through every face (each face flux is a difference of
    equal numbers), so D = 0 and a time step leaves it unchanged bit for bit."""
    M = model(orc)
    u = np.full((9, 13), 0.8)
    assert np.all(orc.flux_divergence(M, u, 0.37) == 0.0)
    u1, res = orc.step(M, orc.Scheme(tol=1e-12), u, 0.37, 0.1)
    assert res.status == orc.OK
    assert np.array_equal(u1, u)


# ---------------------------------------------------------------- P2 mass
def _naive_sum(x):
    s = 0.0
    for v in x:
        s += v
    return s


def test_mass_sum_and_minimum_match_exact_definitions(orc):
    """The mass diagnostic (Sec. "Conservation of Mass": the mean of the cell values) is a
    compensated sum. It is pinned to math.fsum (the correctly rounded exact sum) and the
    minimum to numpy's, on ordinary films and on inputs built so that a plain running sum
    fails: large cancelling pairs, and many addends below half an ulp of the running total.
    A sum that dropped its compensation, skipped cells or returned a constant fails here."""
    rng = np.random.default_rng(17)
    # ordinary films (row-major, ragged shapes): every cell counts, the minimum anywhere
    for ny, nx in ((1, 1), (3, 7), (64, 65), (257, 131)):
        u = 1.0 + 0.01 * rng.uniform(-1.0, 1.0, (ny, nx))
        s, mn = orc.mass(u)
        exact = math.fsum(u.ravel())
        assert abs(s - exact) <= 2 * np.spacing(exact), (ny, nx, s, exact)
        assert mn == np.min(u)
        # the minimum at the last and at the first cell
        v = u.copy()
        v[-1, -1] = 0.25
        assert orc.mass(v)[1] == 0.25
        v[0, 0] = 0.125
        assert orc.mass(v)[1] == 0.125
        assert abs(orc.mass(v)[0] - math.fsum(v.ravel())) <= 2 * np.spacing(math.fsum(v.ravel()))
    # cancellation: +-1e16 pairs interleaved with small values; a plain sum loses every small
    # value that meets a big partial sum
    small = rng.uniform(0.5, 1.5, 3000)
    x = np.empty(4 * small.size)
    x[0::4] = 1e16
    x[1::4] = small
    x[2::4] = -1e16
    x[3::4] = small[::-1]
    u = x.reshape(60, 200)
    s, _ = orc.mass(u)
    exact = math.fsum(x)
    assert abs(s - exact) <= 2 * np.spacing(exact), (s, exact)
    assert abs(_naive_sum(x) - exact) > 1e3 * np.spacing(exact)  # the case does defeat a plain sum
    # 10^6 addends below half an ulp of a unit base: a plain sum stays at 1
    y = np.full(1_000_000, 1e-17)
    y[0] = 1.0
    s, mn = orc.mass(y.reshape(1000, 1000))
    exact = math.fsum(y)
    assert exact == 1.0 + 1e-11 or abs(exact - (1.0 + 1e-11)) <= np.spacing(1.0)
    assert abs(s - exact) <= np.spacing(exact), (s, exact)
    assert _naive_sum(y) == 1.0  # a plain running sum loses every addend
    assert mn == 1e-17
    # negative values and a sum that cancels to (almost) nothing
    z = rng.normal(size=(40, 50))
    z -= z.mean()
    s, mn = orc.mass(z)
    assert abs(s - math.fsum(z.ravel())) <= 4 * np.finfo(float).eps * np.abs(z).sum() * 1e-3
    assert mn == np.min(z)


def test_mass_conserved_every_iteration(orc):
    """Zero boundary flux makes sum(D) telescope to zero (Sec. "Conservation of Mass"),
    and the flux-form J_x, J_y have zero column sums, so every Newton iterate keeps the
    total of u^n up to rounding."""
    M = model(orc)
    u0 = synth.noise_film(21, 17, seed=11, amp=0.05)
    ds = 0.6
    D = orc.flux_divergence(M, u0, ds)
    assert abs(D.sum()) <= 1e-13 * np.abs(D).sum()
    s0, _ = orc.mass(u0)
    uk = u0
    for _ in range(6):
        uk, e, r = orc.adi_iteration(M, u0, uk, ds, 0.1)
        s, _ = orc.mass(uk)
        assert abs(s - s0) <= 1e-13 * s0
    for theta in (0.5, 1.0):
        u1, res = orc.step(M, orc.Scheme(theta=theta, tol=1e-12), u0, ds, 0.2)
        assert res.status == orc.OK
        assert abs(orc.mass(u1)[0] - s0) <= 1e-13 * s0


# ---------------------------------------------------------------- P4 linear model / DCT
def _dct_step(u, ds, dt, c0, c1, theta):
    ny, nx = u.shape
    kx = np.arange(nx)
    ky = np.arange(ny)
    mu = (4 / ds ** 2) * (np.sin(np.pi * kx / (2 * nx))[None, :] ** 2
                          + np.sin(np.pi * ky / (2 * ny))[:, None] ** 2)
    lam = c0 * mu ** 2 - c1 * mu  # eigenvalue of D on the cell-centred Neumann cosine basis
    uh = scipy.fft.dctn(u, type=2, norm="ortho")
    uh = uh * (1 - (1 - theta) * dt * lam) / (1 + theta * dt * lam)
    return scipy.fft.idctn(uh, type=2, norm="ortho")


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("c0,c1", [(1.0, 1.0), (0.5, -0.3)])
def test_linear_model_matches_dct_closed_form(orc, theta, c0, c1):
    """For f0 = c0, f1 = c1 (Sec. "Thin Film Models", first model) D is the linear
    operator c0 L^2 + c1 L with L the cell-centred Neumann Laplacian, diagonal in the
    DCT-II basis; one step of the theta scheme is then a closed form."""
    M = orc.Model.linear(c0, c1)
    u = synth.noise_film(16, 11, seed=5, amp=0.3)
    ds, dt = 0.9, 0.05
    u1, res = orc.step(M, orc.Scheme(theta=theta, tol=1e-14), u, ds, dt)
    assert res.status == orc.OK
    ref = _dct_step(u, ds, dt, c0, c1, theta)
    assert np.max(np.abs(u1 - ref)) <= 1e-12


# ---------------------------------------------------------------- manufactured solution
def _continuous_D(orc, M, u, K2, grad2, h0):
    """div[f0 grad lap u + f1 grad u] for u = h0 + a cos(kx x) cos(ky y):
    lap u = -K2 (u - h0), grad lap u = -K2 grad u, lap^2 u = K2^2 (u - h0)."""
    out = np.empty_like(u)
    for idx, h in np.ndenumerate(u):
        f0, f0p, f1, f1p = orc.coeffs(M, h)
        out[idx] = (-K2 * f0p * grad2[idx] + f0 * K2 ** 2 * (h - h0)
                    + f1p * grad2[idx] - K2 * f1 * (h - h0))
    return out


def test_flux_operator_second_order_against_continuous(orc):
    """Second-order consistency of D (eq. GovEqnCell2, Sec. "Flux Discretization"):
    for a smooth Neumann-compatible field the discrete operator approaches
    div[f0 grad lap u + f1 grad u] at rate ds^2, boundary cells included."""
    M = model(orc)
    h0, a = 1.0, 0.25
    Lx = 20.0
    kx = 2 * np.pi / Lx
    errs = []
    for n in (24, 48, 96):
        nx, ny = n, int(round(0.7 * n))
        ds = Lx / nx
        Ly = ny * ds
        ky = 3 * np.pi / Ly
        x = (np.arange(nx) + 0.5) * ds
        y = (np.arange(ny) + 0.5) * ds
        X, Y = np.meshgrid(x, y)
        u = h0 + a * np.cos(kx * X) * np.cos(ky * Y)
        grad2 = a ** 2 * (kx ** 2 * np.sin(kx * X) ** 2 * np.cos(ky * Y) ** 2
                          + ky ** 2 * np.cos(kx * X) ** 2 * np.sin(ky * Y) ** 2)
        Dc = _continuous_D(orc, M, u, kx ** 2 + ky ** 2, grad2, h0)
        Dd = orc.flux_divergence(M, u, ds)
        errs.append(np.max(np.abs(Dd - Dc)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(1.85 < p < 2.15 for p in orders), (errs, orders)


# ---------------------------------------------------------------- P3 LSA
@pytest.mark.parametrize("axis", ["x", "y"])
def test_discrete_linear_growth_rate(orc, axis):
    """A small cosine eigenmode of the cell-centred Neumann grid grows per backward-Euler
    step by exactly 1 / (1 + dt lambda), lambda = f0(h0) mu^2 - f1(h0) mu,
    mu = (4/ds^2) sin^2(pi k / 2n) (linearisation of D about a flat film, Sec. "Linear
    Stability Analysis"), up to O(amp^2) nonlinear corrections."""
    M = model(orc)
    cfg = synth.CONFIGS["small128"]
    n, k, dt, amp = 128, 8, 0.1, 1e-4
    ds = cfg.ds
    if axis == "x":
        u = synth.cosine_film(n, 4, k, 0, amp=amp)
    else:
        u = synth.cosine_film(4, n, 0, k, amp=amp)
    mode = (u - 1.0) / amp
    f0, _, f1, _ = orc.coeffs(M, 1.0)
    mu = 4 / ds ** 2 * math.sin(math.pi * k / (2 * n)) ** 2
    g_exact = 1.0 / (1.0 + dt * (f0 * mu ** 2 - f1 * mu))
    a_prev = amp
    for _ in range(5):
        u, res = orc.step(M, orc.Scheme(tol=1e-13), u, ds, dt)
        assert res.status == orc.OK
        a = np.sum((u - 1.0) * mode) / np.sum(mode * mode)
        assert a / a_prev == pytest.approx(g_exact, rel=1e-9)
        a_prev = a


def test_small128_mode_amplification_closed_forms(orc):
    """The 128^2, L = 4 lambda_m configuration with the k = 8 mode (q = q_m): the discrete
    100-step backward-Euler factor from the rate formula equals 1.0749513, next to the
    continuous exp(omega_m T) = 1.0749240 with omega_m = h0^3 q_m^2 (kappa f'(h0) - q_m^2)."""
    M = model(orc)
    cfg = synth.CONFIGS["small128"]
    f0, _, f1, _ = orc.coeffs(M, 1.0)
    mu = 4 / cfg.ds ** 2 * math.sin(math.pi * 8 / 256) ** 2
    disc = (1.0 / (1.0 + 0.1 * (f0 * mu ** 2 - f1 * mu))) ** 100
    qm = synth.q_m(10.0)
    cont = math.exp(qm ** 2 * (10 * 0.017 - qm ** 2) * 10.0)
    assert disc == pytest.approx(1.0749513, abs=5e-7)
    assert cont == pytest.approx(1.0749240, abs=5e-7)
    assert abs(disc - cont) < 5e-4


# ---------------------------------------------------------------- P6 banded solver
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 9, 40])
@pytest.mark.parametrize("dominant", [True, False])
def test_band_solver_matches_scipy_and_dense(orc, n, dominant):
    rng = np.random.default_rng(100 + n + 7 * dominant)
    band = rng.standard_normal((5, n))
    if dominant:
        band[2] = 6.0 + rng.random(n)
    for p in range(n):  # zero the entries that fall outside the matrix
        for o in range(5):
            if not 0 <= p + o - 2 < n:
                band[o, p] = 0.0
    rhs = rng.standard_normal(n)
    x = orc.band_solve(band, rhs)
    A = orc.band_to_dense(band)
    assert np.allclose(A @ x, rhs, rtol=0, atol=1e-12 * max(1.0, np.abs(rhs).max()) * np.linalg.cond(A))
    ab = np.zeros((5, n))  # scipy's (l, u) = (2, 2) storage: ab[2 + i - j, j] = A[i, j]
    for i in range(n):
        for j in range(max(0, i - 2), min(n, i + 3)):
            ab[2 + i - j, j] = A[i, j]
    xs = scipy.linalg.solve_banded((2, 2), ab, rhs)
    assert np.max(np.abs(x - xs)) <= 1e-12 * np.linalg.cond(A) * max(1.0, np.abs(xs).max())


def test_band_transpose(orc):
    rng = np.random.default_rng(3)
    n = 11
    band = rng.standard_normal((5, n))
    for p in range(n):
        for o in range(5):
            if not 0 <= p + o - 2 < n:
                band[o, p] = 0.0
    assert np.array_equal(orc.band_to_dense(orc.band_transpose(band)), orc.band_to_dense(band).T)


# ---------------------------------------------------------------- P7 Jacobians
def _fd_dir(orc, M, u, d, ds, eps=1e-6):
    return (orc.flux_divergence(M, u + eps * d, ds) - orc.flux_divergence(M, u - eps * d, ds)) / (2 * eps)


def test_full_jacobian_matches_finite_differences(orc):
    M = model(orc)
    u = synth.noise_film(9, 7, seed=21, amp=0.2)
    ds = 0.8
    rng = np.random.default_rng(2)
    v = rng.standard_normal(u.shape)
    Jv = orc.jacobian_apply(M, u, v, ds)
    fd = _fd_dir(orc, M, u, v, ds)
    assert np.max(np.abs(Jv - fd)) <= 1e-7 * np.max(np.abs(Jv))
    w = rng.standard_normal(u.shape)
    lhs = np.sum(w * Jv)
    rhs = np.sum(orc.jacobian_apply_t(M, u, w, ds) * v)
    assert lhs == pytest.approx(rhs, rel=1e-12)


def _apply_split(orc, M, u, d, ds):
    """(J_x + J_y) d assembled from the oracle's line bands (I + c J) with c = 1."""
    ny, nx = u.shape
    out = np.zeros_like(u)
    for j in range(ny):
        A = orc.band_to_dense(orc.bands_x(M, u, ds, 1.0, j))
        out[j, :] += A @ d[j, :] - d[j, :]
    for i in range(nx):
        A = orc.band_to_dense(orc.bands_y(M, u, ds, 1.0, i))
        out[:, i] += A @ d[:, i] - d[:, i]
    return out


@pytest.mark.parametrize("along", ["x", "y"])
def test_split_jacobians_exact_on_one_directional_perturbations(orc, along):
    """J_x, J_y hold the pure x and y terms of J_D (eq. DirectionSplit). For a
    perturbation that is constant in y (or in x) every mixed term of J_D vanishes, so
    (J_x + J_y) d must equal the directional derivative of D."""
    M = model(orc)
    u = synth.noise_film(10, 8, seed=4, amp=0.2)
    ds = 0.7
    rng = np.random.default_rng(9)
    if along == "x":
        d = np.tile(rng.standard_normal(u.shape[1]), (u.shape[0], 1))
    else:
        d = np.tile(rng.standard_normal(u.shape[0])[:, None], (1, u.shape[1]))
    fd = _fd_dir(orc, M, u, d, ds)
    got = _apply_split(orc, M, u, d, ds)
    assert np.max(np.abs(got - fd)) <= 2e-7 * np.max(np.abs(fd))


def test_split_jacobian_on_flat_film_is_exact_for_any_x_perturbation(orc):
    """About a flat film Lam = Gam = 0, so J_y d = 0 for d that varies along x only and
    J_x d equals the x-directional derivative of D."""
    M = model(orc)
    u = np.full((5, 12), 1.3)
    ds = 0.5
    rng = np.random.default_rng(1)
    d = np.tile(rng.standard_normal(12), (5, 1))
    got = _apply_split(orc, M, u, d, ds)
    fd = _fd_dir(orc, M, u, d, ds)
    assert np.max(np.abs(got - fd)) <= 1e-7 * np.max(np.abs(fd))


# ---------------------------------------------------------------- P5 dense brute force
def _dense_newton(orc, M, un, ds, dt, theta):
    u = un.copy()
    N = u.size
    for _ in range(30):
        G = orc.residual(M, un, u, ds, dt, theta)
        J = np.empty((N, N))
        for q in range(N):
            e = np.zeros(N)
            e[q] = 1.0
            J[:, q] = orc.jacobian_apply(M, u, e.reshape(u.shape), ds).ravel()
        J = np.eye(N) + theta * dt * J
        du = np.linalg.solve(J, -G.ravel()).reshape(u.shape)
        u = u + du
        if np.max(np.abs(du)) < 1e-15:
            break
    return u


@pytest.mark.parametrize("shape", [(4, 4), (5, 7), (8, 6)])
@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_adi_newton_reaches_dense_newton_root(orc, shape, theta):
    """The ADI-preconditioned iteration (eqs. JacobianSystem1-3) converges to the same
    root of G as full Newton with the dense exact Jacobian."""
    M = model(orc)
    un = synth.noise_film(shape[1], shape[0], seed=31, amp=0.05)
    ds, dt = 0.7, 0.1
    ref = _dense_newton(orc, M, un, ds, dt, theta)
    u1, res = orc.step(M, orc.Scheme(theta=theta, tol=1e-14), un, ds, dt)
    assert res.status == orc.OK
    assert np.max(np.abs(u1 - ref)) <= 1e-12


# ---------------------------------------------------------------- P8 convergence orders
def _run(orc, M, u, ds, dt, T, theta):
    steps = int(round(T / dt))
    for _ in range(steps):
        u, res = orc.step(M, orc.Scheme(theta=theta, tol=1e-14), u, ds, dt)
        assert res.status == orc.OK
    return u


@pytest.mark.parametrize("theta,order", [(0.5, 2.0), (1.0, 1.0)])
def test_time_convergence_order(orc, theta, order):
    """Sec. "Convergence": the trapezoidal rule (theta = 1/2) is second order in dt;
    backward Euler (theta = 1) is first order. Self-convergence under dt halving."""
    M = model(orc)
    n = 16
    ds = 0.5
    u0 = synth.cosine_film(n, n, 1, 1, amp=0.2) + 0.05 * synth.cosine_film(n, n, 2, 0, h0=0, amp=1)
    T = 0.8
    sols = [_run(orc, M, u0, ds, T / s, T, theta) for s in (4, 8, 16, 32)]
    errs = [np.max(np.abs(sols[i] - sols[i + 1])) for i in range(3)]
    p = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(q - order) < 0.15 for q in p), (errs, p)


def test_space_convergence_order(orc):
    """Sec. "Convergence": tripling the grid nests the cell centres; the scheme is
    second order in ds."""
    M = model(orc)
    L = 12.0
    T, dt = 0.2, 0.05
    sols = []
    for n in (12, 36, 108):
        ds = L / n
        x = (np.arange(n) + 0.5) * ds
        X, Y = np.meshgrid(x, x)
        u0 = 1.0 + 0.2 * np.cos(2 * np.pi * X / L) * np.cos(np.pi * Y / L)
        sols.append(_run(orc, M, u0, ds, dt, T, 1.0))
    c1 = sols[1][1::3, 1::3]
    c2 = sols[2][4::9, 4::9]
    e1 = np.max(np.abs(sols[0] - c1))
    e2 = np.max(np.abs(sols[0] - c2))
    # e(12) ~ C ds^2 (1 - 1/81), e(12 vs 36) ~ C ds^2 (1 - 1/9): ratio 0.9 for order 2
    f1 = np.max(np.abs(c1 - c2))
    p = math.log(e1 / f1) / math.log(3.0)
    assert 1.8 < p < 2.2, (e1, e2, f1, p)


# ---------------------------------------------------------------- P9 symmetry
def test_step_commutes_with_reflection_and_transpose(orc):
    M = model(orc)
    u = synth.noise_film(12, 12, seed=8, amp=0.05)
    ds, dt = 0.6, 0.2
    S = orc.Scheme(tol=1e-14)
    u1, _ = orc.step(M, S, u, ds, dt)
    uf, _ = orc.step(M, S, u[:, ::-1], ds, dt)
    assert np.max(np.abs(uf[:, ::-1] - u1)) <= 1e-13
    ut, _ = orc.step(M, S, u.T, ds, dt)
    assert np.max(np.abs(ut.T - u1)) <= 1e-12


# ---------------------------------------------------------------- failure paths
def test_failure_paths(orc):
    M = model(orc)
    u = synth.noise_film(8, 8, seed=1)
    bad = u.copy()
    bad[3, 3] = -0.1
    out, res = orc.step(M, orc.Scheme(), bad, 0.7, 0.1)
    assert res.status == orc.ENONPOS and np.array_equal(out, bad)
    nanu = u.copy()
    nanu[0, 0] = np.nan
    assert orc.step(M, orc.Scheme(), nanu, 0.7, 0.1)[1].status == orc.ENONPOS
    out, res = orc.step(M, orc.Scheme(max_newton=1, tol=1e-14), u, 0.7, 0.1)
    assert res.status == orc.ENOCONV and np.array_equal(out, u)
    out, res = orc.step(M, orc.Scheme(max_newton=2, tol=1e-14, adaptive=1, dt_min=1e-3), u, 0.7, 0.1)
    assert res.status == orc.ENOCONV and res.rejections >= 6 and np.array_equal(out, u)
    out, res = orc.step(M, orc.Scheme(max_newton=10, tol=1e-10, adaptive=1), u, 0.7, 0.4)
    assert res.status == orc.OK


def test_adaptive_growth_and_cap(orc):
    """Fig. FlowChartTime: dt grows after grow_after consecutive successes, capped at
    dt_max."""
    M = model(orc)
    u = synth.cosine_film(8, 8, 1, 1, amp=1e-3)
    S = orc.Scheme(max_newton=50, tol=1e-10, adaptive=1, grow_after=2, dt_grow=2.0, dt_max=0.3)
    dt, succ = 0.1, 0
    seen = []
    for _ in range(6):
        u, res = orc.step(M, S, u, 0.7, dt, succ)
        assert res.status == orc.OK
        seen.append(res.dt_used)
        dt, succ = res.dt_next, res.successes
    assert seen == [0.1, 0.1, 0.2, 0.2, 0.3, 0.3]
