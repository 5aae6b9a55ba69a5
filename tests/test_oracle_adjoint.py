"""Pins of the oracle's discrete adjoint (implicit-function-theorem adjoint of one
converged step of G(u^{n+1}; u^n, kappa) = 0, with G from eq. TrapRule in theta form).

Checked against a dense transposed solve built from the forward Jacobian (not from
the transposed code path), and against central finite differences of a loss on
h(T) with respect to the initial perturbation and kappa.
"""
import numpy as np
import pytest

from paper_1806_10550_amd import synth

PL = dict(kappa=10.0, b=0.1, n=3.0, m=2.0)


def _dense_J(orc, M, u, ds):
    N = u.size
    J = np.empty((N, N))
    for q in range(N):
        e = np.zeros(N)
        e[q] = 1.0
        J[:, q] = orc.jacobian_apply(M, u, e.reshape(u.shape), ds).ravel()
    return J


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_adjoint_step_matches_dense_transposed_solve(orc, theta):
    M = orc.Model(**PL)
    un = synth.noise_film(6, 5, seed=3, amp=0.05)
    ds, dt = 0.8, 0.1
    unp1, res = orc.step(M, orc.Scheme(theta=theta, tol=1e-14), un, ds, dt)
    assert res.status == orc.OK
    lam = np.random.default_rng(1).standard_normal(un.shape)
    lam_n, gk, it = orc.adjoint_step(M, un, unp1, lam, ds, dt, theta, tol=1e-15)
    N = un.size
    JG = np.eye(N) + theta * dt * _dense_J(orc, M, unp1, ds)
    mu = np.linalg.solve(JG.T, lam.ravel())
    ref = mu - (1 - theta) * dt * _dense_J(orc, M, un, ds).T @ mu
    assert np.max(np.abs(lam_n.ravel() - ref)) <= 1e-12 * np.max(np.abs(ref))
    Dk = theta * orc.flux_divergence_dkappa(M, unp1, ds) + (1 - theta) * orc.flux_divergence_dkappa(M, un, ds)
    assert gk == pytest.approx(-dt * np.dot(mu, Dk.ravel()), rel=1e-12)


def test_dkappa_operator_is_derivative_of_D(orc):
    u = synth.noise_film(7, 6, seed=2, amp=0.2)
    ds = 0.9
    eps = 1e-4
    Dp = orc.flux_divergence(orc.Model(**{**PL, "kappa": 10 + eps}), u, ds)
    Dm = orc.flux_divergence(orc.Model(**{**PL, "kappa": 10 - eps}), u, ds)
    fd = (Dp - Dm) / (2 * eps)
    got = orc.flux_divergence_dkappa(orc.Model(**PL), u, ds)
    assert np.max(np.abs(got - fd)) <= 1e-8 * np.max(np.abs(fd))


def _loss_and_traj(orc, kappa, h0, target, ds, dt, steps, theta):
    M = orc.Model(**{**PL, "kappa": kappa})
    traj = [h0]
    u = h0
    for _ in range(steps):
        u, res = orc.step(M, orc.Scheme(theta=theta, tol=1e-14), u, ds, dt)
        assert res.status == orc.OK
        traj.append(u)
    return 0.5 * np.sum((u - target) ** 2), traj


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_adjoint_gradient_matches_finite_differences(orc, theta):
    """Gradient of L = 0.5 ||h(T) - h_target||^2 with respect to the initial
    perturbation p0 (h(0) = h0 + p0) and kappa, through 6 steps on a 10 x 8 grid."""
    nx, ny, ds, dt, steps = 10, 8, 0.9, 0.1, 6
    base = synth.noise_film(nx, ny, seed=4, amp=0.01)
    target = synth.noise_film(nx, ny, seed=5, amp=0.01)
    kappa = 10.0
    L0, traj = _loss_and_traj(orc, kappa, base, target, ds, dt, steps, theta)
    M = orc.Model(**{**PL, "kappa": kappa})
    lam = traj[-1] - target
    gk = 0.0
    for n in range(steps - 1, -1, -1):
        lam, g, _ = orc.adjoint_step(M, traj[n], traj[n + 1], lam, ds, dt, theta, tol=1e-15)
        gk += g
    d = np.random.default_rng(7).standard_normal(base.shape)
    eps = 1e-5
    Lp, _ = _loss_and_traj(orc, kappa, base + eps * d, target, ds, dt, steps, theta)
    Lm, _ = _loss_and_traj(orc, kappa, base - eps * d, target, ds, dt, steps, theta)
    fd = (Lp - Lm) / (2 * eps)
    assert np.sum(lam * d) == pytest.approx(fd, rel=1e-6)
    ek = 1e-5
    Lp, _ = _loss_and_traj(orc, kappa + ek, base, target, ds, dt, steps, theta)
    Lm, _ = _loss_and_traj(orc, kappa - ek, base, target, ds, dt, steps, theta)
    assert gk == pytest.approx((Lp - Lm) / (2 * ek), rel=1e-6)
