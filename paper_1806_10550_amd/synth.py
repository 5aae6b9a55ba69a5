"""Seeded synthetic inputs (initial films and ensemble descriptions).

This module holds only random draws and geometry; none of the time-stepping
arithmetic. Both the GPU tests/benchmark and the CPU oracle tests take their
inputs from here, so the two sides always see identical arrays.

Geometry: a square domain of side L = P * lambda_m split into n x n cells,
ds = L / n. lambda_m = 2 pi / q_m is the most unstable wavelength of a flat film
of thickness h0 (linear stability, Sec. "Linear Stability Analysis"): for
h_t + div[f0 grad lap h + f1 grad h] = 0 a mode exp(i q x) grows at
sigma(q) = q^2 (f1(h0) - f0(h0) q^2), largest at q_m^2 = f1(h0) / (2 f0(h0)).
With f0 = h^3 and f1 = kappa h^3 f'(h), f = (b/h)^n - (b/h)^m this is
q_m^2 = kappa f'(h0) / 2.

Noise: NumPy ``default_rng(seed)`` (PCG64), ``uniform(-1, 1, (ny, nx))``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def fprime(h: float, b: float, n: float, m: float) -> float:
    """f'(h) for f(h) = (b/h)^n - (b/h)^m."""
    return -n * b ** n / h ** (n + 1) + m * b ** m / h ** (m + 1)


def q_m(kappa: float, b: float = 0.1, n: float = 3, m: float = 2, h0: float = 1.0) -> float:
    """Most unstable wavenumber of a flat film (geometry helper for the configs)."""
    return math.sqrt(kappa * fprime(h0, b, n, m) / 2.0)


def lambda_m(kappa: float, b: float = 0.1, n: float = 3, m: float = 2, h0: float = 1.0) -> float:
    return 2.0 * math.pi / q_m(kappa, b, n, m, h0)


def omega_m(kappa: float, b: float = 0.1, n: float = 3, m: float = 2, h0: float = 1.0) -> float:
    """Largest linear growth rate h0^3 q_m^4 (geometry/reporting helper)."""
    return h0 ** 3 * q_m(kappa, b, n, m, h0) ** 4


def noise_film(nx: int, ny: int, seed: int, h0: float = 1.0, amp: float = 0.01) -> np.ndarray:
    """h0 + amp * U[-1, 1] iid per cell, shape (ny, nx), float64."""
    rng = np.random.default_rng(seed)
    return h0 + amp * rng.uniform(-1.0, 1.0, (ny, nx))


def cosine_film(nx: int, ny: int, kx: int, ky: int, h0: float = 1.0, amp: float = 1e-4) -> np.ndarray:
    """h0 (1 + amp cos(pi kx (i+1/2)/nx) cos(pi ky (j+1/2)/ny)): a cosine mode sampled at
    the cell centres of a Neumann box (kx or ky may be 0)."""
    x = np.cos(np.pi * kx * (np.arange(nx) + 0.5) / nx)
    y = np.cos(np.pi * ky * (np.arange(ny) + 0.5) / ny)
    return h0 * (1.0 + amp * np.outer(y, x))


def wave_film(n: int, P: float, q: float, h0: float = 1.0, ex: float = 0.1, ey: float = 0.1):
    """Initial condition of eq. IC_LinearWave: h0 (1 + ex cos(q x) + ey cos(q y)) at the cell
    centres of n x n cells on the square [0, P lam]^2, lam = 2 pi / q. Returns (h, ds).
    The printed argument pi x / lam is read as q x, so that q is the wavenumber of the
    perturbation; both forms have zero slope at the walls for integer P."""
    L = P * 2.0 * math.pi / q
    ds = L / n
    c = np.cos(q * (np.arange(n) + 0.5) * ds)
    return h0 * (1.0 + ex * c[None, :] + ey * c[:, None]), ds


def perlin_noise(n: int, seed: int, alpha: float = None) -> np.ndarray:
    """Pseudo-Perlin noise zeta of eq. PerlinNoise on n x n cells: the real part of the
    inverse DFT of |k|^-alpha exp(2 pi i a(k)), a ~ U[-1, 1] iid per wavevector (k = 0
    dropped), scaled so that max |zeta| = 1. alpha defaults to 200 / n."""
    if alpha is None:
        alpha = 200.0 / n
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, (n, n))
    k = np.fft.fftfreq(n, d=1.0 / n)
    m = k[None, :] ** 2 + k[:, None] ** 2
    amp = np.zeros((n, n))
    amp[m > 0] = m[m > 0] ** (-alpha / 2.0)
    z = np.real(np.fft.ifft2(amp * np.exp(2j * np.pi * a)))
    return z / np.max(np.abs(z))


def localized_bumps(n: int, ds: float, lam_m: float, seed: int, count: int = 4, spacing: float = 8.0) -> np.ndarray:
    """eta of eq. 3DRandomLocalTerm: a count x count array of Gaussians
    exp(-((x - chi_i)^2 + (y - xi_j)^2) / (0.04 lam_m^2)) centred at
    chi_i = (spacing i - spacing/2 + (spacing/2) a_i) lam_m, xi_j likewise with b_j,
    a_i, b_j ~ U[-1, 1] (the paper's spacing is 8; the sign between the two squares is read
    as +, a radially symmetric bump)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, count)
    b = rng.uniform(-1.0, 1.0, count)
    idx = np.arange(1, count + 1)
    chi = (spacing * idx - spacing / 2 + spacing / 2 * a) * lam_m
    xi = (spacing * idx - spacing / 2 + spacing / 2 * b) * lam_m
    x = (np.arange(n) + 0.5) * ds
    gx = np.exp(-((x[None, :] - chi[:, None]) ** 2) / (0.04 * lam_m ** 2)).sum(axis=0)
    gy = np.exp(-((x[None, :] - xi[:, None]) ** 2) / (0.04 * lam_m ** 2)).sum(axis=0)
    return np.outer(gy, gx)


def random_film(n: int, P: float, lam_m: float, h0: float, seed: int, eps: float = 0.01):
    """eq. 3D_Random_IC: h0 (1 + eps |zeta|) on [0, P lam_m]^2. Returns (h, ds)."""
    ds = P * lam_m / n
    return h0 * (1.0 + eps * np.abs(perlin_noise(n, seed))), ds


def mixed_film(n: int, P: float, lam_m: float, h0: float, seed: int, eps: float = 0.01):
    """eq. 3DLocalAndRandom: h0 (1 + eps |zeta| + 10 eps eta). Returns (h, ds)."""
    ds = P * lam_m / n
    z = np.abs(perlin_noise(n, seed))
    eta = localized_bumps(n, ds, lam_m, seed + 1)
    return h0 * (1.0 + eps * z + 10.0 * eps * eta), ds


def gaussian_depression(h: np.ndarray, ds: float, depth: float, width: float) -> np.ndarray:
    """h - depth * exp(-r^2 / width^2) about the domain centre (r measured between
    cell centres)."""
    ny, nx = h.shape
    x = (np.arange(nx) + 0.5) * ds
    y = (np.arange(ny) + 0.5) * ds
    xc, yc = nx * ds / 2.0, ny * ds / 2.0
    r2 = (x[None, :] - xc) ** 2 + (y[:, None] - yc) ** 2
    return h - depth * np.exp(-r2 / width ** 2)


@dataclass
class FilmConfig:
    name: str
    n: int                 # cells per side
    periods: float         # domain side in units of lambda_m
    kappa: float = 10.0
    b: float = 0.1
    nexp: float = 3.0
    mexp: float = 2.0
    h0: float = 1.0
    amp: float = 0.01
    seed: int = 0
    dt: float = 0.1
    steps: int = 100
    tol: float = 1e-10
    adaptive: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def L(self) -> float:
        return self.periods * lambda_m(self.kappa, self.b, self.nexp, self.mexp, self.h0)

    @property
    def ds(self) -> float:
        return self.L / self.n

    def film(self) -> np.ndarray:
        h = noise_film(self.n, self.n, self.seed, self.h0, self.amp)
        if self.extra.get("gaussian"):
            lm = lambda_m(self.kappa, self.b, self.nexp, self.mexp, self.h0)
            h = gaussian_depression(h, self.ds, self.extra.get("depth", 0.3), lm / 4.0)
        return h


# The five workloads: small parity case, 2048^2 spinodal/nucleation, 8192^2 throughput,
# 256-film ensemble, 512^2 adjoint.
CONFIGS = {
    "small128": FilmConfig("small128", 128, 4.0, seed=0, dt=0.1, steps=100),
    "spinodal2048": FilmConfig("spinodal2048", 2048, 64.0, seed=1, dt=0.1, steps=2000, adaptive=1),
    "nucleation2048": FilmConfig("nucleation2048", 2048, 64.0, seed=1, dt=0.1, steps=2000,
                                 adaptive=1, extra={"gaussian": True, "depth": 0.3}),
    "large8192": FilmConfig("large8192", 8192, 256.0, seed=2, dt=0.2, steps=500),
    "adjoint512": FilmConfig("adjoint512", 512, 16.0, seed=4, dt=0.1, steps=400,
                             extra={"target_seed": 5, "checkpoint_every": 20}),
}


@dataclass
class EnsembleFilm:
    n: int
    kappa: float
    seed: int
    ds: float


def ensemble_films(nfilms: int = 256, seed: int = 3,
                   sizes=(256, 384, 512, 768, 1024), periods: float = 8.0,
                   kappa_range=(5.0, 20.0), b: float = 0.1, h0: float = 1.0):
    """Draw (size, kappa, per-film seed) for an ensemble of square films, each of side
    periods * lambda_m(kappa)."""
    rng = np.random.default_rng(seed)
    films = []
    for _ in range(nfilms):
        n = int(rng.choice(np.asarray(sizes)))
        kappa = float(rng.uniform(*kappa_range))
        fseed = int(rng.integers(0, 2 ** 31 - 1))
        ds = periods * lambda_m(kappa, b, 3, 2, h0) / n
        films.append(EnsembleFilm(n, kappa, fseed, ds))
    return films
