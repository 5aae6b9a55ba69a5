"""ctypes binding of the C oracle (tf_oracle.c) with NumPy conveniences.

TEST INFRASTRUCTURE ONLY: imported by tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``; never by the product path.

Arrays are float64, C-contiguous, shape (ny, nx) with u[j, i] (i along x).
Each wrapper names the passage of Lam, Cummings & Kondic (arXiv:1806.10550) that
the C function follows; see tf_oracle.c for the formulas.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OK, EINVAL, ENOMEM, ENOCONV, ENONPOS, ESINGULAR = 0, 1, 2, 4, 5, 7
POWERLAW, LINEAR, NLC, POLYMER = 0, 1, 2, 3


class _Model(C.Structure):
    _fields_ = [("kind", C.c_int), ("kappa", C.c_double), ("b", C.c_double), ("n", C.c_double),
                ("m", C.c_double), ("c0", C.c_double), ("c1", C.c_double), ("cap", C.c_double),
                ("K", C.c_double), ("N", C.c_double), ("beta", C.c_double), ("w", C.c_double),
                ("Cst", C.c_double), ("Aox", C.c_double), ("Asi", C.c_double), ("d", C.c_double)]


class _Scheme(C.Structure):
    _fields_ = [("theta", C.c_double), ("tol", C.c_double), ("dt_min", C.c_double),
                ("dt_max", C.c_double), ("dt_shrink", C.c_double), ("dt_grow", C.c_double),
                ("max_newton", C.c_int), ("grow_after", C.c_int), ("adaptive", C.c_int)]


class _StepInfo(C.Structure):
    _fields_ = [("t", C.c_double), ("dt_used", C.c_double), ("e_final", C.c_double),
                ("r_final", C.c_double), ("newton_iters", C.c_int), ("rejections", C.c_int),
                ("status", C.c_int), ("total_iters", C.c_int)]


@dataclass
class Model:
    """Power-law thin-film model f0 = h^3, f1 = kappa h^3 f'(h), f = (b/h)^n - (b/h)^m
    (eq. GeneralDisPreForm with the power-law term of eq. DisjPressNLC), or the linear
    test model f0 = c0, f1 = c1 (Sec. "Thin Film Models")."""
    kappa: float = 10.0
    b: float = 0.1
    n: float = 3.0
    m: float = 2.0
    kind: int = POWERLAW
    c0: float = 0.0
    c1: float = 0.0
    cap: float = 1.0
    K: float = 0.0
    N: float = 0.0
    beta: float = 0.0
    w: float = 0.0
    Cst: float = 0.0
    Aox: float = 0.0
    Asi: float = 0.0
    d: float = 0.0

    @staticmethod
    def linear(c0: float, c1: float) -> "Model":
        return Model(kind=LINEAR, c0=c0, c1=c1)

    @staticmethod
    def nlc(cap=0.0857, K=36.0, N=1.67, beta=1.0, w=0.05, b=0.01) -> "Model":
        """NLC model: f0 = C h^3, f1 = h^3 Pi'(h), Pi of eqs. DisjPressNLC, mh_model; defaults
        are the parameters of eq. NLC_paras."""
        return Model(kind=NLC, cap=cap, K=K, N=N, beta=beta, w=w, b=b)

    @staticmethod
    def polymer(cap=0.00581, Cst=1.181, Aox=41.25, Asi=-243.75, d=191.0) -> "Model":
        """Polymer model: f0 = C h^3, f1 = h^3 Pi'(h), Pi = -psi' of eq. DisjPressPolymer;
        defaults are the parameters of eq. Polymer_scales."""
        return Model(kind=POLYMER, cap=cap, Cst=Cst, Aox=Aox, Asi=Asi, d=d)

    def _c(self) -> _Model:
        return _Model(self.kind, self.kappa, self.b, self.n, self.m, self.c0, self.c1, self.cap, self.K,
                      self.N, self.beta, self.w, self.Cst, self.Aox, self.Asi, self.d)


@dataclass
class Scheme:
    """Time-step control of Fig. FlowChartTime; theta = 1 backward Euler, 1/2 eq. TrapRule."""
    theta: float = 1.0
    tol: float = 1e-10
    dt_min: float = 1e-6
    dt_max: float = 1.0
    dt_shrink: float = 0.5
    dt_grow: float = 1.1
    max_newton: int = 5000
    grow_after: int = 5
    adaptive: int = 0

    def _c(self) -> _Scheme:
        return _Scheme(self.theta, self.tol, self.dt_min, self.dt_max, self.dt_shrink,
                       self.dt_grow, self.max_newton, self.grow_after, self.adaptive)


_lib = None
_DP = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    """Load liboracle.so (build it first with oracle/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        MP = C.POINTER(_Model)
        L.or_set_threads.argtypes = [C.c_int]
        L.or_get_threads.restype = C.c_int
        L.or_coeffs.argtypes = [MP, C.c_double] + [C.POINTER(C.c_double)] * 4
        L.or_disjoining.argtypes = [MP, C.c_double] + [C.POINTER(C.c_double)] * 3
        L.or_flux_divergence.argtypes = [MP, C.c_int, C.c_int, C.c_double, _DP, _DP]
        L.or_flux_divergence_dkappa.argtypes = [MP, C.c_int, C.c_int, C.c_double, _DP, _DP]
        L.or_residual.argtypes = [MP, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                  _DP, _DP, _DP]
        L.or_bands_x.argtypes = [MP, C.c_int, C.c_int, C.c_double, _DP, C.c_double, C.c_int, _DP]
        L.or_bands_y.argtypes = [MP, C.c_int, C.c_int, C.c_double, _DP, C.c_double, C.c_int, _DP]
        L.or_band_solve.argtypes = [C.c_int, _DP, _DP, _DP]
        L.or_band_transpose.argtypes = [C.c_int, _DP, _DP]
        L.or_adi_iteration.argtypes = [MP, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                       _DP, C.c_void_p, _DP, _DP, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double)]
        L.or_step.argtypes = [MP, C.POINTER(_Scheme), C.c_int, C.c_int, C.c_double, _DP,
                              C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(_StepInfo)]
        L.or_jacobian_apply.argtypes = [MP, C.c_int, C.c_int, C.c_double, _DP, _DP, _DP]
        L.or_jacobian_apply_t.argtypes = [MP, C.c_int, C.c_int, C.c_double, _DP, _DP, _DP]
        L.or_adjoint_step.argtypes = [MP, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                      _DP, _DP, _DP, _DP, C.POINTER(C.c_double), C.c_double,
                                      C.c_int, C.POINTER(C.c_int)]
        L.or_mass.argtypes = [C.c_int, C.c_int, _DP, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _arr(u):
    return np.ascontiguousarray(u, dtype=np.float64)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def disjoining(model: Model, h: float):
    """(Pi, Pi', Pi'') at one thickness h for the NLC and polymer models."""
    out = [C.c_double() for _ in range(3)]
    m = model._c()
    lib().or_disjoining(C.byref(m), float(h), *[C.byref(o) for o in out])
    return tuple(o.value for o in out)


def coeffs(model: Model, h: float):
    """(f0, f0', f1, f1') at one thickness h (eq. GeneralDisPreForm)."""
    out = [C.c_double() for _ in range(4)]
    m = model._c()
    lib().or_coeffs(C.byref(m), float(h), *[C.byref(o) for o in out])
    return tuple(o.value for o in out)


def flux_divergence(model: Model, u, ds: float):
    """D(u), the flux-difference operator (eq. FluxDiffOper, eq. GovEqnCell2)."""
    u = _arr(u)
    ny, nx = u.shape
    D = np.empty_like(u)
    m = model._c()
    st = lib().or_flux_divergence(C.byref(m), nx, ny, float(ds), u, D)
    if st != OK:
        raise RuntimeError(f"or_flux_divergence status {st}")
    return D


def flux_divergence_dkappa(model: Model, u, ds: float):
    """dD/dkappa for the power-law model."""
    u = _arr(u)
    ny, nx = u.shape
    D = np.empty_like(u)
    m = model._c()
    st = lib().or_flux_divergence_dkappa(C.byref(m), nx, ny, float(ds), u, D)
    if st != OK:
        raise RuntimeError(f"or_flux_divergence_dkappa status {st}")
    return D


def residual(model: Model, un, u, ds: float, dt: float, theta: float = 1.0):
    """G(u) = u - u^n + dt [theta D(u) + (1 - theta) D(u^n)] (eq. TrapRule, theta form)."""
    un, u = _arr(un), _arr(u)
    ny, nx = u.shape
    G = np.empty_like(u)
    m = model._c()
    st = lib().or_residual(C.byref(m), nx, ny, float(ds), float(dt), float(theta), un, u, G)
    if st != OK:
        raise RuntimeError(f"or_residual status {st}")
    return G


def bands_x(model: Model, u, ds: float, c: float, j: int):
    """5 x nx bands of I + c J_x for grid row j (eq. JacobianSystem2)."""
    u = _arr(u)
    ny, nx = u.shape
    band = np.empty((5, nx))
    m = model._c()
    lib().or_bands_x(C.byref(m), nx, ny, float(ds), u, float(c), int(j), band)
    return band


def bands_y(model: Model, u, ds: float, c: float, i: int):
    """5 x ny bands of I + c J_y for grid column i (eq. JacobianSystem1)."""
    u = _arr(u)
    ny, nx = u.shape
    band = np.empty((5, ny))
    m = model._c()
    lib().or_bands_y(C.byref(m), nx, ny, float(ds), u, float(c), int(i), band)
    return band


def band_solve(band, rhs):
    """Solve a 5-band system by band Gaussian elimination with partial pivoting."""
    band = _arr(band)
    rhs = _arr(rhs)
    n = rhs.shape[0]
    x = np.empty(n)
    st = lib().or_band_solve(n, band, rhs, x)
    if st != OK:
        raise RuntimeError(f"or_band_solve status {st}")
    return x


def band_transpose(band):
    band = _arr(band)
    n = band.shape[1]
    bt = np.empty_like(band)
    lib().or_band_transpose(n, band, bt)
    return bt


def band_to_dense(band):
    n = band.shape[1]
    A = np.zeros((n, n))
    for p in range(n):
        for o in range(5):
            col = p + o - 2
            if 0 <= col < n:
                A[p, col] = band[o, p]
    return A


def adi_iteration(model: Model, un, uk, ds: float, dt: float, theta: float = 1.0, Dn=None):
    """One ADI-Newton iteration (eqs. JacobianSystem1-3): returns (u_{k+1}, e, max|G|)."""
    un, uk = _arr(un), _arr(uk)
    ny, nx = uk.shape
    out = np.empty_like(uk)
    e, r = C.c_double(), C.c_double()
    m = model._c()
    if theta < 1.0 and Dn is None:
        Dn = flux_divergence(model, un, ds)
    dn_ptr = _arr(Dn).ctypes.data_as(C.c_void_p) if Dn is not None else None
    keep = Dn  # noqa: F841  (keeps the buffer alive during the call)
    st = lib().or_adi_iteration(C.byref(m), nx, ny, float(ds), float(dt), float(theta), un,
                                dn_ptr, uk, out, C.byref(e), C.byref(r))
    if st != OK:
        raise RuntimeError(f"or_adi_iteration status {st}")
    return out, e.value, r.value


@dataclass
class StepResult:
    status: int
    dt_used: float
    dt_next: float
    e_final: float
    r_final: float
    newton_iters: int
    rejections: int
    total_iters: int
    successes: int


def step(model: Model, scheme: Scheme, u, ds: float, dt: float, successes: int = 0):
    """One accepted time step with the control of Fig. FlowChartTime. Returns (u_new, result).
    On failure u_new equals u."""
    u = _arr(u).copy()
    ny, nx = u.shape
    dtc = C.c_double(dt)
    sc = C.c_int(successes)
    info = _StepInfo()
    m, s = model._c(), scheme._c()
    st = lib().or_step(C.byref(m), C.byref(s), nx, ny, float(ds), u, C.byref(dtc), C.byref(sc),
                       C.byref(info))
    return u, StepResult(st, info.dt_used, dtc.value, info.e_final, info.r_final,
                         info.newton_iters, info.rejections, info.total_iters, sc.value)


def jacobian_apply(model: Model, u, v, ds: float):
    """J_D(u) v with the full analytic Jacobian of D."""
    u, v = _arr(u), _arr(v)
    ny, nx = u.shape
    out = np.empty_like(u)
    m = model._c()
    lib().or_jacobian_apply(C.byref(m), nx, ny, float(ds), u, v, out)
    return out


def jacobian_apply_t(model: Model, u, mu, ds: float):
    """J_D(u)^T mu."""
    u, mu = _arr(u), _arr(mu)
    ny, nx = u.shape
    out = np.empty_like(u)
    m = model._c()
    lib().or_jacobian_apply_t(C.byref(m), nx, ny, float(ds), u, mu, out)
    return out


def adjoint_step(model: Model, u_n, u_np1, lam_np1, ds: float, dt: float, theta: float = 1.0,
                 tol: float = 1e-13, max_iter: int = 10000):
    """Adjoint of one converged step: returns (lambda^n, dL/dkappa contribution, iterations)."""
    u_n, u_np1, lam_np1 = _arr(u_n), _arr(u_np1), _arr(lam_np1)
    ny, nx = u_n.shape
    lam_n = np.empty_like(u_n)
    g = C.c_double(0.0)
    it = C.c_int(0)
    m = model._c()
    st = lib().or_adjoint_step(C.byref(m), nx, ny, float(ds), float(dt), float(theta), u_n, u_np1,
                               lam_np1, lam_n, C.byref(g), float(tol), int(max_iter), C.byref(it))
    if st != OK:
        raise RuntimeError(f"or_adjoint_step status {st}")
    return lam_n, g.value, it.value


def mass(u):
    """Compensated sum and minimum of the cell values (Sec. "Conservation of Mass")."""
    u = _arr(u)
    ny, nx = u.shape
    s, mn = C.c_double(), C.c_double()
    lib().or_mass(nx, ny, u, C.byref(s), C.byref(mn))
    return s.value, mn.value
