"""ctypes binding of libthinfilm (include/thinfilm.h): argument marshalling only.

Every step of the ADI-Newton path runs in the HIP library; PyTorch supplies device
memory (contiguous float64 CUDA tensors) and the stream. If the built library is
missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libthinfilm.so")

TF_OK, TF_EINVAL, TF_ENOMEM, TF_EDEVICE, TF_ENOCONV, TF_ENONPOS, TF_ESTATE = range(7)
STATUS_NAMES = {0: "TF_OK", 1: "TF_EINVAL", 2: "TF_ENOMEM", 3: "TF_EDEVICE", 4: "TF_ENOCONV",
                5: "TF_ENONPOS", 6: "TF_ESTATE"}


class Scheme(C.Structure):
    """tf_scheme: theta scheme and the dt control of Fig. FlowChartTime."""
    _fields_ = [("theta", C.c_double), ("tol", C.c_double), ("dt_min", C.c_double),
                ("dt_max", C.c_double), ("dt_shrink", C.c_double), ("dt_grow", C.c_double),
                ("max_newton", C.c_int), ("grow_after", C.c_int), ("adaptive", C.c_int)]


class StepInfo(C.Structure):
    _fields_ = [("t", C.c_double), ("dt_used", C.c_double), ("e_final", C.c_double),
                ("r_final", C.c_double), ("mass", C.c_double), ("hmin", C.c_double),
                ("newton_iters", C.c_int), ("rejections", C.c_int), ("status", C.c_int),
                ("total_iters", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# x-sweep line-solver variants (include/thinfilm.h, TF_XSWEEP_*)
XSWEEP = {"auto": -1, "partitioned": 0, "row": 1}
XSWEEP_NAMES = {0: "partitioned", 1: "row"}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; "
                               f"g.build()'` (or python paper_1806_10550_amd/build.py) first")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        D = C.c_double
        L.tf_last_error.restype = C.c_char_p
        L.tf_profile_names.restype = C.c_char_p
        L.tf_create.argtypes = [C.c_int, C.c_int, D, P, C.POINTER(P)]
        L.tf_destroy.argtypes = [P]
        L.tf_set_model.argtypes = [P, D, D, D, D]
        L.tf_set_model_linear.argtypes = [P, D, D]
        L.tf_get_clock.argtypes = [P, C.POINTER(D), C.POINTER(C.c_int)]
        L.tf_set_clock.argtypes = [P, D, C.c_int]
        L.tf_radial_spectrum.argtypes = [P, C.c_int, D, D, D, D, P, P, P, P, C.c_int, P]
        L.tf_spectrum_maxima.argtypes = [P, P, C.c_int, D, C.c_int, P, P, P, C.c_int, P]
        L.tf_model_coeffs.argtypes = [P, P, C.c_int, P]
        L.tf_set_model_nlc.argtypes = [P, D, D, D, D, D, D]
        L.tf_ensemble_set_model_linear.argtypes = [P, D, D]
        L.tf_ensemble_set_model_nlc.argtypes = [P, D, D, D, D, D, D]
        L.tf_ensemble_set_model_polymer.argtypes = [P, D, D, D, D, D]
        L.tf_set_model_polymer.argtypes = [P, D, D, D, D, D]
        L.tf_set_scheme.argtypes = [P, C.POINTER(Scheme)]
        L.tf_get_scheme.argtypes = [P, C.POINTER(Scheme)]
        L.tf_set_diagnostics.argtypes = [P, C.c_int]
        L.tf_set_xsweep.argtypes = [P, C.c_int]
        L.tf_get_xsweep.argtypes = [P]
        L.tf_get_xsweep.restype = C.c_int
        L.tf_bind_state.argtypes = [P, P]
        L.tf_step.argtypes = [P, C.POINTER(D), C.POINTER(StepInfo)]
        L.tf_advance.argtypes = [P, C.c_int, C.POINTER(D), P]
        L.tf_mass.argtypes = [P, C.POINTER(D), C.POINTER(D)]
        L.tf_newton_iteration.argtypes = [P, P, P, P, D, C.POINTER(D), C.POINTER(D), C.POINTER(C.c_int)]
        L.tf_flux_divergence.argtypes = [P, P, P]
        L.tf_profile.argtypes = [P, C.c_int]
        L.tf_profile_read.argtypes = [P, C.POINTER(D), C.POINTER(C.c_long), C.c_int]
        L.tf_profile_read.restype = C.c_int
        IP = C.POINTER(C.c_int)
        DP = C.POINTER(D)
        L.tf_ensemble_create.argtypes = [C.c_int, IP, IP, DP, DP, D, D, D, P, C.POINTER(P)]
        L.tf_ensemble_destroy.argtypes = [P]
        L.tf_ensemble_set_scheme.argtypes = [P, C.POINTER(Scheme)]
        L.tf_ensemble_size.argtypes = [P]
        L.tf_ensemble_size.restype = C.c_longlong
        L.tf_ensemble_offsets.argtypes = [P, C.POINTER(C.c_longlong)]
        L.tf_ensemble_bind.argtypes = [P, P]
        L.tf_ensemble_step.argtypes = [P, C.c_int, DP, IP, IP]
        L.tf_ensemble_film_info.argtypes = [P, C.c_int, C.POINTER(StepInfo)]
        L.tf_adjoint_step.argtypes = [P, P, P, D, P, DP, D, C.c_int, IP]
        L.tf_jacobian_apply_t.argtypes = [P, P, P, P]
        L.tf_adjoint_steps.argtypes = [P, C.c_int, P, D, P, DP, D, C.c_int, IP]
        L.tf_advance_keep.argtypes = [P, C.c_int, C.POINTER(D), P, P]
        L.tf_penta_solve.argtypes = [C.c_int, C.c_int, P, P, P, C.c_int, C.c_int, P]
        L.tf_penta_solve_noalloc.argtypes = [C.c_int, C.c_int, P, P, P, C.c_int, C.c_int, P]
        L.tf_autotune.argtypes = [C.c_int, C.c_int, C.c_int, C.c_char_p]
        L.tf_autotune_load.argtypes = [C.c_char_p]
        L.tf_autotune_choice.argtypes = [C.c_int, C.c_int, C.c_int]
        L.tf_autotune_choice.restype = C.c_int
        L.tf_autotune_xsweep.argtypes = [C.c_int, C.c_int, C.c_char_p]
        L.tf_xsweep_choice.argtypes = [C.c_int, C.c_int]
        L.tf_xsweep_choice.restype = C.c_int
        L.tf_ensemble_set_xsweep.argtypes = [P, C.c_int]
        L.tf_ensemble_xsweep.argtypes = [P, C.c_int]
        L.tf_ensemble_xsweep.restype = C.c_int
        _lib = L
    return _lib


def _check(st):
    if st != TF_OK:
        raise TFError(st, lib().tf_last_error().decode())


def _ptr(t):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64 \
            or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def default_scheme(**kw) -> Scheme:
    s = Scheme(1.0, 1e-10, 1e-6, 1.0, 0.5, 1.1, 5000, 5, 0)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


@dataclass
class StepResult:
    dt_next: float
    info: dict


class Grid:
    """One film of nx x ny cells of side ds; see include/thinfilm.h."""

    def __init__(self, nx: int, ny: int, ds: float, stream=None):
        load_shipped_tuning()  # the x-sweep variant is fixed at creation from the tuning table
        self._h = C.c_void_p()
        _check(lib().tf_create(int(nx), int(ny), float(ds), _stream_ptr(stream), C.byref(self._h)))
        self.nx, self.ny, self.ds = nx, ny, ds
        self._state = None

    def close(self):
        if self._h:
            lib().tf_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_model(self, kappa=10.0, b=0.1, n=3, m=2):
        _check(lib().tf_set_model(self._h, float(kappa), float(b), float(n), float(m)))
        return self

    def set_model_linear(self, c0=1.0, c1=1.0):
        """Linear test model f0 = c0, f1 = c1 (Sec. "Thin Film Models")."""
        _check(lib().tf_set_model_linear(self._h, float(c0), float(c1)))
        return self

    def model_coeffs(self, h, out):
        """out[k] = (f0, f0', f1, f1') at h[k]; h: (n,) and out: (n, 4) float64 CUDA tensors."""
        if out.numel() != 4 * h.numel():
            raise ValueError("out must hold 4 values per thickness")
        _check(lib().tf_model_coeffs(self._h, _ptr(h), int(h.numel()), _ptr(out)))
        return out

    def set_model_nlc(self, C=0.0857, K=36.0, N=1.67, beta=1.0, w=0.05, b=0.01):
        """NLC model (eqs. DisjPressNLC, mh_model); defaults are eq. NLC_paras."""
        _check(lib().tf_set_model_nlc(self._h, *(float(x) for x in (C, K, N, beta, w, b))))
        return self

    def set_model_polymer(self, C=0.00581, Cst=1.181, Aox=41.25, Asi=-243.75, d=191.0):
        """Polymer model (eq. DisjPressPolymer); defaults are eq. Polymer_scales."""
        _check(lib().tf_set_model_polymer(self._h, *(float(x) for x in (C, Cst, Aox, Asi, d))))
        return self

    def set_scheme(self, **kw):
        s = default_scheme(**kw)
        _check(lib().tf_set_scheme(self._h, C.byref(s)))
        return self

    def scheme(self) -> Scheme:
        s = Scheme()
        _check(lib().tf_get_scheme(self._h, C.byref(s)))
        return s

    def set_diagnostics(self, mass_every_step: bool):
        _check(lib().tf_set_diagnostics(self._h, int(bool(mass_every_step))))

    def set_xsweep(self, variant):
        """x-sweep line solver: "partitioned", "row" or "auto" (tf_set_xsweep)."""
        code = XSWEEP[variant] if isinstance(variant, str) else int(variant)
        _check(lib().tf_set_xsweep(self._h, code))

    def xsweep(self) -> str:
        return XSWEEP_NAMES[lib().tf_get_xsweep(self._h)]

    def bind(self, h):
        """Bind a contiguous (ny, nx) float64 CUDA tensor as the state (borrowed)."""
        if tuple(h.shape) != (self.ny, self.nx):
            raise ValueError(f"state must have shape ({self.ny}, {self.nx})")
        _check(lib().tf_bind_state(self._h, _ptr(h)))
        self._state = h
        return self

    def step(self, dt: float) -> StepResult:
        d = C.c_double(dt)
        info = StepInfo()
        _check(lib().tf_step(self._h, C.byref(d), C.byref(info)))
        return StepResult(d.value, info.as_dict())

    def clock(self):
        """(t, successes) of the bound state (tf_get_clock)."""
        t, s = C.c_double(), C.c_int()
        _check(lib().tf_get_clock(self._h, C.byref(t), C.byref(s)))
        return t.value, s.value

    def set_clock(self, t: float, successes: int):
        _check(lib().tf_set_clock(self._h, float(t), int(successes)))
        return self

    def checkpoint(self, dt_next: float) -> dict:
        """What a later run needs to continue this one exactly: a host copy of the state,
        its clock and the dt to try next (a dict of tensors and numbers, torch.save-able)."""
        t, s = self.clock()
        return {"h": self._state.detach().cpu().clone(), "t": t, "successes": s, "dt": float(dt_next)}

    def restore(self, ckpt: dict, h):
        """Copy a checkpoint's state into h (a (ny, nx) float64 CUDA tensor), bind it, set
        the clock; returns the dt to try next."""
        h.copy_(ckpt["h"])
        self.bind(h)
        self.set_clock(ckpt["t"], ckpt["successes"])
        return ckpt["dt"]

    def advance(self, nsteps: int, dt: float, log: bool = False):
        d = C.c_double(dt)
        arr = (StepInfo * max(nsteps, 1))() if log else None
        st = lib().tf_advance(self._h, int(nsteps), C.byref(d),
                              C.cast(arr, C.c_void_p) if log else None)
        infos = [arr[i].as_dict() for i in range(nsteps)] if log else None
        _check(st)
        return d.value, infos

    def try_advance(self, nsteps: int, dt: float):
        """Like advance but returns (status, dt, log) instead of raising."""
        d = C.c_double(dt)
        arr = (StepInfo * max(nsteps, 1))()
        st = lib().tf_advance(self._h, int(nsteps), C.byref(d), C.cast(arr, C.c_void_p))
        return st, d.value, [arr[i].as_dict() for i in range(nsteps)]

    def try_step(self, dt: float):
        d = C.c_double(dt)
        info = StepInfo()
        st = lib().tf_step(self._h, C.byref(d), C.byref(info))
        return st, d.value, info.as_dict()

    def mass(self):
        m, hm = C.c_double(), C.c_double()
        _check(lib().tf_mass(self._h, C.byref(m), C.byref(hm)))
        return m.value, hm.value

    def _fields(self, *ts):
        """The C calls take bare device pointers to (ny, nx) fields: check the shapes here,
        before any device access."""
        for t in ts:
            if tuple(t.shape) != (self.ny, self.nx):
                raise ValueError(f"fields must have shape ({self.ny}, {self.nx}), got {tuple(t.shape)}")

    def newton_iteration(self, un, uk, out, dt: float):
        self._fields(un, uk, out)
        e, r, f = C.c_double(), C.c_double(), C.c_int()
        _check(lib().tf_newton_iteration(self._h, _ptr(un), _ptr(uk), _ptr(out), float(dt),
                                         C.byref(e), C.byref(r), C.byref(f)))
        return e.value, r.value, f.value

    def flux_divergence(self, u, out):
        self._fields(u, out)
        _check(lib().tf_flux_divergence(self._h, _ptr(u), _ptr(out)))
        return out

    def adjoint_step(self, h_n, h_np1, dt: float, lam, tol: float = 1e-13, max_iter: int = 2000,
                     dkappa: bool = True):
        """lam (device, in/out): lambda^{n+1} -> lambda^n. Returns (dL/dkappa contribution,
        Richardson iterations); the contribution is None with dkappa=False (required for the
        NLC and polymer models, which have no kappa)."""
        self._fields(h_n, h_np1, lam)
        g = C.c_double(0.0)
        it = C.c_int(0)
        _check(lib().tf_adjoint_step(self._h, _ptr(h_n), _ptr(h_np1), float(dt), _ptr(lam),
                                     C.byref(g) if dkappa else None, float(tol), int(max_iter), C.byref(it)))
        return (g.value if dkappa else None), it.value

    def advance_keep(self, nsteps: int, dt: float, states):
        """advance(nsteps, dt) keeping every accepted state: states[s] (a (>= nsteps, ny, nx)
        float64 CUDA tensor) receives the state after step s + 1 (tf_advance_keep)."""
        _ptr(states)
        if states.dim() != 3 or states.shape[0] < nsteps or tuple(states.shape[1:]) != (self.ny, self.nx):
            raise ValueError(f"states must be a (>= {nsteps}, {self.ny}, {self.nx}) tensor")
        ptrs = (C.c_void_p * max(nsteps, 1))(*[states[s].data_ptr() for s in range(nsteps)])
        d = C.c_double(dt)
        _check(lib().tf_advance_keep(self._h, int(nsteps), C.byref(d), ptrs, None))
        return d.value

    def adjoint_steps(self, states, dt: float, lam, tol: float = 1e-13, max_iter: int = 2000, dkappa: bool = True):
        """Adjoint steps of a stretch: states (a contiguous (nsteps + 1, ny, nx) tensor, oldest
        first); lam goes from lambda^{nsteps} to lambda^0 (tf_adjoint_steps). Returns (summed
        dL/dkappa contribution or None, Richardson iterations)."""
        _ptr(states)
        self._fields(lam)
        if states.dim() != 3 or states.shape[0] < 1 or tuple(states.shape[1:]) != (self.ny, self.nx):
            raise ValueError(f"states must be a (nsteps + 1, {self.ny}, {self.nx}) tensor")
        n = states.shape[0] - 1
        ptrs = (C.c_void_p * max(n + 1, 1))(*[states[s].data_ptr() for s in range(n + 1)])
        g = C.c_double(0.0)
        it = C.c_int(0)
        _check(lib().tf_adjoint_steps(self._h, int(n), ptrs, float(dt), _ptr(lam), C.byref(g) if dkappa else None,
                                      float(tol), int(max_iter), C.byref(it)))
        return (g.value if dkappa else None), it.value

    def jacobian_apply_t(self, u, mu, out):
        self._fields(u, mu, out)
        _check(lib().tf_jacobian_apply_t(self._h, _ptr(u), _ptr(mu), _ptr(out)))
        return out

    def profile(self, on: bool):
        _check(lib().tf_profile(self._h, int(bool(on))))

    def profile_read(self):
        names = lib().tf_profile_names().decode().split(",")
        n = len(names)
        ms = (C.c_double * n)()
        cnt = (C.c_long * n)()
        lib().tf_profile_read(self._h, ms, cnt, n)
        return {names[i]: (ms[i], cnt[i]) for i in range(n)}


class Ensemble:
    """Films of different sizes / kappa / ds packed in one buffer and stepped in lockstep
    (include/thinfilm.h, tf_ensemble_*); theta scheme with theta in [0.5, 1]."""

    def __init__(self, nx, ny, ds, kappa, b=0.1, n=3, m=2, stream=None):
        load_shipped_tuning()  # per-film x-sweep variants, as single grids take them
        k = len(nx)
        self.nfilms = k
        self._h = C.c_void_p()
        ia = (C.c_int * k)(*[int(v) for v in nx])
        ja = (C.c_int * k)(*[int(v) for v in ny])
        da = (C.c_double * k)(*[float(v) for v in ds])
        ka = (C.c_double * k)(*[float(v) for v in kappa])
        _check(lib().tf_ensemble_create(k, ia, ja, da, ka, float(b), float(n), float(m), _stream_ptr(stream),
                                        C.byref(self._h)))
        self.nx, self.ny = list(nx), list(ny)
        offs = (C.c_longlong * k)()
        _check(lib().tf_ensemble_offsets(self._h, offs))
        self.offsets = [int(v) for v in offs]
        self.size = int(lib().tf_ensemble_size(self._h))
        self._state = None

    def set_xsweep(self, variant):
        """x-sweep line solver of every film: "auto" (each as alone), "row" or "partitioned"."""
        code = XSWEEP[variant] if isinstance(variant, str) else int(variant)
        _check(lib().tf_ensemble_set_xsweep(self._h, code))

    def xsweep(self, film: int) -> str:
        return XSWEEP_NAMES[lib().tf_ensemble_xsweep(self._h, int(film))]

    def set_model_linear(self, c0=1.0, c1=1.0):
        _check(lib().tf_ensemble_set_model_linear(self._h, float(c0), float(c1)))
        return self

    def set_model_nlc(self, C=0.0857, K=36.0, N=1.67, beta=1.0, w=0.05, b=0.01):
        """Every film gets the NLC model (eqs. DisjPressNLC, mh_model; defaults eq. NLC_paras)."""
        _check(lib().tf_ensemble_set_model_nlc(self._h, *(float(x) for x in (C, K, N, beta, w, b))))
        return self

    def set_model_polymer(self, C=0.00581, Cst=1.181, Aox=41.25, Asi=-243.75, d=191.0):
        """Every film gets the polymer model (eq. DisjPressPolymer; defaults eq. Polymer_scales)."""
        _check(lib().tf_ensemble_set_model_polymer(self._h, *(float(x) for x in (C, Cst, Aox, Asi, d))))
        return self

    def close(self):
        if self._h:
            lib().tf_ensemble_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_scheme(self, **kw):
        s = default_scheme(**kw)
        _check(lib().tf_ensemble_set_scheme(self._h, C.byref(s)))
        return self

    def view(self, packed, f):
        """(ny, nx) view of film f inside the packed tensor."""
        o = self.offsets[f]
        return packed[o:o + self.nx[f] * self.ny[f]].view(self.ny[f], self.nx[f])

    def bind(self, packed):
        if packed.numel() != self.size:
            raise ValueError(f"packed buffer must hold {self.size} doubles")
        _check(lib().tf_ensemble_bind(self._h, _ptr(packed)))
        self._state = packed
        return self

    def step(self, nsteps, dt):
        """Advance every film nsteps; dt: float or per-film list. Returns (status, dts,
        statuses, iterations)."""
        k = self.nfilms
        dts = (C.c_double * k)(*([float(dt)] * k if isinstance(dt, (int, float)) else [float(v) for v in dt]))
        sts = (C.c_int * k)()
        its = (C.c_int * k)()
        st = lib().tf_ensemble_step(self._h, int(nsteps), dts, sts, its)
        return st, list(dts), list(sts), list(its)

    def film_info(self, f):
        info = StepInfo()
        _check(lib().tf_ensemble_film_info(self._h, int(f), C.byref(info)))
        return info.as_dict()


VARIANTS = {"auto": -1, "partitioned": 0, "thomas": 1, "pcr": 2, "line": 3}
VARIANT_NAMES = ["partitioned", "thomas", "pcr", "line"]


def penta_solve(bands, rhs, x, transposed=False, variant="auto", stream=None):
    """Batched pentadiagonal solve on stored bands (tf_penta_solve). bands: (5, n, nlines)
    float64 CUDA tensor, rhs and x: (n, nlines)."""
    n, nl = rhs.shape
    if tuple(bands.shape) != (5, n, nl) or tuple(x.shape) != (n, nl):
        raise ValueError("bands must be (5, n, nlines) and rhs, x (n, nlines)")
    _check(lib().tf_penta_solve(int(nl), int(n), _ptr(bands), _ptr(rhs), _ptr(x), int(bool(transposed)),
                                VARIANTS[variant], _stream_ptr(stream)))
    return x


def penta_solve_noalloc(bands, rhs, x, transposed=False, variant="auto", stream=None):
    """tf_penta_solve_noalloc: the same solve with the library's static scratch array (no
    device allocation, no synchronisation: the work is enqueued on the stream)."""
    n, nl = rhs.shape
    if tuple(bands.shape) != (5, n, nl) or tuple(x.shape) != (n, nl):
        raise ValueError("bands must be (5, n, nlines) and rhs, x (n, nlines)")
    _check(lib().tf_penta_solve_noalloc(int(nl), int(n), _ptr(bands), _ptr(rhs), _ptr(x), int(bool(transposed)),
                                        VARIANTS[variant], _stream_ptr(stream)))
    return x


def radial_spectrum(h, ds: float, h0: float, sigma: float = 1.0, qmax: float = None, stream=None):
    """Steps 1-4 of the radial Fourier transform (tf_radial_spectrum) of a square (n, n)
    float64 CUDA film: returns numpy arrays (q, mean, count) over the groups of equal
    |k|^2 with 0 < q <= qmax (default: the whole spectrum)."""
    import numpy as np
    n = int(h.shape[0])
    if tuple(h.shape) != (n, n):
        raise ValueError("the film must be square")
    L = n * ds
    if qmax is None:
        qmax = 2 * math.pi * math.sqrt(2.0) * (n // 2) / L
    cap = int(min((qmax * L / (2 * math.pi)) ** 2 * (1 + 1e-12), 2.0 * (n // 2) ** 2)) + 2
    cap = min(cap, (1 << 26) + 2)
    q = np.empty(cap)
    v = np.empty(cap)
    c = np.empty(cap, dtype=np.int32)
    npts = C.c_int(0)
    _check(lib().tf_radial_spectrum(_ptr(h), n, float(ds), float(h0), float(sigma), float(qmax), _stream_ptr(stream),
                                    q.ctypes.data, v.ctypes.data, c.ctypes.data, cap, C.byref(npts)))
    k = npts.value
    return q[:k].copy(), v[:k].copy(), c[:k].copy()


def spectrum_release() -> None:
    """Free the FFT plans and scratch kept by radial_spectrum (tf_spectrum_release)."""
    _check(lib().tf_spectrum_release())


def spectrum_maxima(q, s, qmax: float, nfine: int = 400, capacity: int = 64):
    """Steps 5-7 (tf_spectrum_maxima): returns (x, smoothed curve, [(q, value) of each
    local maximum])."""
    import numpy as np
    q = np.ascontiguousarray(q, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    curve = np.empty(nfine)
    pq = np.empty(capacity)
    ps = np.empty(capacity)
    npk = C.c_int(0)
    _check(lib().tf_spectrum_maxima(q.ctypes.data, s.ctypes.data, len(q), float(qmax), int(nfine), curve.ctypes.data,
                                    pq.ctypes.data, ps.ctypes.data, int(capacity), C.byref(npk)))
    x = np.linspace(0.0, qmax, nfine)
    return x, curve, [(float(pq[i]), float(ps[i])) for i in range(npk.value)]


def autotune(length: int, batch: int, cache_path: str | None = None, transposed: bool = False) -> str:
    _check(lib().tf_autotune(int(length), int(batch), int(bool(transposed)),
                             cache_path.encode() if cache_path else None))
    return VARIANT_NAMES[lib().tf_autotune_choice(int(length), int(batch), int(bool(transposed)))]


def autotune_xsweep(length: int, batch: int, cache_path: str | None = None) -> str:
    """Time the two forward x-sweep variants on a film of `batch` rows of `length` cells
    (tf_autotune_xsweep); returns the one now chosen for that shape."""
    _check(lib().tf_autotune_xsweep(int(length), int(batch), cache_path.encode() if cache_path else None))
    return xsweep_choice(length, batch)


def xsweep_choice(nx: int, ny: int) -> str:
    """x-sweep variant a film of nx x ny cells takes at creation (tf_xsweep_choice)."""
    return XSWEEP_NAMES[lib().tf_xsweep_choice(int(nx), int(ny))]


def autotune_load(cache_path: str) -> None:
    _check(lib().tf_autotune_load(cache_path.encode()))


_shipped_loaded = False


def load_shipped_tuning() -> bool:
    """Load the solver tuning files shipped beside this module (autotune_<arch>.jsonl,
    written by paper_1806_10550_amd.tune) once per process; entries of other GPU
    architectures are ignored. Returns True if entries for this GPU were loaded."""
    global _shipped_loaded
    if _shipped_loaded:
        return True
    import glob
    for f in sorted(glob.glob(os.path.join(HERE, "autotune_*.jsonl"))):
        if lib().tf_autotune_load(f.encode()) == TF_OK:
            _shipped_loaded = True
    return _shipped_loaded


def autotune_choice(length: int, batch: int, transposed: bool = False) -> str:
    return VARIANT_NAMES[lib().tf_autotune_choice(int(length), int(batch), int(bool(transposed)))]
