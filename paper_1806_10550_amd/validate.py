"""The paper's validation suite (Sec. "Validation") on the GPU path, for its three models:
the linear test model (f0 = f1 = 1, H0 = 1), NLC (H0 = 0.5) and polymer (H0 = 3.9).

    python -m paper_1806_10550_amd.validate [--quick] [--out FILE]

  temporal   Sec. "Convergence": I0 = 256, P = 6, q = q_m, dt_i = 2^-i dt0 with
             dt0 = 1e-3 / omega_m, run to t = dt0; L2 (root-mean-square) error against the
             finest level; Newton tolerance 1e-14 ("machine") or max(dt^2, 1e-14) ("scaled").
  spatial    Sec. "Convergence": I_k = 36 * 3^k (cell centres of level k are cell centres of
             every finer level), one step of dt0 = 1e-8 / omega_m; error against the finest
             level at the shared centres; tolerance 1e-14 or max(ds^2, 1e-14).
  mass       Sec. "Conservation of Mass": 1000 steps of the run's dt, relative change of the
             mean thickness every 100 steps; the spatial family (I = 36 * 3^i, dt0 = 1e-8 /
             omega_m, tolerance max(ds^2, 1e-14)) and the temporal family (I = 1024,
             dt = 2^-i 1e-3 / omega_m, 1000 * 2^i steps sampled every 100 * 2^i,
             tolerance max(dt^2, 1e-14)).
  lsa        Sec. "Comparison to LSA": P = 1 (the domain is one wavelength 2 pi / q),
             I = J = 32, perturbation along x or y, adaptive steps (at most 10 Newton
             iterations) to T = ln(1.3) / |omega(q)|; the growth rate ln(A(T) / A(0)) / T of
             the mode's projection A against omega(q) = q^2 (f1 - f0 q^2).

All runs use the trapezoidal rule (theta = 1/2, eq. TrapRule) and the initial condition of
eq. IC_LinearWave (synth.wave_film; eps_x = eps_y = 0.1 except where stated). The model
coefficients f0(H0), f1(H0) that set q_m and omega_m come from the library's own device
evaluation (tf_model_coeffs).
"""
import argparse
import json
import math

import numpy as np

from . import synth
from .lib import Grid

MODELS = {"linear": 1.0, "nlc": 0.5, "polymer": 3.9}


def _torch():
    import torch
    return torch


def make_grid(kind, n, ds, **scheme):
    g = Grid(n, n, ds)
    getattr(g, "set_model_" + kind)()
    g.set_scheme(**scheme)
    return g


def lsa_params(kind, h0=None):
    """(H0, f0(H0), f1(H0), q_m, omega_m): q_m^2 = f1 / (2 f0), omega_m = f1^2 / (4 f0);
    H0 defaults to the model's thickness in Sec. "Validation"."""
    torch = _torch()
    h0 = MODELS[kind] if h0 is None else h0
    g = make_grid(kind, 4, 1.0)
    out = torch.empty((1, 4), dtype=torch.float64, device="cuda:0")
    g.model_coeffs(torch.full((1,), h0, dtype=torch.float64, device="cuda:0"), out)
    f0, _, f1, _ = out[0].tolist()
    return h0, f0, f1, math.sqrt(f1 / (2.0 * f0)), f1 * f1 / (4.0 * f0)


def _run(kind, u0, ds, dt, nsteps, tol, sample_every=None):
    """Fixed-dt trapezoidal run; returns (u, [mean-thickness change every sample_every])."""
    torch = _torch()
    n = u0.shape[0]
    g = make_grid(kind, n, ds, theta=0.5, tol=tol, max_newton=5000)
    h = torch.from_numpy(np.ascontiguousarray(u0)).to("cuda:0")
    g.bind(h)
    m0, _ = g.mass()
    rel = []
    done = 0
    while done < nsteps:
        k = min(sample_every or nsteps, nsteps - done)
        g.advance(k, dt)
        done += k
        if sample_every:
            rel.append(g.mass()[0] / m0 - 1.0)
    return h.cpu().numpy(), rel


def _rms(a):
    return float(math.sqrt(np.mean(a * a)))


def _orders(errs, ratio):
    return [math.log(errs[i] / errs[i + 1], ratio) if errs[i + 1] > 0 else float("nan")
            for i in range(len(errs) - 1)]


def temporal_solutions(kind, I0=256, levels=6, tol_mode="machine", P=6):
    """Solutions at t = dt0 for dt_i = 2^-i dt0, i = 0..levels."""
    h0, _, _, qm, wm = lsa_params(kind)
    u0, ds = synth.wave_film(I0, P, qm, h0)
    dt0 = 1e-3 / wm
    sols = []
    for i in range(levels + 1):
        dt = dt0 / 2 ** i
        tol = 1e-14 if tol_mode == "machine" else max(dt * dt, 1e-14)
        sols.append(_run(kind, u0, ds, dt, 2 ** i, tol)[0])
    return sols, dt0


def temporal(kind, I0=256, levels=6, tol_mode="machine", P=6):
    sols, dt0 = temporal_solutions(kind, I0, levels, tol_mode, P)
    errs = [_rms(s - sols[-1]) for s in sols[:-1]]
    return {"test": "temporal", "model": kind, "tol": tol_mode, "I0": I0, "dt0": dt0,
            "errors": errs, "orders": _orders(errs, 2.0)}


def nested(u, m):
    """Cells of u whose centres are the centres of the grid m times coarser (m odd)."""
    n = u.shape[0] // m
    idx = m * np.arange(n) + (m - 1) // 2
    return u[np.ix_(idx, idx)]


def spatial_solutions(kind, I0=36, levels=5, tol_mode="machine", P=6):
    """Solutions after one step of dt0 = 1e-8 / omega_m on I0 * 3^k cells, k < levels."""
    h0, _, _, qm, wm = lsa_params(kind)
    dt = 1e-8 / wm
    sols = []
    for k in range(levels):
        u0, ds = synth.wave_film(I0 * 3 ** k, P, qm, h0)
        tol = 1e-14 if tol_mode == "machine" else max(ds * ds, 1e-14)
        sols.append(_run(kind, u0, ds, dt, 1, tol)[0])
    return sols, dt


def spatial(kind, I0=36, levels=5, tol_mode="machine", P=6):
    sols, dt = spatial_solutions(kind, I0, levels, tol_mode, P)
    fine = sols[-1]
    errs = [_rms(sols[k] - nested(fine, 3 ** (levels - 1 - k))) for k in range(levels - 1)]
    return {"test": "spatial", "model": kind, "tol": tol_mode, "I": [I0 * 3 ** k for k in range(levels)],
            "dt": dt, "errors": errs, "orders": _orders(errs, 3.0)}


def mass(kind, family, level, P=6):
    h0, _, _, qm, wm = lsa_params(kind)
    if family == "space":
        n, dt, steps, every = 36 * 3 ** level, 1e-8 / wm, 1000, 100
        u0, ds = synth.wave_film(n, P, qm, h0)
        tol = max(ds * ds, 1e-14)
    else:
        n, dt = 1024, 1e-3 / wm / 2 ** level
        steps, every = 1000 * 2 ** level, 100 * 2 ** level
        u0, ds = synth.wave_film(n, P, qm, h0)
        tol = max(dt * dt, 1e-14)
    _, rel = _run(kind, u0, ds, dt, steps, tol, sample_every=every)
    return {"test": "mass", "model": kind, "family": family, "level": level, "I": n, "dt": dt,
            "steps": steps, "rel_mass_change": rel, "max_abs": max(abs(r) for r in rel)}


def run_to_time(g, T, dt):
    """Adaptive steps until t = T (the last step is shortened to land on T)."""
    t, steps = 0.0, 0
    while t < T * (1.0 - 1e-14):
        res = g.step(min(dt, T - t))
        t += res.info["dt_used"]
        dt = res.dt_next
        steps += 1
    return steps


def lsa_rate(kind, frac, eps=0.1, axis="x", I=32):
    """Growth rate of the mode q = frac * q_m from a P = 1 run (Sec. "Comparison to LSA")."""
    torch = _torch()
    h0, f0, f1, qm, wm = lsa_params(kind)
    q = frac * qm
    w = q * q * (f1 - f0 * q * q)
    T = math.log(1.3) / abs(w)
    ex, ey = (eps, 0.0) if axis == "x" else (0.0, eps)
    u0, ds = synth.wave_film(I, 1, q, h0, ex, ey)
    g = make_grid(kind, I, ds, theta=0.5, tol=1e-10, adaptive=1, max_newton=10, dt_min=1e-9, dt_max=1.0)
    h = torch.from_numpy(np.ascontiguousarray(u0)).to("cuda:0")
    g.bind(h)
    steps = run_to_time(g, T, T / 100.0)
    c = np.cos(q * (np.arange(I) + 0.5) * ds)
    mode = c[None, :] if axis == "x" else c[:, None]
    a0 = float(np.mean((u0 - h0) * mode))
    a1 = float(np.mean((h.cpu().numpy() - h0) * mode))
    ws = math.log(a1 / a0) / T
    return {"test": "lsa", "model": kind, "axis": axis, "eps": eps, "q": q, "q_over_qm": frac, "T": T,
            "omega_lsa": w, "omega_sim": ws, "dev_over_omega_m": (ws - w) / wm, "steps": steps}


LSA_FRACS = (0.25, 0.5, 0.75, 1.0, 1.25, 1.375)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="smaller grids and fewer levels")
    ap.add_argument("--out", help="also write the JSON lines to this file")
    a = ap.parse_args(argv)
    recs = []

    def emit(r):
        recs.append(r)
        print(json.dumps(r), flush=True)

    for kind in MODELS:
        h0, f0, f1, qm, wm = lsa_params(kind)
        emit({"test": "lsa_params", "model": kind, "H0": h0, "f0": f0, "f1": f1, "q_m": qm, "omega_m": wm})
        for tol in ("machine", "scaled"):
            emit(temporal(kind, I0=64 if a.quick else 256, levels=4 if a.quick else 6, tol_mode=tol))
            emit(spatial(kind, levels=3 if a.quick else 5, tol_mode=tol))
        for lvl in range(2 if a.quick else 5):
            emit(mass(kind, "space", lvl))
        for lvl in range(1 if a.quick else 5):
            emit(mass(kind, "time", lvl))
        for eps in (0.1, 1e-3):
            for axis in ("x", "y"):
                for fr in LSA_FRACS:
                    emit(lsa_rate(kind, fr, eps, axis))
    if a.out:
        with open(a.out, "w") as f:
            for r in recs:
                f.write(json.dumps(r) + "\n")


if __name__ == "__main__":
    main()
