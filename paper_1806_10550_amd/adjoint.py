"""Differentiable rollout of the ADI-Newton stepper (torch.autograd.Function).

Forward: h(0) = h_base + p0, then nsteps theta-scheme steps of fixed dt (tf_step; theta = 1
backward Euler, 1/2 the trapezoidal rule of eq. TrapRule), storing h every
`checkpoint_every` steps. Backward: for each checkpoint segment, newest first, the steps are
recomputed from the stored state (bit-identical: same kernels, same order) and the discrete
adjoint of every step is applied (tf_adjoint_step), giving dL/dp0 = lambda^0 and, for the
power-law model, dL/dkappa. The adjoint is that of the converged implicit step map
(implicit-function theorem), with the dt sequence held fixed. The linear, NLC and polymer
models (model="linear" / "nlc" / "polymer", parameters in model_params) have no kappa: their
rollouts take kappa=None and differentiate in p0 only.
"""
from __future__ import annotations

import torch

from .lib import Grid, load_shipped_tuning


# Grids (and with them their device scratch and adjoint buffers) are reused across
# rollouts of the same geometry on the same stream; every forward and backward pass sets
# the model and the scheme it needs before using one. A grid enqueues its work on the torch
# stream that was current when it was created, so the key holds that stream too: the
# tensor copies of a rollout (checkpoint clones, restores) then run in order with the
# library's launches.
_grids = {}


def _grid(nx, ny, ds):
    stream = torch.cuda.current_stream()
    key = (nx, ny, float(ds), stream.device.index, stream.cuda_stream)
    g = _grids.get(key)
    if g is None:
        g = _grids[key] = Grid(nx, ny, ds, stream=stream)
    return g


class Rollout(torch.autograd.Function):
    # totals of the last backward pass: adjoint steps and Richardson iterations
    stats = {"adjoint_steps": 0, "richardson_iters": 0}

    @staticmethod
    def forward(ctx, p0, kappa, h_base, nsteps: int, dt: float, ds: float, checkpoint_every: int = 20,
                tol: float = 1e-10, adj_tol: float = 1e-13, b: float = 0.1, n: int = 3, m: int = 2,
                theta: float = 1.0, kind: str = "power", params=None):
        ny, nx = h_base.shape
        g = _grid(nx, ny, ds)
        if kind == "power":
            model = (kind, (float(kappa.detach().item()), b, n, m))
        else:
            if kappa is not None:
                raise ValueError(f"the {kind} model has no kappa: pass kappa=None")
            model = (kind, dict(params or {}))
        _set_model(g, model)
        g.set_scheme(theta=theta, tol=tol, max_newton=5000)
        h = (h_base + p0).detach().contiguous().clone()
        g.bind(h)
        ckpts = [h.clone()]
        done = 0
        while done < nsteps:  # one library call per checkpoint segment (fixed dt)
            k = min(checkpoint_every, nsteps - done)
            g.advance(k, dt)
            done += k
            if done < nsteps:
                ckpts.append(h.clone())
        ctx.grid = g
        ctx.ckpts = ckpts
        ctx.cfg = (nsteps, dt, checkpoint_every, adj_tol, model, tol, theta)
        ctx.kappa_shape = kappa.shape if kappa is not None else None
        return h.clone()

    @staticmethod
    def backward(ctx, grad_h):
        g = ctx.grid
        nsteps, dt, K, adj_tol, model, tol, theta = ctx.cfg
        _set_model(g, model)
        g.set_scheme(theta=theta, tol=tol, max_newton=5000)
        power = model[0] == "power"
        load_shipped_tuning()  # solver variants tuned for this GPU, if shipped
        steps = iters = 0
        lam = grad_h.detach().contiguous().clone()
        gk = 0.0
        work = torch.empty_like(lam)
        g.bind(work)
        nseg = len(ctx.ckpts)
        # each segment: recompute its states from the checkpoint in one call, then its adjoint
        # steps (newest first) in another
        states = torch.empty((K + 1,) + tuple(lam.shape), dtype=lam.dtype, device=lam.device)
        for seg in range(nseg - 1, -1, -1):
            start = seg * K
            end = min(nsteps, start + K)
            m = end - start
            work.copy_(ctx.ckpts[seg])
            states[0].copy_(ctx.ckpts[seg])
            g.advance_keep(m, dt, states[1:m + 1])
            c, it = g.adjoint_steps(states[:m + 1], dt, lam, tol=adj_tol, dkappa=power)
            gk += c if power else 0.0
            steps += m
            iters += it
        Rollout.stats = {"adjoint_steps": steps, "richardson_iters": iters}
        grad_k = (torch.full(ctx.kappa_shape, gk, dtype=torch.float64, device=lam.device) if power else None)
        return (lam, grad_k) + (None,) * 13


def _set_model(g, model):
    kind, args = model
    if kind == "power":
        g.set_model(*args)
    elif kind in ("linear", "nlc", "polymer"):
        getattr(g, "set_model_" + kind)(**args)
    else:
        raise ValueError(f"unknown model {kind!r}")


def rollout(p0, kappa, h_base, nsteps, dt, ds, checkpoint_every=20, tol=1e-10, adj_tol=1e-13, b=0.1, n=3, m=2,
            theta=1.0, model="power", model_params=None):
    """h(T) of the film h_base + p0 after nsteps steps of the theta scheme; differentiable in
    p0 and (power-law model) kappa, a 0-d float64 tensor. model: "power" (kappa, b, n, m),
    or "linear" / "nlc" / "polymer" with kappa=None and the keyword parameters of
    Grid.set_model_<model> in model_params (defaults: the paper's)."""
    return Rollout.apply(p0, kappa, h_base, nsteps, dt, ds, checkpoint_every, tol, adj_tol, b, n, m, theta, model,
                         model_params)
