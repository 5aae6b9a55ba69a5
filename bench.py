"""Throughput benchmark of the FP64 ADI-Newton thin-film step on one MI355X.

Workload (default): the 8192^2 film, L = 256 lambda_m, h0 = 1 + 0.01 U[-1,1] (seed 2),
backward Euler dt = 0.2, Newton tol 1e-10, fixed dt, 500 steps (the default K; each
workload has its own default step count). A "step" is one accepted time
step (every Newton iteration of it: residual, y sweep, x sweep, update, reductions).
W untimed warm-up steps are taken first, then exactly K steps are timed between
stream synchronisations with the state resident in HBM; the same window is run three
times from the same state (bit-identical work) and the median is reported.

Printed: one JSON line with steps/s, the roofline record of one Newton iteration's
kernels (48 algorithmic bytes per cell over their mean time per iteration, from HIP
events around every launch in a fourth, profiled run of the window) and the oracle's
rate on the host (one full step of the same film, see cpu_baseline.sample).
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("ADI steps/s & HBM GB/s (FP64, 2048²/8192²); ensemble + adjoint cost vs forward")
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell per Newton iteration: the y sweep must read u_k and b^n and
# write w, the x sweep read u_k and w and write u_{k+1}, each once: 48 B.
ALGO_BYTES_PER_CELL_ITERATION = 48.0
# The bytes of each kernel class taken alone (the inputs it reads, the field it writes).
ALGO_BYTES_PER_CELL = {"relations_y": 16, "solve_y": 24, "relations_x": 16, "solve_x": 24, "xrow": 24}
KERNEL_SOURCES = ["paper_1806_10550_amd/csrc/tf_kernels.hip", "paper_1806_10550_amd/csrc/tf_internal.h",
                  "paper_1806_10550_amd/csrc/tf_device.h", "paper_1806_10550_amd/csrc/tf_sweep.h",
                  "paper_1806_10550_amd/csrc/tf_xrow.hip"]
def traffic_file(config="large8192"):
    return os.path.join(ROOT, "profiles", f"traffic_{config}.json")


def kernel_hash():
    """Hash of the kernel sources with their comments and layout removed: it changes when the
    code the committed counter records and kernel traces were taken on changes, not when a
    comment does."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def sq_file(config="large8192"):
    return os.path.join(ROOT, "profiles", f"sq_{config}.json")


def fp64_flops_for(kernel, config="large8192"):
    """FP64 flops per launch of a kernel class from the committed SQ counter summary, or None
    when absent or taken on different kernel sources."""
    try:
        with open(sq_file(config)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    v = t.get("kernels", {}).get(kernel, {}).get("SQ_INSTS_VALU_FLOPS_FP64")
    # the counter adds each wave instruction's flops once (FMA 2, MUL/ADD 1): x 64 lanes
    return 64.0 * v if v else None


def copy_rate_gbs():
    """The plain copy's measured rate from the committed counter summary (any kernel sources)."""
    try:
        with open(traffic_file()) as f:
            return json.load(f).get("copy_gbs")
    except (OSError, ValueError):
        return None


def iteration_traffic(ncells, config="large8192"):
    """HBM bytes of one Newton iteration (the sweep launches) from the committed counter
    summary of the workload, or None when absent or taken on different kernel sources."""
    try:
        with open(traffic_file(config)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    ks = t.get("kernels", {})
    per = {"relations_y": 1, "solve_y": 1, "chain": 1}
    per.update({"xrow": 1} if "xrow" in ks else {"relations_x": 1, "solve_x": 1, "chain": 2})
    if any(k not in ks for k in per):
        return None
    return sum(n * (ks[k]["fetch_kib"] + ks[k]["write_kib"]) * 1024.0 * t.get("copy_scale", 1.0)
               for k, n in per.items())


def traffic_for(kernel, ncells, config="large8192"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when
    absent or taken on different kernel sources."""
    try:
        with open(traffic_file(config)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or kernel not in t.get("kernels", {}):
        return None
    k = t["kernels"][kernel]
    return (k["fetch_kib"] + k["write_kib"]) * 1024.0 * t.get("copy_scale", 1.0)


def cpu_baseline(h_np, ds, dt, scheme, successes, model="power", max_steps=1, budget_s=10.0):
    """The oracle (plain C, OpenMP over independent lines) timed on the host cores for whole
    accepted steps (every Newton iteration of each) of the same film from the state the GPU
    run ended at, with the same scheme: consecutive steps until `budget_s` seconds have been
    spent or `max_steps` steps taken (at least one), steps/s = steps / time. Also per Newton
    iteration (the unit that does not depend on the step window) and one thread on a 1/64
    sub-film."""
    from oracle import oracle as orc
    threads = len(os.sched_getaffinity(0))
    orc.set_threads(threads)
    M = orc.Model(kappa=10.0, b=0.1, n=3.0, m=2.0) if model == "power" else getattr(orc.Model, model)()
    S = orc.Scheme(**scheme)
    u, steps, iters, status = h_np, 0, 0, 0
    t0 = time.perf_counter()
    while True:
        u, res = orc.step(M, S, u, ds, dt, successes)
        steps += 1
        iters += res.total_iters
        status = res.status
        dt, successes = res.dt_next, res.successes
        t_all = time.perf_counter() - t0
        if res.status != 0 or steps >= max_steps or t_all >= budget_s:
            break
    cores = orc.get_threads()
    # one thread: one Newton iteration on the top-left eighth by eighth of the film, scaled
    # by the cell count
    sub = np.ascontiguousarray(h_np[: max(h_np.shape[0] // 8, 4), : max(h_np.shape[1] // 8, 4)])
    orc.set_threads(1)
    t0 = time.perf_counter()
    orc.adi_iteration(M, sub, sub, ds, dt, scheme.get("theta", 1.0))
    t_1 = (time.perf_counter() - t0) * (h_np.size / sub.size)
    orc.set_threads(threads)
    return {"value": steps / t_all, "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": (f"{steps} consecutive accepted step(s) of the {h_np.shape[1]}x{h_np.shape[0]} film from the "
                       f"state the GPU run ended at ({iters} Newton iterations, {t_all:.2f} s, last status {status})"),
            "steps": steps,
            "newton_iters": iters,
            "ms_per_newton_iteration": 1e3 * t_all / max(iters, 1),
            "grid_point_iterations_per_s": h_np.size * iters / t_all,
            "single_thread_ms_per_newton_iteration": 1e3 * t_1,
            "single_thread_sample": (f"one Newton iteration on {sub.shape[1]}x{sub.shape[0]} cells of the same "
                                     f"film on one thread, scaled to the full film")}


def bench_ensemble(args):
    """256-film ensemble (sizes from {256..1024}^2, kappa ~ U[5,20], L = 8 lambda_m each,
    noise 0.01, backward Euler from dt = 0.1 with the adaptive control of Fig.
    FlowChartTime, K = 10) in one packed buffer with graph-captured iterations, against a
    loop of plain single-film solves of the same films. The finest films have ds ~ 0.12,
    where a fixed dt = 0.1 would need tens of thousands of Newton iterations per step, so
    every film adapts its own dt."""
    import numpy as np
    import torch

    from paper_1806_10550_amd import synth
    from paper_1806_10550_amd.lib import Ensemble, Grid

    films = synth.ensemble_films(args.films)
    nx = [f.n for f in films]
    ds = [f.ds for f in films]
    kap = [f.kappa for f in films]
    h0 = [synth.noise_film(f.n, f.n, f.seed, 1.0, 0.01) for f in films]
    dev = torch.device("cuda:0")
    ens = Ensemble(nx, nx, ds, kap)
    ens.set_xsweep(args.xsweep)
    scheme = dict(tol=1e-10, max_newton=10, adaptive=1, dt_min=1e-9, dt_max=1.0, dt_shrink=0.5, dt_grow=1.1,
                  grow_after=5)
    ens.set_scheme(**scheme)
    packed = torch.empty(ens.size, dtype=torch.float64, device=dev)
    for f, h in enumerate(h0):
        ens.view(packed, f).copy_(torch.from_numpy(h))
    ens.bind(packed)
    dts = [0.1] * len(films)
    if args.warmup:
        st, dts, _, _ = ens.step(args.warmup, dts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, dts, sts, its = ens.step(args.steps, dts)
    torch.cuda.synchronize()
    t_ens = time.perf_counter() - t0
    # the same films, one single-film solve after another
    grids, states = [], []
    for f in range(len(films)):
        g = Grid(nx[f], nx[f], ds[f])
        g.set_model(kap[f], 0.1, 3, 2)
        g.set_scheme(**scheme)
        g.set_xsweep(ens.xsweep(f))  # the variant the ensemble gives this film
        h = torch.from_numpy(h0[f]).to(dev)
        g.bind(h)
        dtf = 0.1
        if args.warmup:
            dtf, _ = g.advance(args.warmup, dtf)
        grids.append((g, dtf))
        states.append(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loop_iters = 0
    for g, dtf in grids:
        _, log = g.advance(args.steps, dtf, log=True)
        loop_iters += sum(x["total_iters"] for x in log)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    same = all(torch.equal(ens.view(packed, f), states[f]) for f in range(len(films)))
    cells = sum(n * n for n in nx)
    out = {"metric": "ensemble film-steps/s vs loop of single-film solves", "value": len(films) * args.steps / t_ens,
           "unit": "film-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"ensemble of {len(films)} films, sizes {{256..1024}}^2, kappa~U[5,20], "
                                  f"L=8 lambda_m, noise 0.01 (default_rng(3)), backward Euler, adaptive dt from 0.1 "
                                  f"(K=10), tol 1e-10",
                      "cells": cells},
           "xsweep": {v: sum(ens.xsweep(f) == v for f in range(len(films))) for v in ("row", "partitioned")},
           "ensemble_s": t_ens, "loop_s": t_loop, "loop_over_ensemble": t_loop / t_ens,
           "newton_iters_total": int(sum(its)), "loop_newton_iters_total": loop_iters,
           "bitwise_equal_to_loop": bool(same), "status_ok": st == 0,
           "dt_range": [min(dts), max(dts)],
           "cell_iterations_per_s": sum(n * n * i for n, i in zip(nx, its)) / t_ens,
           # 48 algorithmic bytes per cell per Newton iteration of each film still iterating
           "iteration_roofline_frac": 48.0 * sum(n * n * i for n, i in zip(nx, its)) / t_ens / (HBM_PEAK_GBS * 1e9)}
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """512^2 film (L = 16 lambda_m), kappa = 10, backward Euler dt = 0.1 for `steps`
    steps; loss 0.5 ||h(T) - h_target||^2 with h_target a forward run from another seed;
    gradient in the initial perturbation and kappa by the checkpointed discrete adjoint
    (h stored every 20 steps, steps in between recomputed). Reports the time of forward +
    backward against the plain forward."""
    import torch

    from paper_1806_10550_amd import synth
    from paper_1806_10550_amd.adjoint import Rollout, rollout
    from paper_1806_10550_amd.lib import Grid, autotune_choice

    cfg = synth.CONFIGS["adjoint512"]
    n, dt, steps = cfg.n, cfg.dt, args.steps
    dev = torch.device("cuda:0")
    base = torch.from_numpy(synth.noise_film(n, n, cfg.seed, 1.0, 0.01)).to(dev)
    tgt = torch.from_numpy(synth.noise_film(n, n, cfg.extra["target_seed"], 1.0, 0.01)).to(dev)
    g = Grid(n, n, cfg.ds)
    g.set_model(cfg.kappa, cfg.b, 3, 2)
    g.set_scheme(theta=1.0, tol=cfg.tol, max_newton=5000)
    if args.xsweep != "auto":
        # the x-sweep variant of the forward and of the adjoint's transposed row solves
        from paper_1806_10550_amd import adjoint
        g.set_xsweep(args.xsweep)
        adjoint._grid(n, n, cfg.ds).set_xsweep(args.xsweep)
    g.bind(tgt)
    g.advance(steps, dt)                      # target = forward run from seed 5
    h = base.clone()
    g.bind(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, log = g.advance(steps, dt, log=True)   # plain forward
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    fwd_iters = sum(x["total_iters"] for x in log)
    p0 = torch.zeros_like(base, requires_grad=True)
    kap = torch.tensor(cfg.kappa, dtype=torch.float64, device=dev, requires_grad=True)
    # warm-up: a short rollout through forward and backward (first kernel loads, the
    # adjoint scratch of a grid, the solver tuning table), as the forward was warmed up
    # by the target run
    w = rollout(p0, kap, base, cfg.extra["checkpoint_every"], dt, cfg.ds,
                checkpoint_every=cfg.extra["checkpoint_every"], tol=cfg.tol, adj_tol=cfg.tol)
    (0.5 * torch.sum((w - tgt) ** 2)).backward()
    p0.grad = None
    kap.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the adjoint iteration stops at the forward Newton tolerance: the states it
    # differentiates are themselves converged only to that level
    hT = rollout(p0, kap, base, steps, dt, cfg.ds, checkpoint_every=cfg.extra["checkpoint_every"],
                 tol=cfg.tol, adj_tol=cfg.tol)
    loss = 0.5 * torch.sum((hT - tgt) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    out = {"metric": "adjoint (forward + recompute + backward) time vs plain forward", "value": t_adj / t_fwd,
           "unit": "ratio", "n_gpus": 1, "steps": steps, "higher_is_better": False, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"adjoint512: {n}x{n} film, L=16 lambda_m, kappa=10, backward Euler dt={dt}, "
                                  f"{steps} steps, checkpoints every {cfg.extra['checkpoint_every']}, "
                                  f"loss 0.5||h(T)-h_target||^2"},
           "forward_s": t_fwd, "forward_plus_adjoint_s": t_adj, "forward_newton_iters": fwd_iters,
           "richardson_iters": Rollout.stats["richardson_iters"],
           "solver_variant": autotune_choice(n, n, transposed=True), "xsweep": g.xsweep(),
           "loss": loss.item(), "grad_p0_norm": p0.grad.norm().item(), "grad_kappa": kap.grad.item()}
    print(json.dumps(out), flush=True)


def bench_spectrum(args):
    """Radial Fourier transform (steps 1-4 on the GPU, 5-7 in the library on the host) of an
    NLC film at the paper's largest grid: I = 4000, P = 40 wavelengths at H0 = 0.5,
    pseudo-Perlin noise (eq. 3D_Random_IC, seed 7); sigma = 1, q <= 5 q_m."""
    import torch

    from paper_1806_10550_amd import synth
    from paper_1806_10550_amd.lib import radial_spectrum, spectrum_maxima

    n, P, h0, qm = 4000, 40, 0.5, 1.4821222565068524
    lam = 2 * math.pi / qm
    h_np, ds = synth.random_film(n, P, lam, h0, seed=7)
    h = torch.from_numpy(h_np).to("cuda:0")
    qmax = 5 * qm
    for _ in range(args.warmup):
        radial_spectrum(h, ds, h0, 1.0, qmax)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        q, v, _ = radial_spectrum(h, ds, h0, 1.0, qmax)
        _, _, peaks = spectrum_maxima(q, v, qmax)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    algo = 8.0 * n * n  # the film must be read once
    out = {"metric": "radial Fourier spectra per second (App. Radial Fourier Transform)", "value": 1.0 / t,
           "unit": "spectra/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t,
           "higher_is_better": True, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"NLC film {n}x{n}, P={P} wavelengths at H0={h0}, pseudo-Perlin noise seed 7, "
                                  f"sigma=1, q<=5q_m"},
           "roofline": {"bound": "hbm", "kernel": "whole call (FFT + smoothing + group sums + readback)",
                        "achieved": algo / t / 1e9, "peak": 8000.0, "unit": "GB/s", "frac": algo / t / 8e12,
                        "traffic": None},
           "groups": int(len(q)), "peaks": len(peaks)}
    if not args.no_cpu_baseline:
        from oracle import radial as R
        t1 = time.perf_counter()
        R.dominant_wavenumbers(h_np, h0, ds, 1.0, qmax)
        tc = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": 1.0 / tc, "unit": "spectra/s", "cores": 1, "kind": "oracle",
                               "sample": "one full spectrum of the same film (NumPy FFT, one thread)"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps; default: the workload's own count (single film: the config's steps, "
                         "500 for the 8192^2 film; ensemble: 300; adjoint: 400; spectrum: 60)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="large8192")
    ap.add_argument("--workload", default="single", choices=["single", "ensemble", "adjoint", "spectrum"],
                    help="single: the 8192^2 film (default); ensemble: 256 ragged films; "
                         "adjoint: 512^2 gradient by the checkpointed adjoint; "
                         "spectrum: radial Fourier transform of a 4000^2 film")
    ap.add_argument("--films", type=int, default=256)
    ap.add_argument("--xsweep", default="auto", choices=["auto", "row", "partitioned"],
                    help="ensemble and adjoint workloads: x-sweep line solver (auto: as tuned for the shape)")
    ap.add_argument("--model", default="power", choices=["power", "nlc", "polymer"],
                    help="single workload only: the power law of the default workload, or the NLC "
                         "(H0 = 0.5) / polymer (H0 = 3.9) film on the same grid with L = 256 lambda_m "
                         "and the same dt * omega_m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--print-hash", action="store_true", help="print the kernel-source hash and exit")
    args = ap.parse_args()
    if args.print_hash:
        print(kernel_hash())
        return
    if args.calibrate_copy:
        import torch
        n = (1 << 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = {"ensemble": 300, "adjoint": 400, "spectrum": 60}.get(args.workload)
    if args.steps is None:
        from paper_1806_10550_amd import synth
        args.steps = synth.CONFIGS[args.config].steps
    if args.steps < 1:
        print("--steps must be >= 1", file=sys.stderr)
        sys.exit(2)

    if args.workload == "ensemble":
        bench_ensemble(args)
        return
    if args.workload == "adjoint":
        bench_adjoint(args)
        return
    if args.workload == "spectrum":
        bench_spectrum(args)
        return

    import torch

    from paper_1806_10550_amd import synth
    from paper_1806_10550_amd.lib import Grid

    cfg = synth.CONFIGS[args.config]
    n = cfg.n
    dev = torch.device("cuda:0")
    if args.model == "power":
        h_np, ds, dt0 = cfg.film(), cfg.ds, cfg.dt
        g = Grid(n, n, ds)
        g.set_model(cfg.kappa, cfg.b, cfg.nexp, cfg.mexp)
        workload = (f"{cfg.name}: {n}x{n} film, L={cfg.periods:g} lambda_m, noise 0.01 seed {cfg.seed}, "
                    f"backward Euler dt={cfg.dt}, tol {cfg.tol}, fixed dt")
    else:
        from paper_1806_10550_amd.validate import lsa_params
        h0, _, _, qm, wm = lsa_params(args.model)
        ds = cfg.periods * 2 * math.pi / qm / n
        dt0 = cfg.dt * synth.omega_m(cfg.kappa, cfg.b, cfg.nexp, cfg.mexp) / wm
        h_np = synth.noise_film(n, n, cfg.seed, h0, 0.01 * h0)
        g = Grid(n, n, ds)
        getattr(g, "set_model_" + args.model)()
        workload = (f"{args.model}{n}: {n}x{n} {args.model.upper()} film at H0={h0}, L={cfg.periods:g} lambda_m, "
                    f"noise 0.01 H0 seed {cfg.seed}, backward Euler dt={dt0:.4g} (dt omega_m as {cfg.name}), "
                    f"tol {cfg.tol}, fixed dt")
    h = torch.from_numpy(h_np).to(dev)
    if cfg.adaptive:
        scheme = dict(theta=1.0, tol=cfg.tol, max_newton=10, adaptive=1, dt_min=1e-6, dt_max=1.0, dt_shrink=0.5,
                      dt_grow=1.1, grow_after=5)
        workload = workload.replace("fixed dt", "adaptive dt (K=10)")
    else:
        scheme = dict(theta=1.0, tol=cfg.tol, max_newton=5000, adaptive=0)
    g.set_scheme(**scheme)
    g.bind(h)
    dt = dt0
    if args.warmup > 0:
        dt, _ = g.advance(args.warmup, dt)
    # the timed window starts from this state; every run below repeats it exactly
    torch.cuda.synchronize()
    saved, (t_clock, succ), dt_start = h.clone(), g.clock(), dt

    def run(profiled):
        h.copy_(saved)
        g.set_clock(t_clock, succ)
        g.profile(profiled)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dt_end, log = g.advance(args.steps, dt_start, log=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = g.profile_read() if profiled else None
        g.profile(False)
        return el, log, prof, dt_end

    # headline: median of three unprofiled runs of the same window (no events in them)
    runs = sorted((run(False) for _ in range(3)), key=lambda r: r[0])
    elapsed, log, _, dt_end = runs[1]
    # kernel breakdown: one more run of the same window with an event pair per launch
    el_prof, log_prof, prof, _ = run(True)
    iters = [x["newton_iters"] for x in log]
    total_iters = sum(x["total_iters"] for x in log)
    assert sum(x["total_iters"] for x in log_prof) == total_iters
    ncells = n * n
    steps_per_s = args.steps / elapsed

    # The roofline record covers the kernels of one Newton iteration (the six launches of the
    # y and x sweeps) as a unit: 48 algorithmic bytes per cell per iteration (each sweep reads
    # its two inputs and writes its output once) over their mean time per iteration from the
    # per-launch HIP events of the profiled run.
    # the kernels of one iteration: the y sweep's three, then the x sweep's (one whole-row
    # kernel, or three with the partitioned variant)
    sweep = ["relations_y", "chain_y", "solve_y"] + (
        ["xrow"] if prof.get("xrow", (0, 0))[1] else ["relations_x", "chain_x", "solve_x"])
    iter_kernel_s = sum(prof[k][0] for k in sweep) / 1e3 / total_iters
    achieved = ALGO_BYTES_PER_CELL_ITERATION * ncells / iter_kernel_s / 1e9
    traffic = iteration_traffic(ncells, args.config) if args.model == "power" else None
    kernel_ms = sum(v[0] for v in prof.values())
    iter_frac = (ALGO_BYTES_PER_CELL_ITERATION * ncells * total_iters) / (elapsed * HBM_PEAK_GBS * 1e9)
    dom = max((k for k in ALGO_BYTES_PER_CELL if k in prof), key=lambda k: prof[k][0])
    dom_s = prof[dom][0] / 1e3 / max(prof[dom][1], 1)

    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "nx": n, "ny": n, "dt": dt0, "tol": cfg.tol},
        "roofline": {"bound": "hbm", "kernel": "newton_iteration (" + ", ".join(sweep) + ")",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic},
        "ms_per_newton_iteration": 1e3 * elapsed / total_iters,
        "kernel_ms_per_newton_iteration": 1e3 * iter_kernel_s,
        "newton_iters_per_step": total_iters / args.steps,
        "newton_iters_distribution": {"min": min(iters), "median": sorted(iters)[len(iters) // 2],
                                      "max": max(iters)},
        "runs_s": [r[0] for r in runs],
        "profiled_run_s": el_prof,
        "copy_kernel_gbs": copy_rate_gbs(),
        "grid_point_steps_per_s": steps_per_s * ncells,
        "grid_point_iterations_per_s": total_iters * ncells / elapsed,
        # the same 48 B per cell-iteration over the whole wall time of the timed window
        "iteration_roofline_frac": iter_frac,
        "kernel_ms": {k: round(v[0], 3) for k, v in prof.items()},
        "kernel_launches": {k: v[1] for k, v in prof.items()},
        "kernel_mean_us": {k: round(1e3 * v[0] / v[1], 2) for k, v in prof.items() if v[1]},
        "kernel_busy_frac": kernel_ms / (1e3 * el_prof),
        # the longest kernel class alone, with its own share of the bytes (counters: actual HBM
        # bytes per launch) and its FP64 rate from the committed SQ counters
        "dominant_kernel": {"kernel": dom, "mean_us": 1e6 * dom_s,
                            "algorithmic_gbs": ALGO_BYTES_PER_CELL[dom] * ncells / dom_s / 1e9,
                            "traffic": traffic_for(dom, ncells, args.config) if args.model == "power" else None,
                            "fp64_tflops": ((fp64_flops_for(dom, args.config) / dom_s / 1e12)
                                            if fp64_flops_for(dom, args.config) else None)},
    }
    if not args.no_cpu_baseline:
        h_now = h.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(h_now, ds, dt_end, scheme, g.clock()[1], args.model,
                                           max_steps=args.steps)
    print(json.dumps(out), flush=True)
    g.close()


if __name__ == "__main__":
    main()
