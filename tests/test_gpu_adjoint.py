"""GPU adjoint path: transposed Jacobian, stored-band pentadiagonal solves, one adjoint
step and the checkpointed rollout gradient, against the CPU oracle and finite
differences."""
import json
import math

import numpy as np
import pytest
import torch

from paper_1806_10550_amd import synth
from paper_1806_10550_amd.adjoint import rollout
from paper_1806_10550_amd.lib import Grid, TFError, autotune, autotune_choice, autotune_load, penta_solve

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def grid(nx, ny, ds, theta=1.0, kappa=10.0, **kw):
    g = Grid(nx, ny, ds)
    g.set_model(kappa, 0.1, 3, 2)
    g.set_scheme(theta=theta, **kw)
    return g


@pytest.mark.parametrize("nx,ny", [(9, 7), (70, 66), (130, 67)])
def test_jacobian_transpose_matches_oracle(orc, nx, ny):
    u = synth.noise_film(nx, ny, seed=nx + ny, amp=0.2)
    mu = np.random.default_rng(nx).standard_normal((ny, nx))
    ds = 0.8
    g = grid(nx, ny, ds)
    out = torch.empty((ny, nx), dtype=torch.float64, device=DEV)
    g.jacobian_apply_t(gpu(u), gpu(mu), out)
    ref = orc.jacobian_apply_t(orc.Model(), u, mu, ds)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("nx,ny", [(8, 6), (67, 130)])
def test_jacobian_transpose_dot_product(orc, nx, ny):
    """<w, J_D v> (oracle forward Jacobian) = <J_D^T w, v> (GPU transposed apply): ties the
    GPU gather form to the forward operator, not only to the oracle's own transpose."""
    u = synth.noise_film(nx, ny, seed=3 * nx + ny, amp=0.2)
    rng = np.random.default_rng(nx * ny)
    v, w = rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx))
    ds = 0.7
    g = grid(nx, ny, ds)
    jtw = torch.empty((ny, nx), dtype=torch.float64, device=DEV)
    g.jacobian_apply_t(gpu(u), gpu(w), jtw)
    jv = orc.jacobian_apply(orc.Model(), u, v, ds)
    jt = jtw.cpu().numpy()
    lhs, rhs = float(np.sum(w * jv)), float(np.sum(jt * v))
    scale = float(np.sum(np.abs(w * jv)) + np.sum(np.abs(jt * v)))
    assert abs(lhs - rhs) <= 1e-12 * scale


def _bands(n, nl, seed, dominant=True):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((5, n, nl))
    if dominant:
        b[2] = 6.0 + rng.random((n, nl))
    for p in range(n):
        for o in range(5):
            if not 0 <= p + o - 2 < n:
                b[o, p, :] = 0.0
    return b


@pytest.mark.parametrize("n,nl", [(2, 3), (5, 7), (64, 64), (65, 130), (200, 33), (1000, 5), (2047, 3), (4096, 2)])
@pytest.mark.parametrize("transposed", [False, True])
@pytest.mark.parametrize("variant", ["partitioned", "thomas", "pcr", "line"])
def test_penta_solve_matches_oracle(orc, n, nl, transposed, variant):
    b = _bands(n, nl, seed=n * 7 + nl)
    rhs = np.random.default_rng(n + nl).standard_normal((n, nl))
    x = torch.empty((n, nl), dtype=torch.float64, device=DEV)
    if (variant == "line" and n < 4) or (variant == "pcr" and n > 2048):
        # outside the variant's range of line lengths: refused before any launch
        with pytest.raises(TFError):
            penta_solve(gpu(b), gpu(rhs), x, transposed=transposed, variant=variant)
        return
    penta_solve(gpu(b), gpu(rhs), x, transposed=transposed, variant=variant)
    got = x.cpu().numpy()
    for l in range(nl):
        band = np.ascontiguousarray(b[:, :, l])
        if transposed:
            band = orc.band_transpose(band)
        ref = orc.band_solve(band, rhs[:, l])
        assert np.max(np.abs(got[:, l] - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref))), l


@pytest.mark.parametrize("variant", ["partitioned", "thomas", "pcr", "line"])
def test_transposed_solve_dot_product(variant):
    """<w, A^-1 r> = <A^-T w, r> with both solves on the GPU (plain and transposed)."""
    n, nl = 130, 70
    b = gpu(_bands(n, nl, seed=11))
    rng = np.random.default_rng(12)
    r, w = rng.standard_normal((n, nl)), rng.standard_normal((n, nl))
    x = torch.empty((n, nl), dtype=torch.float64, device=DEV)
    y = torch.empty_like(x)
    penta_solve(b, gpu(r), x, transposed=False, variant=variant)
    penta_solve(b, gpu(w), y, transposed=True, variant=variant)
    xs, ys = x.cpu().numpy(), y.cpu().numpy()
    lhs, rhs = np.sum(w * xs, axis=0), np.sum(ys * r, axis=0)
    scale = np.sum(np.abs(w * xs), axis=0) + np.sum(np.abs(ys * r), axis=0)
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * scale)


@pytest.mark.parametrize("variant", ["partitioned", "thomas", "pcr", "line"])
def test_penta_solve_on_model_bands(orc, variant):
    """Real (I + c J_x) systems of a noisy film (not diagonally dominant)."""
    nx, ny = 300, 40
    u = synth.noise_film(nx, ny, seed=5, amp=0.01)
    M = orc.Model()
    b = np.stack([orc.bands_x(M, u, 0.67347, 0.2, j) for j in range(ny)], axis=2)  # (5, nx, ny)
    rhs = np.random.default_rng(1).standard_normal((nx, ny))
    x = torch.empty((nx, ny), dtype=torch.float64, device=DEV)
    penta_solve(gpu(b), gpu(rhs), x, variant=variant)
    got = x.cpu().numpy()
    for j in range(ny):
        ref = orc.band_solve(np.ascontiguousarray(b[:, :, j]), rhs[:, j])
        assert np.max(np.abs(got[:, j] - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_adjoint_step_matches_oracle(orc, theta):
    nx, ny, ds, dt = 40, 30, 0.67347, 0.1
    un = synth.noise_film(nx, ny, seed=2, amp=0.01)
    M = orc.Model()
    unp1, res = orc.step(M, orc.Scheme(theta=theta, tol=1e-14), un, ds, dt)
    assert res.status == orc.OK
    lam = np.random.default_rng(3).standard_normal((ny, nx))
    ref, gk_ref, _ = orc.adjoint_step(M, un, unp1, lam, ds, dt, theta, tol=1e-14)
    g = grid(nx, ny, ds, theta=theta)
    lg = gpu(lam)
    gk, it = g.adjoint_step(gpu(un), gpu(unp1), dt, lg, tol=1e-14)
    got = lg.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert gk == pytest.approx(gk_ref, rel=1e-9)


@pytest.mark.parametrize("xsweep", ["partitioned", "row"])
@pytest.mark.parametrize("nx,ny", [(37, 23), (130, 67), (300, 41), (1030, 9)])
def test_adjoint_x_solve_variants_match_oracle(orc, xsweep, nx, ny):
    """The adjoint's transposed row solves take the grid's x-sweep variant: whole rows in one
    kernel (rows whose first sub-segment is ragged, several rows per workgroup, up to 4
    waves per row) or the partitioned solver. One adjoint step of each against the oracle."""
    ds, dt = 0.67347, 0.1
    un = synth.noise_film(nx, ny, seed=12, amp=0.01)
    M = orc.Model()
    unp1, res = orc.step(M, orc.Scheme(tol=1e-14), un, ds, dt)
    assert res.status == orc.OK
    lam = np.random.default_rng(13).standard_normal((ny, nx))
    ref, gk_ref, _ = orc.adjoint_step(M, un, unp1, lam, ds, dt, 1.0, tol=1e-14)
    g = grid(nx, ny, ds)
    g.set_xsweep(xsweep)
    assert g.xsweep() == xsweep
    lg = gpu(lam)
    gk, _ = g.adjoint_step(gpu(un), gpu(unp1), dt, lg, tol=1e-14)
    assert np.max(np.abs(lg.cpu().numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert gk == pytest.approx(gk_ref, rel=1e-9)


def _loss(h, target):
    return 0.5 * torch.sum((h - target) ** 2)


def test_rollout_gradient_matches_finite_differences():
    """32 x 32 film, 10 backward-Euler steps (forward tol 1e-14): the checkpointed
    adjoint gradient in p0 and kappa matches central differences."""
    n, steps, dt = 32, 10, 0.1
    ds = 16 * synth.lambda_m(10.0) / 512  # the 512^2 adjoint case's cell size
    base = gpu(synth.noise_film(n, n, seed=4, amp=0.01))
    target = gpu(synth.noise_film(n, n, seed=5, amp=0.01))
    p0 = torch.zeros((n, n), dtype=torch.float64, device=DEV, requires_grad=True)
    kap = torch.tensor(10.0, dtype=torch.float64, device=DEV, requires_grad=True)
    h = rollout(p0, kap, base, steps, dt, ds, checkpoint_every=4, tol=1e-14, adj_tol=1e-14)
    L = _loss(h, target)
    L.backward()
    d = gpu(np.random.default_rng(7).standard_normal((n, n)))
    eps = 1e-5
    with torch.no_grad():
        Lp = _loss(rollout(p0 + eps * d, kap, base, steps, dt, ds, tol=1e-14), target).item()
        Lm = _loss(rollout(p0 - eps * d, kap, base, steps, dt, ds, tol=1e-14), target).item()
        fd = (Lp - Lm) / (2 * eps)
        assert torch.sum(p0.grad * d).item() == pytest.approx(fd, rel=1e-6)
        ek = 1e-5
        Lp = _loss(rollout(p0, kap + ek, base, steps, dt, ds, tol=1e-14), target).item()
        Lm = _loss(rollout(p0, kap - ek, base, steps, dt, ds, tol=1e-14), target).item()
        assert kap.grad.item() == pytest.approx((Lp - Lm) / (2 * ek), rel=1e-6)


def test_rollout_gradient_matches_oracle_adjoint(orc):
    """Same rollout: GPU gradient vs the oracle's forward + adjoint chain, 1e-8 relative."""
    n, steps, dt = 32, 10, 0.1
    ds = 16 * synth.lambda_m(10.0) / 512
    b_np = synth.noise_film(n, n, seed=4, amp=0.01)
    t_np = synth.noise_film(n, n, seed=5, amp=0.01)
    p0 = torch.zeros((n, n), dtype=torch.float64, device=DEV, requires_grad=True)
    kap = torch.tensor(10.0, dtype=torch.float64, device=DEV, requires_grad=True)
    h = rollout(p0, kap, gpu(b_np), steps, dt, ds, checkpoint_every=3, tol=1e-14, adj_tol=1e-14)
    _loss(h, gpu(t_np)).backward()
    M = orc.Model()
    traj = [b_np]
    u = b_np
    for _ in range(steps):
        u, res = orc.step(M, orc.Scheme(tol=1e-14), u, ds, dt)
        traj.append(u)
    lam = traj[-1] - t_np
    gk = 0.0
    for s in range(steps - 1, -1, -1):
        lam, c, _ = orc.adjoint_step(M, traj[s], traj[s + 1], lam, ds, dt, 1.0, tol=1e-14)
        gk += c
    g = p0.grad.cpu().numpy()
    assert np.max(np.abs(g - lam)) <= 1e-8 * np.max(np.abs(lam))
    assert kap.grad.item() == pytest.approx(gk, rel=1e-8)


def test_advance_keep_and_adjoint_steps_match_single_steps():
    """tf_advance_keep keeps exactly the states that single tf_step calls reach, and
    tf_adjoint_steps over the stretch equals tf_adjoint_step newest first (lambda bit for bit,
    the summed dL/dkappa to rounding)."""
    n, steps, dt = 48, 7, 0.1
    ds = 16 * synth.lambda_m(10.0) / 512
    b = gpu(synth.noise_film(n, n, seed=4, amp=0.01))
    g = grid(n, n, ds, tol=1e-12)
    h = b.clone()
    g.bind(h)
    ref = [h.clone()]
    for _ in range(steps):
        g.step(dt)
        ref.append(h.clone())
    states = torch.empty((steps + 1, n, n), dtype=torch.float64, device=DEV)
    states[0].copy_(b)
    h2 = b.clone()
    g.bind(h2)
    g.advance_keep(steps, dt, states[1:])
    for s in range(steps + 1):
        assert torch.equal(states[s], ref[s]), s
    assert torch.equal(h2, ref[-1])
    lam0 = gpu(np.random.default_rng(9).standard_normal((n, n)))
    lam1 = lam0.clone()
    gk1, it1 = 0.0, 0
    for s in range(steps - 1, -1, -1):
        c, it = g.adjoint_step(ref[s], ref[s + 1], dt, lam1, tol=1e-12)
        gk1 += c
        it1 += it
    lam2 = lam0.clone()
    gk2, it2 = g.adjoint_steps(states, dt, lam2, tol=1e-12)
    assert torch.equal(lam1, lam2) and it1 == it2
    assert gk2 == pytest.approx(gk1, rel=1e-13, abs=1e-300)


def test_rollout_on_a_side_stream_matches_default_stream():
    """A rollout run under another torch stream uses a grid bound to that stream (the grid
    cache is keyed by stream), so its checkpoint copies and the library's launches stay in
    order: same h(T) and gradients, bit for bit, as on the default stream."""
    n, steps, dt = 48, 12, 0.1
    ds = 16 * synth.lambda_m(10.0) / 512
    b = gpu(synth.noise_film(n, n, seed=4, amp=0.01))
    t = gpu(synth.noise_film(n, n, seed=5, amp=0.01))

    def run():
        p0 = torch.zeros((n, n), dtype=torch.float64, device=DEV, requires_grad=True)
        kap = torch.tensor(10.0, dtype=torch.float64, device=DEV, requires_grad=True)
        h = rollout(p0, kap, b, steps, dt, ds, checkpoint_every=4, tol=1e-12, adj_tol=1e-12)
        _loss(h, t).backward()
        return h.detach().clone(), p0.grad.clone(), kap.grad.clone()

    ref = run()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        got = run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for a, r in zip(got, ref):
        assert torch.equal(a, r)


@pytest.fixture(scope="module")
def adjoint512_step(orc):
    """u^n (the seed-4 film of the 512^2 adjoint workload), the oracle's u^{n+1} after one
    backward-Euler step of dt = 0.1, a random lambda^{n+1} and the oracle's adjoint step."""
    cfg = synth.CONFIGS["adjoint512"]
    un = synth.noise_film(cfg.n, cfg.n, cfg.seed, 1.0, 0.01)
    M = orc.Model()
    unp1, res = orc.step(M, orc.Scheme(tol=1e-13), un, cfg.ds, cfg.dt)
    assert res.status == orc.OK
    lam = np.random.default_rng(21).standard_normal((cfg.n, cfg.n))
    ref, gk_ref, _ = orc.adjoint_step(M, un, unp1, lam, cfg.ds, cfg.dt, 1.0, tol=1e-13)
    return un, unp1, lam, ref, gk_ref


@pytest.mark.parametrize("xsweep", ["row", "partitioned"])
def test_512_adjoint_step_matches_oracle(adjoint512_step, xsweep):
    """One adjoint step at the full size of the 512^2 adjoint workload (L = 16 lambda_m),
    on the solver variants its timed run uses (whole-row transposed row solves and the tuned
    column solves) and on the partitioned ones: lambda^n and the dL/dkappa contribution
    against the oracle's adjoint step from the same u^n, u^{n+1} and lambda^{n+1}."""
    un, unp1, lam, ref, gk_ref = adjoint512_step
    cfg = synth.CONFIGS["adjoint512"]
    n, ds, dt = cfg.n, cfg.ds, cfg.dt
    g = grid(n, n, ds)
    g.set_xsweep(xsweep)
    lg = gpu(lam)
    gk, _ = g.adjoint_step(gpu(un), gpu(unp1), dt, lg, tol=1e-13)
    assert np.max(np.abs(lg.cpu().numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert gk == pytest.approx(gk_ref, rel=1e-9)


def test_512_adjoint_batched_richardson_iterations(adjoint512_step):
    """At 512^2 both transposed solves are whole-line kernels, so the Richardson iterations
    run in batches whose launches test the previous iteration on the device. The result and
    the iteration count do not depend on the batch size the grid's previous step left; a limit
    of exactly the iterations needed converges to the same result, one fewer fails with
    TF_ENOCONV, and a NaN in lambda is reported as TF_ENONPOS."""
    import os
    import paper_1806_10550_amd as pkg
    from paper_1806_10550_amd.lib import TF_ENOCONV, TF_ENONPOS
    autotune_load(os.path.join(os.path.dirname(pkg.__file__), "autotune_gfx950.jsonl"))
    assert autotune_choice(512, 512, transposed=True) == "line"
    un, unp1, lam, ref, gk_ref = adjoint512_step
    cfg = synth.CONFIGS["adjoint512"]
    n, ds, dt = cfg.n, cfg.ds, cfg.dt
    g = grid(n, n, ds)
    g.set_xsweep("row")
    hn, hnp1 = gpu(un), gpu(unp1)

    def run(lam_in, **kw):
        lg = gpu(lam_in)
        gk, it = g.adjoint_step(hn, hnp1, dt, lg, **kw)
        return lg, gk, it

    l1, gk1, it1 = run(lam, tol=1e-13)      # first step of the grid: the smallest batch
    assert np.max(np.abs(l1.cpu().numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert gk1 == pytest.approx(gk_ref, rel=1e-9)
    assert it1 > 2
    l2, gk2, it2 = run(lam, tol=1e-13)      # batch sized from it1
    assert it2 == it1 and torch.equal(l2, l1) and gk2 == gk1
    _, _, it3 = run(lam, tol=1e-4)          # fewer iterations: a smaller next batch
    assert it3 < it1
    l4, gk4, it4 = run(lam, tol=1e-13)
    assert it4 == it1 and torch.equal(l4, l1) and gk4 == gk1
    l5, gk5, it5 = run(lam, tol=1e-13, max_iter=it1)
    assert it5 == it1 and torch.equal(l5, l1) and gk5 == gk1
    with pytest.raises(TFError) as e:
        run(lam, tol=1e-13, max_iter=it1 - 1)
    assert e.value.status == TF_ENOCONV
    bad = lam.copy()
    bad[7, 9] = np.nan
    with pytest.raises(TFError) as e:
        run(bad, tol=1e-13)
    assert e.value.status == TF_ENONPOS
    l6, gk6, it6 = run(lam, tol=1e-13)      # the grid recovers
    assert it6 == it1 and torch.equal(l6, l1) and gk6 == gk1


def test_full_size_rollout_gradient_matches_finite_differences():
    """The 512^2 adjoint workload as timed (L = 16 lambda_m, 400 backward-Euler steps of dt = 0.1,
    checkpoints every 20, p0 = 0 on the seed-4 film, target = the seed-5 film run forward over the
    same 400 steps, loss 0.5 ||h(T) - target||^2), with forward and adjoint tolerances 1e-12: the
    directional derivatives in p0 (random direction) and kappa match central differences with
    step 1e-4 to 1e-5 relative (differences of the loss carry the forward tolerance over the
    step, ~1e-8 relative; the truncation error is O(step^2))."""
    cfg = synth.CONFIGS["adjoint512"]
    n, dt, steps, ds, ck = cfg.n, cfg.dt, cfg.steps, cfg.ds, cfg.extra["checkpoint_every"]
    tol = 1e-12
    base = gpu(synth.noise_film(n, n, cfg.seed, 1.0, 0.01))
    tgt = gpu(synth.noise_film(n, n, cfg.extra["target_seed"], 1.0, 0.01))
    g = grid(n, n, ds, tol=tol, max_newton=5000)
    g.bind(tgt)
    g.advance(steps, dt)
    p0 = torch.zeros_like(base, requires_grad=True)
    kap = torch.tensor(cfg.kappa, dtype=torch.float64, device=DEV, requires_grad=True)
    h = rollout(p0, kap, base, steps, dt, ds, checkpoint_every=ck, tol=tol, adj_tol=tol)
    _loss(h, tgt).backward()
    d = gpu(np.random.default_rng(7).standard_normal((n, n)))
    eps = 1e-4
    with torch.no_grad():
        Lp = _loss(rollout(p0 + eps * d, kap, base, steps, dt, ds, tol=tol), tgt).item()
        Lm = _loss(rollout(p0 - eps * d, kap, base, steps, dt, ds, tol=tol), tgt).item()
        assert torch.sum(p0.grad * d).item() == pytest.approx((Lp - Lm) / (2 * eps), rel=1e-5)
        Lp = _loss(rollout(p0, kap + eps, base, steps, dt, ds, tol=tol), tgt).item()
        Lm = _loss(rollout(p0, kap - eps, base, steps, dt, ds, tol=tol), tgt).item()
        assert kap.grad.item() == pytest.approx((Lp - Lm) / (2 * eps), rel=1e-5)


def test_autotune_cache_roundtrip(tmp_path):
    path = str(tmp_path / "tune.jsonl")
    choice = autotune(512, 512, path)
    assert choice in ("partitioned", "thomas", "pcr", "line")
    rec = json.loads(open(path).read().strip().splitlines()[-1])
    assert rec["length"] == 512 and rec["batch"] == 512 and rec["variant"] == choice
    assert set(rec["ms"]) == {"partitioned", "thomas/64", "thomas/128", "thomas/256", "pcr", "line"}
    assert all(math.isfinite(v) for v in rec["ms"].values())
    best = min(rec["ms"], key=rec["ms"].get)
    assert best.split("/")[0] == choice
    if choice == "thomas":
        assert rec["block"] == int(best.split("/")[1])
    autotune_load(path)
    assert autotune_choice(512, 512) == choice
    # long lines: no cyclic reduction candidate; transposed solves are tuned separately
    ct = autotune(4096, 8, path, transposed=True)
    rec = json.loads(open(path).read().strip().splitlines()[-1])
    assert "pcr" not in rec["ms"] and "line" in rec["ms"] and rec["length"] == 4096 and rec["transposed"] == 1
    assert autotune_choice(4096, 8, transposed=True) == ct
    # beyond 4096 cells the whole-line kernel is no candidate either
    autotune(4100, 4, path, transposed=True)
    rec = json.loads(open(path).read().strip().splitlines()[-1])
    assert set(rec["ms"]) == {"partitioned", "thomas/64", "thomas/128", "thomas/256"}


def test_pcr_rejects_long_lines():
    n, nl = 2050, 2
    b = gpu(_bands(n, nl, seed=1))
    rhs = gpu(np.ones((n, nl)))
    x = torch.empty((n, nl), dtype=torch.float64, device=DEV)
    with pytest.raises(Exception):
        penta_solve(b, rhs, x, variant="pcr")


@pytest.mark.parametrize("model,theta", [("power", 0.5), ("nlc", 1.0), ("nlc", 0.5), ("polymer", 0.5)])
def test_rollout_other_models_and_theta_match_finite_differences(model, theta):
    """Checkpointed rollouts with the trapezoidal rule and with the NLC / polymer models
    (which have no kappa: gradient in p0 only): the adjoint gradient matches central
    differences of the loss (24 x 24 film, 8 steps, forward tolerance 1e-14)."""
    import math
    n, steps = 24, 8
    if model == "power":
        h0, ds, dt = 1.0, 16 * synth.lambda_m(10.0) / 512, 0.1
    elif model == "nlc":
        h0, ds, dt = 0.5, 2 * math.pi / 1.482 / 16, 0.5
    else:
        h0, ds, dt = 3.9, 2 * math.pi / 1.5599 / 16, 0.01
    base = gpu(synth.noise_film(n, n, seed=8, h0=h0, amp=0.01 * h0))
    target = gpu(synth.noise_film(n, n, seed=9, h0=h0, amp=0.01 * h0))
    p0 = torch.zeros((n, n), dtype=torch.float64, device=DEV, requires_grad=True)
    kap = torch.tensor(10.0, dtype=torch.float64, device=DEV, requires_grad=True) if model == "power" else None
    kw = dict(checkpoint_every=3, tol=1e-14, adj_tol=1e-14, theta=theta, model=model)
    L = _loss(rollout(p0, kap, base, steps, dt, ds, **kw), target)
    L.backward()
    d = gpu(np.random.default_rng(10).standard_normal((n, n)))
    eps = 1e-5 * h0
    with torch.no_grad():
        Lp = _loss(rollout(p0 + eps * d, kap, base, steps, dt, ds, **kw), target).item()
        Lm = _loss(rollout(p0 - eps * d, kap, base, steps, dt, ds, **kw), target).item()
        assert torch.sum(p0.grad * d).item() == pytest.approx((Lp - Lm) / (2 * eps), rel=1e-6)
        if model == "power":
            ek = 1e-5
            Lp = _loss(rollout(p0, kap + ek, base, steps, dt, ds, **kw), target).item()
            Lm = _loss(rollout(p0, kap - ek, base, steps, dt, ds, **kw), target).item()
            assert kap.grad.item() == pytest.approx((Lp - Lm) / (2 * ek), rel=1e-6)


def test_adjoint_step_general_power_law_matches_oracle(orc):
    """Exponents n = 5, m = 2 (the general power-law adjoint kernels): one adjoint step and
    its dL/dkappa contribution against the oracle, and J_D^T against the oracle's transpose."""
    nx, ny, ds, dt = 40, 30, 0.67347, 0.1
    M = orc.Model(kappa=10.0, b=0.1, n=5.0, m=2.0)
    un = synth.noise_film(nx, ny, seed=8, amp=0.01)
    unp1, res = orc.step(M, orc.Scheme(theta=1.0, tol=1e-14), un, ds, dt)
    assert res.status == orc.OK
    lam = np.random.default_rng(9).standard_normal((ny, nx))
    ref, gk_ref, _ = orc.adjoint_step(M, un, unp1, lam, ds, dt, 1.0, tol=1e-14)
    g = Grid(nx, ny, ds)
    g.set_model(10.0, 0.1, 5, 2)
    g.set_scheme(theta=1.0)
    out = torch.empty((ny, nx), dtype=torch.float64, device=DEV)
    g.jacobian_apply_t(gpu(unp1), gpu(lam), out)
    jt_ref = orc.jacobian_apply_t(M, unp1, lam, ds)
    assert np.max(np.abs(out.cpu().numpy() - jt_ref)) <= 1e-12 * np.max(np.abs(jt_ref))
    lg = gpu(lam)
    gk, _ = g.adjoint_step(gpu(un), gpu(unp1), dt, lg, tol=1e-14)
    assert np.max(np.abs(lg.cpu().numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert gk == pytest.approx(gk_ref, rel=1e-9)


def test_autotune_xsweep_roundtrip(tmp_path):
    """Forward x-sweep tuning: both variants timed on a 2500-cell row film, the faster one
    recorded (kind "xsweep") and taken for that shape by new grids; rows above 4096 cells
    always take the partitioned solver whatever the timing."""
    from paper_1806_10550_amd.lib import autotune_xsweep, xsweep_choice
    path = str(tmp_path / "xs.jsonl")
    choice = autotune_xsweep(2500, 4, path)
    rec = json.loads(open(path).read().strip().splitlines()[-1])
    assert rec["kind"] == "xsweep" and rec["length"] == 2500 and rec["batch"] == 4
    assert set(rec["ms"]) == {"partitioned", "row"} and all(math.isfinite(v) for v in rec["ms"].values())
    assert rec["variant"] == min(rec["ms"], key=rec["ms"].get) == choice
    assert xsweep_choice(2500, 4) == choice
    g = grid(2500, 4, 0.67)
    assert g.xsweep() == choice
    g.close()
    autotune_xsweep(8000, 4, path)
    assert xsweep_choice(8000, 4) == "partitioned"
    autotune_load(path)
    assert xsweep_choice(2500, 4) == choice
