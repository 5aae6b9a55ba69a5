"""Ensemble path (packed ragged films, device-side control, captured graph) against the
single-film GPU path (bit for bit: same kernels, same arithmetic) and the CPU oracle."""
import numpy as np
import pytest
import torch

from paper_1806_10550_amd import synth
from paper_1806_10550_amd.lib import Ensemble, Grid, TF_ENONPOS, TF_ENOCONV, TF_OK

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

FILMS = [(70, 66, 5.0), (64, 64, 10.0), (130, 40, 20.0), (200, 129, 8.0), (96, 96, 15.0), (4, 9, 12.0)]


def films_setup(films, amp=0.01):
    nx = [f[0] for f in films]
    ny = [f[1] for f in films]
    kap = [f[2] for f in films]
    ds = [8 * synth.lambda_m(k) / n for n, _, k in films]
    h0 = [synth.noise_film(a, b, seed=100 + i, amp=amp) for i, (a, b, _) in enumerate(films)]
    return nx, ny, kap, ds, h0


def pack(ens, h0):
    packed = torch.empty(ens.size, dtype=torch.float64, device=DEV)
    for f, h in enumerate(h0):
        ens.view(packed, f).copy_(torch.from_numpy(h))
    return packed


def single(nx, ny, ds, kappa, h0, steps, dt, xsweep="auto", **scheme):
    g = Grid(nx, ny, ds)
    g.set_model(kappa, 0.1, 3, 2)
    g.set_scheme(**scheme)
    g.set_xsweep(xsweep)
    h = torch.from_numpy(h0).to(DEV)
    g.bind(h)
    st, dtn, log = g.try_advance(steps, dt)
    return st, dtn, log, h


def test_ensemble_equals_single_film_path_bitwise():
    nx, ny, kap, ds, h0 = films_setup(FILMS)
    ens = Ensemble(nx, ny, ds, kap)
    ens.set_scheme(tol=1e-10)
    packed = pack(ens, h0)
    ens.bind(packed)
    st, dts, sts, its = ens.step(4, 0.1)
    assert st == TF_OK and all(s == TF_OK for s in sts)
    for f in range(len(FILMS)):
        s1, _, log, h = single(nx[f], ny[f], ds[f], kap[f], h0[f], 4, 0.1, xsweep=ens.xsweep(f), tol=1e-10)
        assert s1 == TF_OK
        assert torch.equal(ens.view(packed, f), h), f
        assert its[f] == sum(x["total_iters"] for x in log)


def test_ensemble_matches_oracle(orc):
    nx, ny, kap, ds, h0 = films_setup(FILMS[:4])
    ens = Ensemble(nx, ny, ds, kap)
    packed = pack(ens, h0)
    ens.bind(packed)
    st, _, sts, _ = ens.step(3, 0.1)
    assert st == TF_OK
    for f in range(4):
        M = orc.Model(kappa=kap[f], b=0.1, n=3.0, m=2.0)
        u = h0[f]
        for _ in range(3):
            u, res = orc.step(M, orc.Scheme(tol=1e-10), u, ds[f], 0.1)
            assert res.status == orc.OK
        got = ens.view(packed, f).cpu().numpy()
        assert np.max(np.abs(got - u) / u) <= 1e-10


def test_ensemble_failure_is_isolated():
    nx, ny, kap, ds, h0 = films_setup(FILMS[:3])
    h0[1] = h0[1].copy()
    h0[1][3, 3] = -0.2
    ens = Ensemble(nx, ny, ds, kap)
    packed = pack(ens, h0)
    ens.bind(packed)
    st, _, sts, _ = ens.step(2, 0.1)
    assert st == TF_ENONPOS
    assert sts == [TF_OK, TF_ENONPOS, TF_OK]
    assert torch.equal(ens.view(packed, 1).cpu(), torch.from_numpy(h0[1]))
    # a fixed-dt film that cannot converge within max_newton fails alone
    ens2 = Ensemble(nx, ny, ds, kap)
    ens2.set_scheme(max_newton=1, tol=1e-14)
    h1 = films_setup(FILMS[:3])[4]
    p2 = pack(ens2, h1)
    ens2.bind(p2)
    st, _, sts, _ = ens2.step(1, 0.1)
    assert st == TF_ENOCONV and all(s == TF_ENOCONV for s in sts)
    for f in range(3):
        assert torch.equal(ens2.view(p2, f).cpu(), torch.from_numpy(h1[f]))


def test_ensemble_adaptive_schedules_match_single_films():
    nx, ny, kap, ds, h0 = films_setup(FILMS[:5])
    kw = dict(tol=1e-10, max_newton=10, adaptive=1, dt_min=1e-6, dt_max=1.0, dt_shrink=0.5, dt_grow=1.1,
              grow_after=5)
    ens = Ensemble(nx, ny, ds, kap)
    ens.set_scheme(**kw)
    packed = pack(ens, h0)
    ens.bind(packed)
    dts = [0.1] * 5
    for _ in range(3):
        st, dts, sts, its = ens.step(4, dts)
        assert st == TF_OK
    for f in range(5):
        s1, dtn, log, h = single(nx[f], ny[f], ds[f], kap[f], h0[f], 12, 0.1, xsweep=ens.xsweep(f), **kw)
        assert s1 == TF_OK
        assert dts[f] == dtn
        assert torch.equal(ens.view(packed, f), h), f


@pytest.mark.parametrize("kind,h0s,dt", [("nlc", (0.3, 0.5, 0.7), 0.05), ("polymer", (3.0, 3.9, 5.0), 1e-3)])
def test_model_ensemble_equals_single_film_path_bitwise(orc, kind, h0s, dt):
    """Films of the NLC or polymer model with different sizes and thicknesses H0 (each on
    8 of its own most unstable wavelengths) advance in one ensemble exactly as one by one."""
    import math
    sizes = [(70, 66), (130, 40), (96, 97)]
    M = getattr(orc.Model, kind)()
    nx, ny, ds, h0 = [], [], [], []
    for i, ((a, b), H) in enumerate(zip(sizes, h0s)):
        f0, _, f1, _ = orc.coeffs(M, H)
        lam = 2 * math.pi / math.sqrt(f1 / (2 * f0))
        nx.append(a)
        ny.append(b)
        ds.append(8 * lam / a)
        h0.append(synth.noise_film(a, b, seed=300 + i, h0=H, amp=0.01 * H))
    ens = Ensemble(nx, ny, ds, [1.0] * len(sizes))
    getattr(ens, "set_model_" + kind)()
    ens.set_scheme(tol=1e-10)
    packed = pack(ens, h0)
    ens.bind(packed)
    st, dts, sts, its = ens.step(3, dt)
    assert st == TF_OK and all(s == TF_OK for s in sts)
    for f in range(len(sizes)):
        g = Grid(nx[f], ny[f], ds[f])
        g.set_xsweep(ens.xsweep(f))  # the variant the ensemble gives this film
        getattr(g, "set_model_" + kind)()
        g.set_scheme(tol=1e-10)
        h = torch.from_numpy(h0[f]).to(DEV)
        g.bind(h)
        s1, _, log = g.try_advance(3, dt)
        assert s1 == TF_OK
        assert torch.equal(ens.view(packed, f), h), f
        assert its[f] == sum(x["total_iters"] for x in log)


def test_model_ensemble_rejects_bad_parameters():
    from paper_1806_10550_amd.lib import TFError
    ens = Ensemble([64], [64], [0.5], [10.0])
    with pytest.raises(TFError):
        ens.set_model_nlc(w=0.0)
    with pytest.raises(TFError):
        ens.set_model_polymer(C=-1.0)
    with pytest.raises(TFError):
        ens.set_model_linear(c0=0.0)


@pytest.mark.parametrize("adaptive,dt0", [(0, 0.1), (1, 2.0)])
def test_theta_half_ensemble_equals_single_film_path_bitwise(adaptive, dt0):
    """The trapezoidal rule (theta = 1/2, eq. TrapRule) in the ensemble: b^n is formed on the
    device at the first iteration of each attempt; with adaptive steps from dt = 2 the films
    reject and retry with smaller dt. Every film ends bit for bit where it ends alone, with the
    same dt and iteration count."""
    nx, ny, kap, ds, h0 = films_setup(FILMS[:5])
    kw = dict(theta=0.5, tol=1e-10, max_newton=10 if adaptive else 5000, adaptive=adaptive, dt_min=1e-6,
              dt_max=4.0, dt_shrink=0.5, dt_grow=1.1, grow_after=5)
    ens = Ensemble(nx, ny, ds, kap)
    ens.set_scheme(**kw)
    packed = pack(ens, h0)
    ens.bind(packed)
    st, dts, sts, its = ens.step(6, dt0)
    assert st == TF_OK and all(s == TF_OK for s in sts)
    rejected = 0
    for f in range(5):
        s1, dtn, log, h = single(nx[f], ny[f], ds[f], kap[f], h0[f], 6, dt0, xsweep=ens.xsweep(f), **kw)
        assert s1 == TF_OK
        assert dts[f] == dtn
        assert its[f] == sum(x["total_iters"] for x in log)
        assert torch.equal(ens.view(packed, f), h), f
        rejected += sum(x["rejections"] for x in log)
    if adaptive:
        assert rejected > 0  # the retry path (b^n recomputed with the shrunk dt) was exercised


def test_full_ensemble_matches_oracle_on_sampled_films(orc):
    """The 256-film ensemble as timed (sizes {256..1024}^2, kappa ~ U[5, 20], L = 8 lambda_m,
    noise 0.01 from default_rng(3); adaptive dt from 0.1, K = 10, tol 1e-10): after 3 steps,
    8 films drawn by a seeded generator agree with the oracle's own adaptive run of the same
    film to 1e-10 relative, with the same next dt."""
    films = synth.ensemble_films(256)
    nx = [f.n for f in films]
    ds = [f.ds for f in films]
    kap = [f.kappa for f in films]
    h0 = [synth.noise_film(f.n, f.n, f.seed, 1.0, 0.01) for f in films]
    scheme = dict(tol=1e-10, max_newton=10, adaptive=1, dt_min=1e-9, dt_max=1.0, dt_shrink=0.5, dt_grow=1.1,
                  grow_after=5)
    ens = Ensemble(nx, nx, ds, kap)
    ens.set_scheme(**scheme)
    packed = pack(ens, h0)
    ens.bind(packed)
    st, dts, sts, _ = ens.step(3, [0.1] * len(films))
    assert st == TF_OK and all(s == TF_OK for s in sts)
    pick = np.random.default_rng(11).choice(len(films), 8, replace=False)
    S = orc.Scheme(theta=1.0, **scheme)
    for f in pick:
        M = orc.Model(kappa=kap[f], b=0.1, n=3.0, m=2.0)
        u, dt, succ = h0[f], 0.1, 0
        for _ in range(3):
            u, res = orc.step(M, S, u, ds[f], dt, succ)
            assert res.status == orc.OK
            dt, succ = res.dt_next, res.successes
        got = ens.view(packed, int(f)).cpu().numpy()
        assert np.max(np.abs(got - u) / u) <= 1e-10, f
        assert dts[f] == dt, f


def test_general_power_law_ensemble_equals_single_film_path_bitwise():
    """Exponents n = 5, m = 2 (the general power-law instantiation of the ensemble passes):
    every film equals its single-film run bit for bit."""
    nx, ny, kap, ds, h0 = films_setup(FILMS)
    ens = Ensemble(nx, ny, ds, kap, b=0.1, n=5, m=2)
    ens.set_scheme(tol=1e-10)
    packed = pack(ens, h0)
    ens.bind(packed)
    st, _, sts, its = ens.step(3, 0.1)
    assert st == TF_OK and all(s == TF_OK for s in sts)
    for f in range(len(FILMS)):
        g = Grid(nx[f], ny[f], ds[f])
        g.set_xsweep(ens.xsweep(f))  # the variant the ensemble gives this film
        g.set_model(kap[f], 0.1, 5, 2)
        g.set_scheme(tol=1e-10)
        h = torch.from_numpy(h0[f]).to(DEV)
        g.bind(h)
        s1, _, log = g.try_advance(3, 0.1)
        assert s1 == TF_OK
        assert torch.equal(ens.view(packed, f), h), f
        assert its[f] == sum(x["total_iters"] for x in log)


def test_film_info_matches_single_film_log():
    """tf_ensemble_film_info after a call: time, last dt, Newton iterations and update ratio
    of each film's last step equal the single-film path's log of the same steps."""
    nx, ny, kap, ds, h0 = films_setup(FILMS[:4])
    kw = dict(tol=1e-10, max_newton=10, adaptive=1, dt_min=1e-6, dt_max=1.0, dt_shrink=0.5, dt_grow=1.1,
              grow_after=2)
    ens = Ensemble(nx, ny, ds, kap)
    ens.set_scheme(**kw)
    packed = pack(ens, h0)
    ens.bind(packed)
    st, _, _, _ = ens.step(5, 0.5)
    assert st == TF_OK
    for f in range(4):
        s1, _, log, _ = single(nx[f], ny[f], ds[f], kap[f], h0[f], 5, 0.5, xsweep=ens.xsweep(f), **kw)
        assert s1 == TF_OK
        info = ens.film_info(f)
        last = log[-1]
        assert info["t"] == last["t"] and info["dt_used"] == last["dt_used"], f
        assert info["newton_iters"] == last["newton_iters"] and info["e_final"] == last["e_final"], f
        assert info["status"] == TF_OK


def test_scheme_round_trip():
    g = Grid(16, 12, 0.5)
    kw = dict(theta=0.5, tol=3e-11, max_newton=17, adaptive=1, dt_min=1e-7, dt_max=2.5, dt_shrink=0.25,
              dt_grow=1.3, grow_after=4)
    g.set_scheme(**kw)
    s = g.scheme()
    for k, v in kw.items():
        assert getattr(s, k) == v, k


def test_random_ragged_ensemble_equals_single_films_bitwise():
    """Twelve seeded random films (4..299 cells a side, kappa in [5, 20]) in one ensemble,
    adaptive dt: each film equals its single-film run bit for bit, with the same iterations."""
    rng = np.random.default_rng(77)
    films = [(int(rng.integers(4, 300)), int(rng.integers(4, 300)), float(rng.uniform(5.0, 20.0)))
             for _ in range(12)]
    nx, ny, kap, ds, h0 = films_setup(films)
    kw = dict(tol=1e-10, max_newton=10, adaptive=1, dt_min=1e-9, dt_max=1.0, dt_shrink=0.5, dt_grow=1.1,
              grow_after=2)
    ens = Ensemble(nx, ny, ds, kap)
    ens.set_scheme(**kw)
    packed = pack(ens, h0)
    ens.bind(packed)
    st, dts, sts, its = ens.step(4, 0.2)
    assert st == TF_OK and all(s == TF_OK for s in sts)
    for f in range(len(films)):
        s1, dtn, log, h = single(nx[f], ny[f], ds[f], kap[f], h0[f], 4, 0.2, xsweep=ens.xsweep(f), **kw)
        assert s1 == TF_OK
        assert torch.equal(ens.view(packed, f), h), films[f]
        assert its[f] == sum(x["total_iters"] for x in log) and dts[f] == dtn, films[f]


def test_mixed_xsweep_variants_bitwise():
    """Films whose x sweep takes different variants in one ensemble: rows above 4096 cells take
    the partitioned solver, shorter rows the whole-row kernel (each as it would alone; the
    per-film choice is reported by xsweep_choice). The ensemble equals the single-film path bit
    for bit, adaptive dt."""
    from paper_1806_10550_amd.lib import xsweep_choice
    films = [(4200, 12, 10.0), (500, 40, 8.0), (37, 23, 12.0), (3000, 9, 15.0), (64, 130, 6.0)]
    nx, ny, kap, ds, h0 = films_setup(films)
    kinds = [xsweep_choice(a, b) for a, b in zip(nx, ny)]
    assert kinds[0] == "partitioned" and "row" in kinds
    sch = dict(tol=1e-10, max_newton=10, adaptive=1, dt_min=1e-9, dt_max=1.0, dt_shrink=0.5, dt_grow=1.1,
               grow_after=5)
    ens = Ensemble(nx, ny, ds, kap)
    ens.set_scheme(**sch)
    packed = pack(ens, h0)
    ens.bind(packed)
    st, dts, sts, its = ens.step(3, 0.1)
    assert st == TF_OK
    for f in range(len(films)):
        s1, dtn, log, h = single(nx[f], ny[f], ds[f], kap[f], h0[f], 3, 0.1, xsweep=ens.xsweep(f), **sch)
        assert s1 == TF_OK
        assert torch.equal(ens.view(packed, f), h), (f, kinds[f])
        assert its[f] == sum(x["total_iters"] for x in log)
        assert dts[f] == dtn


@pytest.mark.parametrize("variant", ["row", "partitioned"])
def test_ensemble_forced_xsweep_bitwise(variant):
    """tf_ensemble_set_xsweep forces one variant on every film (rows above 4096 cells stay
    partitioned); each film equals a single film run with the same variant, bit for bit."""
    films = FILMS + [(4200, 8, 9.0)]
    nx, ny, kap, ds, h0 = films_setup(films)
    sch = dict(tol=1e-10, max_newton=10, adaptive=1, dt_min=1e-9, dt_max=1.0, dt_shrink=0.5, dt_grow=1.1,
               grow_after=5)  # the 4200-cell film (ds ~ 0.04) needs a much smaller dt
    ens = Ensemble(nx, ny, ds, kap)
    ens.set_scheme(**sch)
    ens.set_xsweep(variant)
    for f in range(len(films)):
        assert ens.xsweep(f) == (variant if nx[f] <= 4096 else "partitioned")
    packed = pack(ens, h0)
    ens.bind(packed)
    st, dts, sts, its = ens.step(3, 0.1)
    assert st == TF_OK
    for f in range(len(films)):
        s1, _, log, h = single(nx[f], ny[f], ds[f], kap[f], h0[f], 3, 0.1, xsweep=ens.xsweep(f), **sch)
        assert s1 == TF_OK
        assert torch.equal(ens.view(packed, f), h), (f, variant)
