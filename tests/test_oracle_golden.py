"""Oracle against values printed in the paper (fixtures under tests/golden/)."""
import math
import os

import numpy as np
import pytest

from paper_1806_10550_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


def test_linear_model_growth_rate_matches_printed_lsa(orc):
    """Sec. "Comparison to LSA": one wavelength lambda_m = 2 pi / q_m on I = J = 32
    cells, perturbed along x, run with the trapezoidal rule to T = log(1.3)/omega; the
    growth rate extracted from the simulation matches the printed omega_m = 1/4 at the
    printed q_m = 1/sqrt(2) (within the O(ds^2) discretisation error of 32 cells per
    wavelength)."""
    g = _read("lsa_linear_model.txt")
    M = orc.Model.linear(g["c0"], g["c1"])
    qm = g["q_m"]
    n = 32
    ds = (2 * math.pi / qm) / n
    amp = 1e-3
    u = synth.cosine_film(n, n, 2, 0, amp=amp)  # cos(q_m x) on [0, lambda_m]
    mode = (u - 1.0) / amp
    T = math.log(1.3) / g["omega_m"]
    steps = 200
    dt = T / steps
    for _ in range(steps):
        u, res = orc.step(M, orc.Scheme(theta=0.5, tol=1e-13), u, ds, dt)
        assert res.status == orc.OK
    a = np.sum((u - 1.0) * mode) / np.sum(mode * mode)
    rate = math.log(a / amp) / T
    assert rate == pytest.approx(g["omega_m"], rel=1e-2)
    # the discrete rate is the closed form q^2(c1 - c0 q^2) with q^2 -> mu(ds)
    mu = 4 / ds ** 2 * math.sin(math.pi * 2 / (2 * n)) ** 2
    assert rate == pytest.approx(mu * (g["c1"] - g["c0"] * mu), rel=1e-5)
