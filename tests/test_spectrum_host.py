"""Steps 5-7 of the radial Fourier transform (tf_spectrum_maxima: least-squares
piecewise-linear fit, moving averages, maxima; App. "Radial Fourier Transform") run on the
host inside the library: compared with the oracle on noisy scatter data, plus its argument
checks. No GPU needed."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1806_10550_amd", "libthinfilm.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libthinfilm.so not built")


@pytest.mark.parametrize("npts,seed", [(5, 0), (57, 1), (400, 2), (1234, 3)])
def test_maxima_match_oracle(npts, seed):
    from oracle import radial as R
    from paper_1806_10550_amd.lib import spectrum_maxima
    rng = np.random.default_rng(seed)
    q = np.unique(rng.uniform(0.01, 6.0, npts))
    s = q ** 2 * np.exp(-q) + 0.3 * np.exp(-((q - 4.5) / 0.3) ** 2) + 0.01 * rng.normal(size=len(q))
    x, curve, peaks = spectrum_maxima(q, s, 6.0)
    t, a = R.piecewise_fit(q, s, 6.0)
    xo, co = R.smooth_curve(t, a, 6.0)
    po = R.local_maxima(xo, co)
    assert np.array_equal(x, xo)
    assert np.max(np.abs(curve - co)) <= 1e-12 * np.max(np.abs(co))
    assert len(peaks) == len(po)
    for (a1, b1), (a2, b2) in zip(peaks, po):
        assert a1 == pytest.approx(a2, rel=1e-12)
        assert b1 == pytest.approx(b2, rel=1e-11)


def test_maxima_argument_errors():
    from paper_1806_10550_amd.lib import TFError, spectrum_maxima
    q = np.linspace(0.1, 1.0, 20)
    with pytest.raises(TFError):
        spectrum_maxima(q[::-1], q, 2.0)        # not increasing
    with pytest.raises(TFError):
        spectrum_maxima(q, q, 0.5)              # beyond qmax
    with pytest.raises(TFError):
        spectrum_maxima(q, q * np.nan, 2.0)     # not finite
    with pytest.raises(TFError):
        q2 = np.linspace(0.01, 1.0, 100)
        spectrum_maxima(q2, np.exp(-((q2 - 0.5) / 0.1) ** 2), 1.0, capacity=0)  # one peak, no room
