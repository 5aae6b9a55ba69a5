"""CPU oracle of the radial Fourier transform of a film (App. "Radial Fourier Transform").

TEST INFRASTRUCTURE ONLY: a plain NumPy FP64 statement of each step, used by the tests, the
smoke check and the benchmark's CPU baseline to check the GPU library. It shares no code with
the library.

Steps (readings of the appendix where it leaves details open):
  1. zeta = h - H0; |F(kx, ky)| = |DFT2(zeta)| / n^2 with F indexed by the signed integer
     wavenumbers kx, ky in [-n/2, n/2) (q = 2 pi k / L, L = n ds; square n x n grids).
  2. smooth |F| by a periodic convolution over (kx, ky) with the separable Gaussian weights
     w(d) = exp(-d^2 / (2 sigma^2)) / Z for |d| <= ceil(4 sigma) (sigma in wavenumber index
     units; sigma = 0 leaves |F| unchanged).
  3-4. average the smoothed values over the points of equal q_r (eq. FFT_radial_averaging):
     equal q_r means equal m = kx^2 + ky^2, so the groups are exact; the radial data are the
     points 0 < q_r <= qmax.
  5. least-squares fit of a continuous piecewise-linear function with value 0 at q = 0
     (eq. PiecewiseFunction): knots at q = 0, at every 10th data point, and at qmax, so
     that each interval holds 10 points (the last holds the remainder); unknowns: the values
     at the knots after q = 0.
  6. evaluate the fit at nfine = 400 equispaced points of [0, qmax] and apply moving averages
     of half widths 3, 2, 1 (windows truncated at the ends).
  7. local maxima: second-order differences for the derivative (one-sided at the ends), a
     root where it changes sign from + to - between two grid points, located by linear
     interpolation of the derivative; accepted when the second difference there is < 0.
"""
import math

import numpy as np


def spectrum_magnitude(h, h0):
    """Step 1: |DFT2(h - H0)| / n^2, in NumPy's FFT index order."""
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    assert h.shape == (n, n)
    return np.abs(np.fft.fft2(h - h0)) / (n * n)


def gaussian_weights(sigma):
    """Step 2 weights w(d), d = -R..R."""
    if sigma <= 0:
        return np.ones(1)
    R = int(math.ceil(4.0 * sigma))
    d = np.arange(-R, R + 1, dtype=np.float64)
    w = np.exp(-d * d / (2.0 * sigma * sigma))
    return w / np.sum(w)


def smooth(a, sigma):
    """Step 2: periodic separable convolution with gaussian_weights (explicit shifts)."""
    w = gaussian_weights(sigma)
    R = (len(w) - 1) // 2
    out = np.zeros_like(a)
    for i, wi in enumerate(w):
        out += wi * np.roll(a, i - R, axis=1)
    res = np.zeros_like(a)
    for i, wi in enumerate(w):
        res += wi * np.roll(out, i - R, axis=0)
    return res


def radial_average(s, L, qmax):
    """Steps 3-4: (q, mean, count) for each m = kx^2 + ky^2 with 0 < q <= qmax."""
    n = s.shape[0]
    k = np.fft.fftfreq(n, d=1.0 / n).astype(np.int64)
    m = k[None, :] ** 2 + k[:, None] ** 2
    M = int(math.floor((qmax * L / (2.0 * math.pi)) ** 2 * (1 + 1e-12)))
    M = min(M, int(m.max()))
    sums = np.bincount(m.ravel(), weights=s.ravel(), minlength=M + 1)[: M + 1]
    cnt = np.bincount(m.ravel(), minlength=M + 1)[: M + 1]
    ms = np.nonzero(cnt)[0]
    ms = ms[(ms > 0) & (2.0 * math.pi * np.sqrt(ms) / L <= qmax)]
    return 2.0 * math.pi * np.sqrt(ms) / L, sums[ms] / cnt[ms], cnt[ms]


def knots(q, qmax, per=10):
    """Step 5 knots: 0, q[per-1], q[2 per-1], ..., then qmax (the last interval takes the
    remainder, so it holds between per and 2 per - 1 points)."""
    N = len(q)
    K = max(1, N // per)
    return np.array([0.0] + [q[per * k - 1] for k in range(1, K)] + [qmax])


def hat_matrix(x, t):
    """Values at x of the hat functions of knots t[1:] (the knot t[0] = 0 is pinned to 0)."""
    A = np.zeros((len(x), len(t) - 1))
    for p, xv in enumerate(x):
        k = int(np.searchsorted(t, xv, side="right") - 1)
        k = min(max(k, 0), len(t) - 2)
        s = (xv - t[k]) / (t[k + 1] - t[k])
        if k >= 1:
            A[p, k - 1] += 1.0 - s
        A[p, k] += s
    return A


def piecewise_fit(q, y, qmax, per=10):
    """Step 5: knot positions and fitted knot values (value 0 at q = 0 included)."""
    t = knots(q, qmax, per)
    A = hat_matrix(q, t)
    a, *_ = np.linalg.lstsq(A, y, rcond=None)
    return t, np.concatenate([[0.0], a])


def moving_average(v, half):
    """One moving-average pass of half width `half` (window truncated at the ends)."""
    n = len(v)
    out = np.empty(n)
    for j in range(n):
        lo, hi = max(0, j - half), min(n, j + half + 1)
        out[j] = np.mean(v[lo:hi])
    return out


def smooth_curve(t, a, qmax, nfine=400):
    """Step 6: the fit on nfine equispaced points of [0, qmax], then half widths 3, 2, 1."""
    x = np.linspace(0.0, qmax, nfine)
    v = hat_matrix(x, t) @ a[1:]
    for half in (3, 2, 1):
        v = moving_average(v, half)
    return x, v


def local_maxima(x, v):
    """Step 7: (q, value) of each local maximum of the sampled curve."""
    n = len(v)
    h = x[1] - x[0]
    d = np.empty(n)
    d[1:-1] = (v[2:] - v[:-2]) / (2 * h)
    d[0] = (-3 * v[0] + 4 * v[1] - v[2]) / (2 * h)
    d[-1] = (3 * v[-1] - 4 * v[-2] + v[-3]) / (2 * h)
    peaks = []
    for j in range(n - 1):
        if d[j] > 0 and d[j + 1] <= 0:
            r = d[j] / (d[j] - d[j + 1])
            jj = j if r < 0.5 else j + 1
            jj = min(max(jj, 1), n - 2)
            if v[jj + 1] - 2 * v[jj] + v[jj - 1] < 0:
                peaks.append((x[j] + r * h, v[j] + r * (v[j + 1] - v[j])))
    return peaks


def radial_spectrum(h, h0, ds, sigma, qmax):
    """Steps 1-4: the radial scatter data (q, value, count)."""
    n = h.shape[0]
    s = smooth(spectrum_magnitude(h, h0), sigma)
    return radial_average(s, n * ds, qmax)


def dominant_wavenumbers(h, h0, ds, sigma, qmax, nfine=400):
    """Steps 1-7: local maxima (q, value) of the smoothed radial spectrum."""
    q, y, _ = radial_spectrum(h, h0, ds, sigma, qmax)
    t, a = piecewise_fit(q, y, qmax)
    x, v = smooth_curve(t, a, qmax, nfine)
    return local_maxima(x, v)
