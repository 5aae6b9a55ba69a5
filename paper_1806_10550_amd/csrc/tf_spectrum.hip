// Radial Fourier spectrum of a film (App. "Radial Fourier Transform"; see include/thinfilm.h,
// tf_radial_spectrum and tf_spectrum_maxima).
//
// Device part (steps 1-4): the film minus H0 is transformed by an in-place 2D real-to-complex
// FFT (hipFFT; half spectrum, the other half by conjugate symmetry); the magnitudes are
// gathered into a window of the wavenumber plane that covers the disk
// |k|^2 <= M plus the Gaussian's reach (indices taken modulo n, so the smoothing is the
// periodic convolution over the whole plane); two separable passes smooth the window; one
// thread per group m = kx^2 + ky^2 (all wavevectors of a group have the same |q|) sums its
// smoothed values in a fixed order (an index of the window by group, built once per
// window on the host), so spectra are bit-reproducible. Only the FFT touches all
// n^2 values; the window holds (2 sqrt(M) + 2 r + 1)^2 values.
//
// Host part (steps 5-7): the fit has about N/10 unknowns, the smoothed curve 400 points: a
// tridiagonal normal-equation solve and a few passes over 400 doubles, done in plain C++.
#include "tf_internal.h"
#include "../../include/thinfilm.h"

#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace tf {

// buf[j * pitch + i] = h[j * n + i] - h0: the film minus H0 in the padded row layout of an
// in-place real-to-complex transform (pitch = 2 (n/2 + 1) doubles).
__global__ void __launch_bounds__(256) k_spec_load(const double *__restrict__ h, double h0, int n, int pitch,
                                                   double *__restrict__ buf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= n) return;
    buf[(size_t)j * pitch + i] = h[(size_t)j * n + i] - h0;
}

// A[(wy + E) * W + (wx + E)] = |F(wx mod n, wy mod n)| / n^2 for wx, wy in [-E, E], from the
// half spectrum F[iy][ix], ix <= n/2, of the real transform: the other half follows from
// F(-k) = conj F(k).
__global__ void __launch_bounds__(256) k_spec_window(const hipfftDoubleComplex *__restrict__ F, int n, int E,
                                                     double inv_n2, double *__restrict__ A)
{
    const int W = 2 * E + 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= W * W) return;
    const int wx = t % W - E, wy = t / W - E;
    int ix = ((wx % n) + n) % n, iy = ((wy % n) + n) % n;
    if (ix > n / 2) {
        ix = n - ix;
        iy = (n - iy) % n;
    }
    const hipfftDoubleComplex c = F[(size_t)iy * (n / 2 + 1) + ix];
    A[t] = sqrt(c.x * c.x + c.y * c.y) * inv_n2;
}

// One separable smoothing pass over a window of side W (input) into a window of side
// W - 2r (output), along x (DIR 0) or y (DIR 1); the other index keeps its range when
// DIR says so: out is (Wo x Wi) with Wi = W along the untouched axis.
template <int DIR>
__global__ void __launch_bounds__(256) k_spec_smooth(const double *__restrict__ in, int Win_x, int Win_y,
                                                     const double *__restrict__ w, int r, double *__restrict__ out)
{
    const int Wo_x = DIR == 0 ? Win_x - 2 * r : Win_x;
    const int Wo_y = DIR == 1 ? Win_y - 2 * r : Win_y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Wo_x * Wo_y) return;
    const int ox = t % Wo_x, oy = t / Wo_x;
    double s = 0.0;
    for (int d = 0; d <= 2 * r; ++d) {
        const int ix = DIR == 0 ? ox + d : ox;
        const int iy = DIR == 1 ? oy + d : oy;
        s = fma(w[d], in[(size_t)iy * Win_x + ix], s);
    }
    out[t] = s;
}

// Group sums over the disk: S is the smoothed window of side 2R+1 centred on k = 0. One
// thread per group m = kx^2 + ky^2 (0 <= m <= M) adds its wavevectors' values in the
// order of the index (window positions sorted by group, then by position), so the sums
// do not depend on scheduling.
__global__ void __launch_bounds__(256) k_spec_groups(const double *__restrict__ S, const int *__restrict__ perm,
                                                     const long long *__restrict__ off, long long M,
                                                     double *__restrict__ sum, int *__restrict__ cnt)
{
    const long long m = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (m > M) return;
    const long long b = off[m], e = off[m + 1];
    double acc = 0.0;
    for (long long i = b; i < e; ++i) acc += S[perm[i]];
    sum[m] = acc;
    cnt[m] = (int)(e - b);
}

} // namespace tf

namespace {

tf_status sfail(tf_status s, const std::string &msg)
{
    tf_detail::set_error(msg);
    return s;
}

// Plan and scratch of one (device, n), kept until tf_spectrum_release: the padded real /
// half-complex buffer of the in-place transform and the small window and group arrays
// (grown on demand).
struct SpecWork {
    hipfftHandle plan = 0;
    bool has_plan = false;
    double *buf = nullptr;
    double *small = nullptr; // A | B | C | weights | sums, doubles
    int *cnt = nullptr;
    size_t small_cap = 0, cnt_cap = 0;
    // index of the window by group for the last (M, R): perm lists window positions sorted
    // by m = kx^2 + ky^2 (then by position), group m owns perm[off[m] .. off[m+1])
    int *perm = nullptr;
    long long *off = nullptr;
    long long idx_M = -1;
    int idx_R = -1;
};
struct WorkKey {
    int device, n;
    bool operator<(const WorkKey &o) const { return device != o.device ? device < o.device : n < o.n; }
};
std::mutex g_spec_mu;
std::map<WorkKey, SpecWork> g_spec;

void free_work(SpecWork &w)
{
    if (w.has_plan) (void)hipfftDestroy(w.plan);
    if (w.buf) (void)hipFree(w.buf);
    if (w.small) (void)hipFree(w.small);
    if (w.cnt) (void)hipFree(w.cnt);
    if (w.perm) (void)hipFree(w.perm);
    if (w.off) (void)hipFree(w.off);
    w = SpecWork{};
}

// The window index for groups 0..M over a window of half side R (n x n spectrum), built on
// the host by a counting sort over m (positions in increasing order within a group) and kept
// until the next call with another (M, R). Called with g_spec_mu held.
tf_status get_index(SpecWork &w, int n, int R, long long M)
{
    if (w.idx_M == M && w.idx_R == R) return TF_OK;
    const int Wr = 2 * R + 1;
    const int lo = -(n / 2), hi = (n - 1) / 2;
    const long long npos = (long long)Wr * Wr;
    std::vector<long long> off(M + 2, 0);
    auto group = [&](long long t) -> long long {
        const int kx = (int)(t % Wr) - R, ky = (int)(t / Wr) - R;
        if (kx < lo || kx > hi || ky < lo || ky > hi) return -1;
        const long long m = (long long)kx * kx + (long long)ky * ky;
        return m <= M ? m : -1;
    };
    for (long long t = 0; t < npos; ++t) {
        const long long m = group(t);
        if (m >= 0) ++off[m + 1];
    }
    for (long long m = 0; m <= M; ++m) off[m + 1] += off[m];
    std::vector<int> perm((size_t)off[M + 1]);
    std::vector<long long> next(off.begin(), off.end() - 1);
    for (long long t = 0; t < npos; ++t) {
        const long long m = group(t);
        if (m >= 0) perm[(size_t)next[m]++] = (int)t;
    }
    if (w.perm) (void)hipFree(w.perm);
    if (w.off) (void)hipFree(w.off);
    w.perm = nullptr;
    w.off = nullptr;
    w.idx_M = -1;
    if (hipMalloc(&w.perm, std::max<size_t>(perm.size(), 1) * sizeof(int)) != hipSuccess
        || hipMalloc(&w.off, off.size() * sizeof(long long)) != hipSuccess) {
        if (w.perm) (void)hipFree(w.perm);
        w.perm = nullptr;
        w.off = nullptr;
        return sfail(TF_ENOMEM, "spectrum index allocation failed");
    }
    if (hipMemcpy(w.perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess
        || hipMemcpy(w.off, off.data(), off.size() * sizeof(long long), hipMemcpyHostToDevice) != hipSuccess)
        return sfail(TF_EDEVICE, "spectrum index upload failed");
    w.idx_M = M;
    w.idx_R = R;
    return TF_OK;
}

// Called with g_spec_mu held.
tf_status get_work(int n, size_t small_doubles, size_t groups, SpecWork **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return sfail(TF_EDEVICE, "hipGetDevice failed");
    SpecWork &w = g_spec[WorkKey{dev, n}];
    if (!w.has_plan) {
        if (hipfftPlan2d(&w.plan, n, n, HIPFFT_D2Z) != HIPFFT_SUCCESS) return sfail(TF_EDEVICE, "hipfftPlan2d failed");
        w.has_plan = true;
    }
    if (w.buf == nullptr
        && hipMalloc(&w.buf, (size_t)n * (n / 2 + 1) * sizeof(hipfftDoubleComplex)) != hipSuccess) {
        w.buf = nullptr;
        return sfail(TF_ENOMEM, "spectrum buffer allocation failed");
    }
    if (w.small_cap < small_doubles) {
        if (w.small) (void)hipFree(w.small);
        w.small = nullptr;
        w.small_cap = 0;
        if (hipMalloc(&w.small, small_doubles * sizeof(double)) != hipSuccess) {
            w.small = nullptr;
            return sfail(TF_ENOMEM, "spectrum scratch allocation failed");
        }
        w.small_cap = small_doubles;
    }
    if (w.cnt_cap < groups) {
        if (w.cnt) (void)hipFree(w.cnt);
        w.cnt = nullptr;
        w.cnt_cap = 0;
        if (hipMalloc(&w.cnt, groups * sizeof(int)) != hipSuccess) {
            w.cnt = nullptr;
            return sfail(TF_ENOMEM, "spectrum scratch allocation failed");
        }
        w.cnt_cap = groups;
    }
    *out = &w;
    return TF_OK;
}

// Waits for the stream on every exit, so that no work of a failed call is left queued.
struct StreamDrain {
    hipStream_t s;
    ~StreamDrain() { (void)hipStreamSynchronize(s); }
};

} // namespace

extern "C" {

tf_status tf_radial_spectrum(const double *h, int n, double ds, double h0, double sigma, double qmax, void *stream,
                             double *q_out, double *s_out, int *count_out, int capacity, int *npoints)
{
    if (h == nullptr || npoints == nullptr) return sfail(TF_EINVAL, "NULL argument");
    if (n < 4 || n > (1 << 14)) return sfail(TF_EINVAL, "need 4 <= n <= 16384");
    if (!(ds > 0.0) || !std::isfinite(ds) || !std::isfinite(h0)) return sfail(TF_EINVAL, "need finite ds > 0 and h0");
    if (!(sigma >= 0.0) || sigma > 64.0) return sfail(TF_EINVAL, "need 0 <= sigma <= 64");
    if (!(qmax > 0.0) || !std::isfinite(qmax)) return sfail(TF_EINVAL, "need finite qmax > 0");
    const double L = n * ds;
    const double kmax = qmax * L / (2.0 * M_PI);
    // groups beyond the spectrum's largest |k|^2 are empty
    const double mcap = 2.0 * (double)(n / 2) * (double)(n / 2);
    long long M = (long long)std::floor(std::min(kmax * kmax * (1.0 + 1e-12), mcap));
    if (M < 1) {
        *npoints = 0;
        return TF_OK;
    }
    if (M > (1LL << 26)) return sfail(TF_EINVAL, "qmax too large: more than 2^26 wavenumber groups");
    const int R = std::min((int)std::floor(std::sqrt((double)M)), n / 2);
    const int r = sigma > 0.0 ? (int)std::ceil(4.0 * sigma) : 0;
    const int E = R + r, W = 2 * E + 1, Wr = 2 * R + 1;
    std::vector<double> w(2 * r + 1, 1.0);
    if (r > 0) {
        double z = 0.0;
        for (int d = -r; d <= r; ++d) z += (w[d + r] = std::exp(-(double)d * d / (2.0 * sigma * sigma)));
        for (double &v : w) v /= z;
    }
    hipStream_t s = (hipStream_t)stream;
    // small scratch: A (W x W) | B (Wr x W) | C (Wr x Wr) | weights | group sums
    const size_t oA = 0, oB = oA + (size_t)W * W, oC = oB + (size_t)W * Wr, oW = oC + (size_t)Wr * Wr,
                 oS = oW + w.size(), small = oS + (size_t)(M + 1);
    std::lock_guard<std::mutex> lk(g_spec_mu);
    SpecWork *wk;
    tf_status st = get_work(n, small, (size_t)(M + 1), &wk);
    if (st != TF_OK) return st;
    if ((st = get_index(*wk, n, R, M)) != TF_OK) return st;
    StreamDrain drain{s};
    double *A = wk->small + oA, *B = wk->small + oB, *C = wk->small + oC, *wd = wk->small + oW,
           *sum = wk->small + oS;
    const int pitch = 2 * (n / 2 + 1);
    tf::k_spec_load<<<dim3((n + 255) / 256, n), 256, 0, s>>>(h, h0, n, pitch, wk->buf);
    if (hipGetLastError() != hipSuccess) return sfail(TF_EDEVICE, "spectrum load launch failed");
    auto *F = (hipfftDoubleComplex *)wk->buf;
    if (hipfftSetStream(wk->plan, s) != HIPFFT_SUCCESS || hipfftExecD2Z(wk->plan, wk->buf, F) != HIPFFT_SUCCESS)
        return sfail(TF_EDEVICE, "hipfftExecD2Z failed");
    if (hipMemcpyAsync(wd, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return sfail(TF_EDEVICE, "spectrum scratch setup failed");
    const double inv_n2 = 1.0 / ((double)n * (double)n);
    tf::k_spec_window<<<(W * W + 255) / 256, 256, 0, s>>>(F, n, E, inv_n2, A);
    tf::k_spec_smooth<0><<<(Wr * W + 255) / 256, 256, 0, s>>>(A, W, W, wd, r, B);
    tf::k_spec_smooth<1><<<(Wr * Wr + 255) / 256, 256, 0, s>>>(B, Wr, W, wd, r, C);
    tf::k_spec_groups<<<(unsigned)((M + 1 + 255) / 256), 256, 0, s>>>(C, wk->perm, wk->off, M, sum, wk->cnt);
    if (hipGetLastError() != hipSuccess) return sfail(TF_EDEVICE, "spectrum kernel launch failed");
    std::vector<double> hs(M + 1);
    std::vector<int> hc(M + 1);
    if (hipMemcpyAsync(hs.data(), sum, (M + 1) * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess
        || hipMemcpyAsync(hc.data(), wk->cnt, (M + 1) * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess
        || hipStreamSynchronize(s) != hipSuccess)
        return sfail(TF_EDEVICE, "spectrum readback failed");
    int np = 0;
    for (long long m = 1; m <= M; ++m) {
        if (hc[m] == 0) continue;
        const double q = 2.0 * M_PI * std::sqrt((double)m) / L;
        if (q > qmax) continue;
        if (np < capacity && q_out != nullptr && s_out != nullptr) {
            q_out[np] = q;
            s_out[np] = hs[m] / hc[m];
            if (count_out != nullptr) count_out[np] = hc[m];
        }
        ++np;
    }
    *npoints = np;
    if (np > capacity || (np > 0 && (q_out == nullptr || s_out == nullptr)))
        return sfail(TF_EINVAL, "output capacity too small (npoints holds the number needed)");
    return TF_OK;
}

tf_status tf_spectrum_release(void)
{
    std::lock_guard<std::mutex> lk(g_spec_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_spec) {
        (void)hipSetDevice(kv.first.device);
        (void)hipDeviceSynchronize();
        free_work(kv.second);
    }
    g_spec.clear();
    (void)hipSetDevice(cur);
    return TF_OK;
}

tf_status tf_spectrum_maxima(const double *q, const double *s, int npoints, double qmax, int nfine, double *curve_out,
                             double *peak_q, double *peak_s, int capacity, int *npeaks)
{
    if (q == nullptr || s == nullptr || npeaks == nullptr) return sfail(TF_EINVAL, "NULL argument");
    if (npoints < 1 || nfine < 8 || !(qmax > 0.0)) return sfail(TF_EINVAL, "need npoints >= 1, nfine >= 8, qmax > 0");
    for (int p = 0; p < npoints; ++p)
        if (!(q[p] > 0.0) || q[p] > qmax || (p > 0 && !(q[p] > q[p - 1])) || !std::isfinite(s[p]))
            return sfail(TF_EINVAL, "q must increase strictly within (0, qmax] and s be finite");
    // knots: 0, q[9], q[19], ..., qmax; unknowns: the values at knots 1..K
    const int per = 10;
    const int K = std::max(1, npoints / per);
    std::vector<double> t(K + 1);
    t[0] = 0.0;
    for (int k = 1; k < K; ++k) t[k] = q[per * k - 1];
    t[K] = qmax;
    // normal equations of the hat basis: tridiagonal (K x K), unknown j <-> knot j + 1
    std::vector<double> dg(K, 0.0), up(K, 0.0), rhs(K, 0.0);
    int k = 0;
    for (int p = 0; p < npoints; ++p) {
        while (k < K - 1 && q[p] >= t[k + 1]) ++k;
        const double u = (q[p] - t[k]) / (t[k + 1] - t[k]);
        const double wl = 1.0 - u, wr = u; // weights of knots k and k+1
        if (k >= 1) {
            dg[k - 1] += wl * wl;
            up[k - 1] += wl * wr;
            rhs[k - 1] += wl * s[p];
        }
        dg[k] += wr * wr;
        rhs[k] += wr * s[p];
    }
    // symmetric tridiagonal solve (sub-diagonal = up shifted)
    std::vector<double> c(K, 0.0), d(K, 0.0);
    for (int j = 0; j < K; ++j) {
        const double sub = j > 0 ? up[j - 1] : 0.0;
        const double den = dg[j] - (j > 0 ? sub * c[j - 1] : 0.0);
        if (!(std::fabs(den) > 0.0)) return sfail(TF_EINVAL, "degenerate fit (an interval holds no data)");
        c[j] = up[j] / den;
        d[j] = (rhs[j] - (j > 0 ? sub * d[j - 1] : 0.0)) / den;
    }
    std::vector<double> a(K + 1, 0.0);
    for (int j = K - 1; j >= 0; --j) a[j + 1] = d[j] - (j < K - 1 ? c[j] * a[j + 2] : 0.0);
    // the fit on nfine equispaced points of [0, qmax]
    const double hstep = qmax / (nfine - 1);
    std::vector<double> x(nfine), v(nfine), tmp(nfine);
    k = 0;
    for (int j = 0; j < nfine; ++j) {
        x[j] = j == nfine - 1 ? qmax : j * hstep;
        while (k < K - 1 && x[j] >= t[k + 1]) ++k;
        const double u = (x[j] - t[k]) / (t[k + 1] - t[k]);
        v[j] = (1.0 - u) * a[k] + u * a[k + 1];
    }
    // moving averages, half widths 3, 2, 1, windows truncated at the ends
    for (int half : {3, 2, 1}) {
        for (int j = 0; j < nfine; ++j) {
            const int lo = std::max(0, j - half), hi = std::min(nfine - 1, j + half);
            double acc = 0.0;
            for (int i = lo; i <= hi; ++i) acc += v[i];
            tmp[j] = acc / (hi - lo + 1);
        }
        v.swap(tmp);
    }
    if (curve_out != nullptr) std::copy(v.begin(), v.end(), curve_out);
    // maxima: derivative by second-order differences, sign change + to -, second difference < 0
    std::vector<double> dv(nfine);
    for (int j = 1; j < nfine - 1; ++j) dv[j] = (v[j + 1] - v[j - 1]) / (2.0 * hstep);
    dv[0] = (-3.0 * v[0] + 4.0 * v[1] - v[2]) / (2.0 * hstep);
    dv[nfine - 1] = (3.0 * v[nfine - 1] - 4.0 * v[nfine - 2] + v[nfine - 3]) / (2.0 * hstep);
    int np = 0;
    for (int j = 0; j < nfine - 1; ++j) {
        if (!(dv[j] > 0.0 && dv[j + 1] <= 0.0)) continue;
        const double u = dv[j] / (dv[j] - dv[j + 1]);
        int jj = u < 0.5 ? j : j + 1;
        jj = std::min(std::max(jj, 1), nfine - 2);
        if (!(v[jj + 1] - 2.0 * v[jj] + v[jj - 1] < 0.0)) continue;
        if (np < capacity && peak_q != nullptr && peak_s != nullptr) {
            peak_q[np] = x[j] + u * hstep;
            peak_s[np] = v[j] + u * (v[j + 1] - v[j]);
        }
        ++np;
    }
    *npeaks = np;
    if (np > capacity) return sfail(TF_EINVAL, "peak capacity too small (npeaks holds the number found)");
    return TF_OK;
}

} // extern "C"
