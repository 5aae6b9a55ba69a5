// Discrete adjoint of the converged ADI-Newton step and the stored-band batched
// pentadiagonal solvers it uses (see include/thinfilm.h: tf_adjoint_step,
// tf_penta_solve, tf_autotune).
//
// The adjoint differentiates the implicit step map G(u^{n+1}; u^n, kappa) = 0 with
// G = u - u^n + dt[theta D(u) + (1 - theta) D(u^n)] (eq. TrapRule in theta form):
//   (I + theta dt J_D(u^{n+1}))^T mu = lambda^{n+1},
//   lambda^n = mu - (1 - theta) dt J_D(u^n)^T mu,
//   dL/dkappa -= dt mu . [theta dD/dkappa(u^{n+1}) + (1 - theta) dD/dkappa(u^n)].
// The transposed system is solved by Richardson iteration preconditioned with the
// transposed ADI factors P^-T = (I + c J_y)^-T (I + c J_x)^-T (a transposed row solve,
// then a transposed column solve), the same split as the forward Newton iteration
// (eqs. DirectionSplit, JacobianSystem1-2).
#include "tf_device.h"
#include "../../include/thinfilm.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace tf {

// ---- cell quantities straight from global memory (reflected ghosts) -------------------
template <bool P32>
__device__ __forceinline__ Cell cell_glob(const double *u, int nx, int ny, int i, int j, const Model &M, double ids2)
{
    const int ic = crefl(i, nx), jc = crefl(j, ny);
    const int im = crefl(ic - 1, nx), ip = crefl(ic + 1, nx), jm = crefl(jc - 1, ny), jp = crefl(jc + 1, ny);
    Cell c;
    c.u = u[(size_t)jc * nx + ic];
    c.lap = (u[(size_t)jc * nx + ip] + u[(size_t)jc * nx + im] + u[(size_t)jp * nx + ic] + u[(size_t)jm * nx + ic]
             - 4.0 * c.u) * ids2;
    model_coefs<P32>(M, c.u, c.f0, c.f1, c.f0p, c.f1p);
    c.f0p *= 0.5;
    c.f1p *= 0.5;
    return c;
}

// Bands (a, b, c, d, e) of I + c J along direction DIR at every cell, stored
// position-major for the stored-band solver: DIR 0 (y) as [j][i], DIR 1 (x) as [i][j];
// with LM (DIR 1) line-major as [j][i] for the whole-line row solver.
template <int DIR, bool P32, bool LM = false>
__global__ void __launch_bounds__(256) k_bands_store(int nx, int ny, double ids, double ids2, double k1, double k3,
                                                     Model M, const double *u, double *bands)
{
    // lanes along the contiguous index of the layout: i for [j][i], j for [i][j]
    constexpr bool LANES_I = DIR == 0 || LM;
    const int a0 = blockIdx.x * 64 + (threadIdx.x & 63), b0 = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int i = LANES_I ? a0 : b0, j = LANES_I ? b0 : a0;
    if (i >= nx || j >= ny) return;
    const int Np = DIR == 0 ? ny : nx;
    const int gp = DIR == 0 ? j : i;
    const int di = DIR == 0 ? 0 : 1, dj = DIR == 0 ? 1 : 0;
    const Cell cm = cell_glob<P32>(u, nx, ny, i - di, j - dj, M, ids2);
    const Cell c0 = cell_glob<P32>(u, nx, ny, i, j, M, ids2);
    const Cell cp = cell_glob<P32>(u, nx, ny, i + di, j + dj, M, ids2);
    const FaceQ fm = face_q<false>(cm, c0, gp > 0, ids, k1, k3);
    const FaceQ fp = face_q<false>(c0, cp, gp < Np - 1, ids, k1, k3);
    double a = fm.kA;
    double b = -fp.kA - 3.0 * fm.kA - fm.P;
    double c = 1.0 + 3.0 * fp.kA + fp.P + 3.0 * fm.kA - fm.Q;
    double d = -3.0 * fp.kA + fp.Q - fm.kA;
    double e = fp.kA;
    if (gp == 0) { c += b; d += a; b = 0.0; a = 0.0; }
    else if (gp == 1) { b += a; a = 0.0; }
    if (gp == Np - 1) { c += d; b += e; d = 0.0; e = 0.0; }
    else if (gp == Np - 2) { d += e; e = 0.0; }
    const size_t N = (size_t)nx * ny;
    const size_t o = LANES_I ? (size_t)j * nx + i : (size_t)i * ny + j;
    bands[o] = a;
    bands[N + o] = b;
    bands[2 * N + o] = c;
    bands[3 * N + o] = d;
    bands[4 * N + o] = e;
}

// ---- stored-band batched pentadiagonal solves ------------------------------------------
// Data layout [position][line] (lanes = consecutive lines); bands as 5 arrays a..e.
// TRANS: solve with the transposed matrix, whose row p is
//   (e_{p-2}, d_{p-1}, c_p, b_{p+1}, a_{p+2}).
template <bool TRANS>
__device__ __forceinline__ void load_band_row(const double *bands, size_t N, int nl, int np, int p, int line,
                                              double &a, double &b, double &c, double &d, double &e)
{
    const size_t o = (size_t)p * nl + line;
    if (!TRANS) {
        a = bands[o]; b = bands[N + o]; c = bands[2 * N + o]; d = bands[3 * N + o]; e = bands[4 * N + o];
    } else {
        a = p >= 2 ? bands[4 * N + o - 2 * (size_t)nl] : 0.0;
        b = p >= 1 ? bands[3 * N + o - (size_t)nl] : 0.0;
        c = bands[2 * N + o];
        d = p + 1 < np ? bands[N + o + (size_t)nl] : 0.0;
        e = p + 2 < np ? bands[o + 2 * (size_t)nl] : 0.0;
    }
}

// LU elimination over a (sub-)segment with its two left outer unknowns kept symbolic
// and two rows of the inverse upper factor accumulated on the fly (same algebra as the
// forward sweep): yields the segment's top/bottom relation record.
struct Elim {
    double al1 = 0.0, be1 = 0.0, al2 = 0.0, be2 = 0.0;
    double z1 = 0.0, ph1 = 0.0, ps1 = 1.0, z2 = 0.0, ph2 = 1.0, ps2 = 0.0;
    double g1 = 0.0, g2 = 0.0, h1 = 0.0, h2 = 0.0;
    double sgz = 0.0, sgph = 0.0, sgps = 0.0, shz = 0.0, shph = 0.0, shps = 0.0;
    __device__ __forceinline__ void step(int k, double a, double b, double c, double d, double e, double rhs,
                                         double &al, double &be, double &z, double &ph, double &pss)
    {
        const double gam = b - a * al2;
        const double mu = c - a * be2 - gam * al1;
        const double rm = rcp(mu);
        al = (d - gam * be1) * rm;
        be = e * rm;
        z = (rhs - a * z2 - gam * z1) * rm;
        ph = (-a * ph2 - gam * ph1) * rm;
        pss = (-a * ps2 - gam * ps1) * rm;
        const double g = k == 0 ? 1.0 : -al1 * g1 - be2 * g2;
        const double h = k == 1 ? 1.0 : (k == 0 ? 0.0 : -al1 * h1 - be2 * h2);
        sgz += g * z; sgph += g * ph; sgps += g * pss;
        shz += h * z; shph += h * ph; shps += h * pss;
        g2 = g1; g1 = g; h2 = h1; h1 = h;
        al2 = al1; be2 = be1; al1 = al; be1 = be;
        z2 = z1; ph2 = ph1; ps2 = ps1; z1 = z; ph1 = ph; ps1 = pss;
    }
    __device__ __forceinline__ void finish(Rel &r) const
    {
        r.B[1][0] = z1; r.B[1][1] = ph1; r.B[1][2] = ps1; r.B[1][3] = -al1; r.B[1][4] = -be1;
        r.B[0][0] = z2 - al2 * z1; r.B[0][1] = ph2 - al2 * ph1; r.B[0][2] = ps2 - al2 * ps1;
        r.B[0][3] = -be2 + al2 * al1; r.B[0][4] = al2 * be1;
        r.T[0][0] = sgz; r.T[0][1] = sgph; r.T[0][2] = sgps;
        r.T[0][3] = -g2 * be2 - g1 * al1; r.T[0][4] = -g1 * be1;
        r.T[1][0] = shz; r.T[1][1] = shph; r.T[1][2] = shps;
        r.T[1][3] = -h2 * be2 - h1 * al1; r.T[1][4] = -h1 * be1;
    }
};

struct SBParams {
    int nl, np;               // lines, cells per line
    const double *bands;      // 5 arrays of nl*np
    const double *rhs;
    double *out;              // MODE 0: x; MODE 1: out += x
    double *rel;
    const double *ext;
    unsigned long long *red;  // MODE 1: {max|x|, max|out|}
};

// Partitioned solve over tiles of 64 lines x 64 cells (4 waves x 16-cell sub-segments):
// SOLVE false emits the tile's relation record per line, SOLVE true back-substitutes.
// ROWIO: rhs (and, MODE 0, out) are line-major [line][position] instead of [position][line];
// the tile's 64 x 64 block goes through LDS so that global accesses stay coalesced (this
// spares the row solves of the adjoint a transpose in and a transpose out).
template <bool SOLVE, bool TRANS, int MODE, bool ROWIO = false>
__global__ void __launch_bounds__(BLOCK) k_sb_pass(SBParams P)
{
    static_assert(!(ROWIO && MODE == 1), "line-major output is for MODE 0");
    constexpr int RP = TILE + 1; // LDS pitch of the line-major staging tile
    __shared__ double sB[NSUB * NREL * 64];
    __shared__ double sRed[NSUB][2];
    __shared__ double sR[ROWIO ? TILE * RP : 1];
    const int nlg = (P.nl + 63) / 64;
    const int t = xcd_tile(blockIdx.x, nlg * seg_count(P.np));
    const int lg = t % nlg, q = t / nlg;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int line = lg * 64 + lane;
    const bool owned = line < P.nl;
    const int lc = owned ? line : P.nl - 1;
    const int s0 = seg_start(q, P.np), s1 = seg_start(q + 1, P.np);
    const int npos = s1 - s0;
    const int nsub = min(NSUB, npos / 2);
    const int ps = (wave * npos) / nsub;
    const int len = wave < nsub ? ((wave + 1) * npos) / nsub - ps : 0;
    const size_t N = (size_t)P.nl * P.np;
    if (ROWIO) {
        // sR[k * RP + l] = rhs of line lg*64 + l (clamped) at position s0 + k
        for (int e = tid; e < 64 * npos; e += BLOCK) {
            const int l = e / npos, k = e - l * npos;
            const int gl = min(lg * 64 + l, P.nl - 1);
            sR[k * RP + l] = P.rhs[(size_t)gl * P.np + s0 + k];
        }
        __syncthreads();
    }
    double fa[SUB], fb[SUB], fz[SUB], fph[SUB], fps[SUB];
    Rel mine;
    if (len > 0) {
        Elim E;
#pragma unroll
        for (int k = 0; k < SUB; ++k) {
            if (k < len) {
                const int p = s0 + ps + k;
                double a, b, c, d, e;
                load_band_row<TRANS>(P.bands, N, P.nl, P.np, p, lc, a, b, c, d, e);
                const double rhs = ROWIO ? sR[(ps + k) * RP + lane] : P.rhs[(size_t)p * P.nl + lc];
                double al, be, z, ph, pss;
                E.step(k, a, b, c, d, e, rhs, al, be, z, ph, pss);
                if (SOLVE) { fa[k] = al; fb[k] = be; fz[k] = z; fph[k] = ph; fps[k] = pss; }
            }
        }
        E.finish(mine);
        double *dst = sB + (size_t)wave * NREL * 64 + lane;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                dst[(i * 5 + j) * 64] = mine.T[i][j];
                dst[(10 + i * 5 + j) * 64] = mine.B[i][j];
            }
    }
    __syncthreads();
    if (!SOLVE) {
        if (wave == 0 && owned) {
            Rel seg;
            Rel first;
            load_rel(sB, 0, lane, first);
            chain_symbolic(first, sB + NREL * 64, lane, nsub, seg);
            rel_store(P.rel + (size_t)q * NREL * P.nl + 2 * (size_t)line, P.nl, seg);
        }
        return;
    }
    double xm = 0.0, om = 0.0;
    if (len > 0) {
        const double *ex = P.ext + (size_t)q * NEXT * P.nl + lc;
        double wl1, wl2, xr1, xr2;
        chain_numeric(sB, lane, nsub, wave, ex[0], ex[(size_t)P.nl], ex[(size_t)2 * P.nl], ex[(size_t)3 * P.nl],
                      wl1, wl2, xr1, xr2);
#pragma unroll
        for (int k = SUB - 1; k >= 0; --k) {
            if (k < len) {
                const double x = fz[k] + fph[k] * wl1 + fps[k] * wl2 - fa[k] * xr1 - fb[k] * xr2;
                xr2 = xr1;
                xr1 = x;
                if (ROWIO) {
                    sR[(ps + k) * RP + lane] = x; // every rhs read happened before the exchange barrier
                } else if (owned) {
                    const size_t o = (size_t)(s0 + ps + k) * P.nl + line;
                    if (MODE == 0) {
                        P.out[o] = x;
                    } else {
                        const double v = P.out[o] + x;
                        P.out[o] = v;
                        xm = max_nan(xm, fabs(x));
                        om = max_nan(om, fabs(v));
                            }
                }
            }
        }
    }
    if (ROWIO) {
        __syncthreads();
        for (int e = tid; e < 64 * npos; e += BLOCK) {
            const int l = e / npos, k = e - l * npos;
            const int gl = lg * 64 + l;
            if (gl < P.nl) P.out[(size_t)gl * P.np + s0 + k] = sR[k * RP + l];
        }
    }
    if (MODE == 1) {
        const double wx = wave_max_nan(xm), wo = wave_max_nan(om);
        if (lane == 0) { sRed[wave][0] = wx; sRed[wave][1] = wo; }
        __syncthreads();
        if (tid == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < NSUB; ++w) { a = max_nan(a, sRed[w][0]); b = max_nan(b, sRed[w][1]); }
            atomicMax(&P.red[0], (unsigned long long)__double_as_longlong(a));
            atomicMax(&P.red[1], (unsigned long long)__double_as_longlong(b));
        }
    }
}

// Interleaved Thomas: one lane per line over the whole line, factors kept in a
// position-major workspace (3 doubles per cell), then back-substitution. The block size
// (64, 128 or 256 lines) is a tuning parameter.
template <bool TRANS, int MODE>
__global__ void __launch_bounds__(256) k_sb_thomas(SBParams P, double *work)
{
    const int line = blockIdx.x * blockDim.x + threadIdx.x;
    double xm = 0.0, om = 0.0;
    const size_t N = (size_t)P.nl * P.np;
    if (line < P.nl) {
        double al1 = 0.0, be1 = 0.0, al2 = 0.0, be2 = 0.0, z1 = 0.0, z2 = 0.0;
        for (int p = 0; p < P.np; ++p) {
            double a, b, c, d, e;
            load_band_row<TRANS>(P.bands, N, P.nl, P.np, p, line, a, b, c, d, e);
            const double rhs = P.rhs[(size_t)p * P.nl + line];
            const double gam = b - a * al2;
            const double mu = c - a * be2 - gam * al1;
            const double rm = rcp(mu);
            const double al = (d - gam * be1) * rm, be = e * rm, z = (rhs - a * z2 - gam * z1) * rm;
            const size_t o = (size_t)p * P.nl + line;
            work[o] = al;
            work[N + o] = be;
            work[2 * N + o] = z;
            al2 = al1; be2 = be1; al1 = al; be1 = be; z2 = z1; z1 = z;
        }
        double x1 = 0.0, x2 = 0.0;
        for (int p = P.np - 1; p >= 0; --p) {
            const size_t o = (size_t)p * P.nl + line;
            const double x = work[2 * N + o] - work[o] * x1 - work[N + o] * x2;
            x2 = x1;
            x1 = x;
            if (MODE == 0) {
                P.out[o] = x;
            } else {
                const double v = P.out[o] + x;
                P.out[o] = v;
                xm = max_nan(xm, fabs(x));
                om = max_nan(om, fabs(v));
            }
        }
    }
    if (MODE == 1) {
        const double wx = wave_max_nan(xm), wo = wave_max_nan(om);
        if ((threadIdx.x & 63) == 0) {
            atomicMax(&P.red[0], (unsigned long long)__double_as_longlong(wx));
            atomicMax(&P.red[1], (unsigned long long)__double_as_longlong(wo));
        }
    }
}

// Block cyclic reduction in LDS. With X_i = (x_2i, x_2i+1) the pentadiagonal system of a
// line is block tridiagonal in 2x2 blocks,
//   A_i X_{i-1} + B_i X_i + C_i X_{i+1} = R_i,
//   A_i = [a_2i b_2i; 0 a_2i+1], B_i = [c_2i d_2i; b_2i+1 c_2i+1], C_i = [e_2i 0; d_2i+1 e_2i+1]
// (an odd line gets one identity row). Parallel cyclic reduction lets every block row
// eliminate its neighbours at distance s = 1, 2, 4, ...,
//   al = -A_i B_{i-s}^-1, ga = -C_i B_{i+s}^-1,
//   A_i <- al A_{i-s}, C_i <- ga C_{i+s}, B_i <- B_i + al C_{i-s} + ga A_{i+s},
//   R_i <- R_i + al R_{i-s} + ga R_{i+s},
// until every block row stands alone: X_i = B_i^-1 R_i. One workgroup per line, the
// whole line in LDS (lines of at most PCR_MAX cells). O(n log n) work, but log-depth:
// it pays for few long lines.
constexpr int PCR_MAX = 2048, PCR_THREADS = 256;
constexpr int PCR_RPT = PCR_MAX / 2 / PCR_THREADS; // block rows per thread

__device__ __forceinline__ M2 inv2(const M2 &x)
{
    const double r = rcp(x.a * x.d - x.b * x.c);
    return {x.d * r, -x.b * r, -x.c * r, x.a * r};
}
__device__ __forceinline__ M2 add2(const M2 &x, const M2 &y) { return {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d}; }

template <bool TRANS, int MODE>
__global__ void __launch_bounds__(PCR_THREADS) k_sb_pcr(SBParams P)
{
    constexpr int MB = PCR_MAX / 2;
    __shared__ double sM[14][MB]; // A (4), B (4), C (4), R (2) per block row
    __shared__ double sRed[PCR_THREADS / 64][2];
    const int line = blockIdx.x, tid = threadIdx.x;
    const int np = P.np, m = (np + 1) / 2;
    const size_t N = (size_t)P.nl * np;
    auto ld = [&](int i, M2 &A, M2 &B, M2 &C, double &r0, double &r1) {
        A = {sM[0][i], sM[1][i], sM[2][i], sM[3][i]};
        B = {sM[4][i], sM[5][i], sM[6][i], sM[7][i]};
        C = {sM[8][i], sM[9][i], sM[10][i], sM[11][i]};
        r0 = sM[12][i];
        r1 = sM[13][i];
    };
    auto st = [&](int i, const M2 &A, const M2 &B, const M2 &C, double r0, double r1) {
        sM[0][i] = A.a; sM[1][i] = A.b; sM[2][i] = A.c; sM[3][i] = A.d;
        sM[4][i] = B.a; sM[5][i] = B.b; sM[6][i] = B.c; sM[7][i] = B.d;
        sM[8][i] = C.a; sM[9][i] = C.b; sM[10][i] = C.c; sM[11][i] = C.d;
        sM[12][i] = r0; sM[13][i] = r1;
    };
    for (int i = tid; i < m; i += PCR_THREADS) {
        double a0, b0, c0, d0, e0, a1 = 0.0, b1 = 0.0, c1 = 1.0, d1 = 0.0, e1 = 0.0, r1 = 0.0;
        load_band_row<TRANS>(P.bands, N, P.nl, np, 2 * i, line, a0, b0, c0, d0, e0);
        const double r0 = P.rhs[(size_t)(2 * i) * P.nl + line];
        if (2 * i + 1 < np) {
            load_band_row<TRANS>(P.bands, N, P.nl, np, 2 * i + 1, line, a1, b1, c1, d1, e1);
            r1 = P.rhs[(size_t)(2 * i + 1) * P.nl + line];
        }
        st(i, {a0, b0, 0.0, a1}, {c0, d0, b1, c1}, {e0, 0.0, d1, e1}, r0, r1);
    }
    __syncthreads();
    for (int s = 1; s < m; s <<= 1) {
        M2 nA[PCR_RPT], nB[PCR_RPT], nC[PCR_RPT];
        double nr0[PCR_RPT], nr1[PCR_RPT];
#pragma unroll
        for (int k = 0; k < PCR_RPT; ++k) {
            const int i = tid + k * PCR_THREADS;
            if (i < m) {
                M2 A, B, C;
                double r0, r1;
                ld(i, A, B, C, r0, r1);
                M2 oA = {0, 0, 0, 0}, oC = {0, 0, 0, 0};
                if (i - s >= 0) {
                    M2 Al, Bl, Cl;
                    double l0, l1;
                    ld(i - s, Al, Bl, Cl, l0, l1);
                    const M2 al = mul(A, inv2(Bl));
                    oA = {-(al.a * Al.a + al.b * Al.c), -(al.a * Al.b + al.b * Al.d),
                          -(al.c * Al.a + al.d * Al.c), -(al.c * Al.b + al.d * Al.d)};
                    const M2 t = mul(al, Cl);
                    B = {B.a - t.a, B.b - t.b, B.c - t.c, B.d - t.d};
                    r0 -= al.a * l0 + al.b * l1;
                    r1 -= al.c * l0 + al.d * l1;
                }
                if (i + s < m) {
                    M2 Ar, Br, Cr;
                    double q0, q1;
                    ld(i + s, Ar, Br, Cr, q0, q1);
                    const M2 ga = mul(C, inv2(Br));
                    oC = {-(ga.a * Cr.a + ga.b * Cr.c), -(ga.a * Cr.b + ga.b * Cr.d),
                          -(ga.c * Cr.a + ga.d * Cr.c), -(ga.c * Cr.b + ga.d * Cr.d)};
                    const M2 t = mul(ga, Ar);
                    B = {B.a - t.a, B.b - t.b, B.c - t.c, B.d - t.d};
                    r0 -= ga.a * q0 + ga.b * q1;
                    r1 -= ga.c * q0 + ga.d * q1;
                }
                nA[k] = oA; nB[k] = B; nC[k] = oC; nr0[k] = r0; nr1[k] = r1;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PCR_RPT; ++k) {
            const int i = tid + k * PCR_THREADS;
            if (i < m) st(i, nA[k], nB[k], nC[k], nr0[k], nr1[k]);
        }
        __syncthreads();
    }
    double xm = 0.0, om = 0.0;
    for (int i = tid; i < m; i += PCR_THREADS) {
        M2 A, B, C;
        double r0, r1;
        ld(i, A, B, C, r0, r1);
        const M2 Bi = inv2(B);
        const double x[2] = {Bi.a * r0 + Bi.b * r1, Bi.c * r0 + Bi.d * r1};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = 2 * i + h;
            if (p >= np) break;
            const size_t o = (size_t)p * P.nl + line;
            if (MODE == 0) {
                P.out[o] = x[h];
            } else {
                const double v = P.out[o] + x[h];
                P.out[o] = v;
                xm = max_nan(xm, fabs(x[h]));
                om = max_nan(om, fabs(v));
            }
        }
    }
    if (MODE == 1) {
        const double wx = wave_max_nan(xm), wo = wave_max_nan(om);
        if ((tid & 63) == 0) { sRed[tid >> 6][0] = wx; sRed[tid >> 6][1] = wo; }
        __syncthreads();
        if (tid == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < PCR_THREADS / 64; ++w) { a = max_nan(a, sRed[w][0]); b = max_nan(b, sRed[w][1]); }
            atomicMax(&P.red[0], (unsigned long long)__double_as_longlong(a));
            atomicMax(&P.red[1], (unsigned long long)__double_as_longlong(b));
        }
    }
}

// ---- transposed Jacobian apply ---------------------------------------------------------
// J_D^T mu = local + L(xi) with, over the four faces f of a cell (omega_f = (mu_L - mu_R)/ds):
//   local_c = sum_f omega_f [ f0'_c Lam_f / 2 + f1'_c Gam_f / 2 -+ B_f / ds ]  (- if c = L)
//   xi_c    = sum_f omega_f A_f (+1 if c = R, -1 if c = L) / ds
// and L the cell-centred Laplacian (symmetric under the even reflection).
template <bool P32>
__device__ __forceinline__ void jdt_cell(int nx, int ny, double ids, double ids2, const Model &M, const double *u,
                                         const double *mu, int i, int j, double &xi, double &loc)
{
    const Cell c = cell_glob<P32>(u, nx, ny, i, j, M, ids2);
    const double mc = mu[(size_t)j * nx + i];
    double lo = 0.0, x = 0.0;
    const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
    const bool inside[4] = {i > 0, i < nx - 1, j > 0, j < ny - 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!inside[k]) continue;
        const int ni = i + di[k], nj = j + dj[k];
        const Cell n = cell_glob<P32>(u, nx, ny, ni, nj, M, ids2);
        const double mn = mu[(size_t)nj * nx + ni];
        const bool cIsR = (k == 0 || k == 2); // neighbour is the lower-index cell L
        const double A = 0.5 * (cIsR ? n.f0 + c.f0 : c.f0 + n.f0);
        const double B = 0.5 * (cIsR ? n.f1 + c.f1 : c.f1 + n.f1);
        const double Lam = (cIsR ? c.lap - n.lap : n.lap - c.lap) * ids;
        const double Gam = (cIsR ? c.u - n.u : n.u - c.u) * ids;
        const double om = (cIsR ? mn - mc : mc - mn) * ids;
        lo += om * (c.f0p * Lam + c.f1p * Gam + (cIsR ? B * ids : -B * ids));
        x += (cIsR ? om * A : -om * A) * ids;
    }
    xi = x;
    loc = lo;
}

// out = a lam + b mu + g J_D(u)^T mu in one kernel: a workgroup owns a JT_X x JT_Y tile,
// forms xi on the tile and its one-cell ring (ghost positions take the reflected cell's
// value) and local on the tile in LDS, then applies the Laplacian to xi from LDS.
// clr (nullable): two reduction words zeroed for a later kernel of the stream.
// Richardson iterations enqueued in a batch (ctl non-null): ctl[0] is the stop word. A
// launch that finds it set does nothing; one that finds the previous iteration's record
// chk = {max|z|, max|mu|} converged (max|z| <= tol max|mu|) or NaN does nothing either and
// sets ctl[0] (1: converged, 2: NaN) and ctl[1] = it - 1, the converged iteration. Every
// workgroup reads the same record, so all take the same decision.
constexpr int JT_X = 64, JT_Y = 16;
template <bool P32>
__global__ void __launch_bounds__(256) k_jdt(int nx, int ny, double ids, double ids2, Model M, const double *u,
                                             const double *mu, const double *lam, double a, double b, double g,
                                             double *out, unsigned long long *clr, const unsigned long long *chk,
                                             unsigned long long *ctl, double tol, int it)
{
    constexpr int RX = JT_X + 2, RY = JT_Y + 2;
    __shared__ double sxi[RY * RX], sloc[RY * RX];
    if (ctl != nullptr) {
        if (ctl[0] != 0ull) return;
        if (chk != nullptr) {
            const double zmax = __longlong_as_double((long long)chk[0]), mmax = __longlong_as_double((long long)chk[1]);
            const bool nan = !(zmax == zmax) || !(mmax == mmax);
            if (nan || zmax <= tol * mmax) {
                if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
                    ctl[1] = (unsigned long long)(it - 1);
                    ctl[0] = nan ? 2ull : 1ull;
                }
                return;
            }
        }
    }
    if (clr != nullptr && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 2) clr[threadIdx.x] = 0ull;
    const int i0 = blockIdx.x * JT_X, j0 = blockIdx.y * JT_Y;
    for (int e = threadIdx.x; e < RX * RY; e += 256) {
        const int li = e % RX, lj = e / RX;
        const int ri = i0 - 1 + li, rj = j0 - 1 + lj; // -1 and nx / ny are the ghost layer
        if (ri > nx || rj > ny) continue;             // beyond it: never read
        double x, l;
        jdt_cell<P32>(nx, ny, ids, ids2, M, u, mu, crefl(ri, nx), crefl(rj, ny), x, l);
        sxi[e] = x;
        sloc[e] = l;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < JT_X * JT_Y; e += 256) {
        const int ti = e % JT_X, tj = e / JT_X;
        const int i = i0 + ti, j = j0 + tj;
        if (i >= nx || j >= ny) continue;
        const int c = (tj + 1) * RX + ti + 1;
        const double lx = (sxi[c + 1] + sxi[c - 1] + sxi[c + RX] + sxi[c - RX] - 4.0 * sxi[c]) * ids2;
        const size_t o = (size_t)j * nx + i;
        double v = g * (sloc[c] + lx);
        if (b != 0.0) v += b * mu[o];
        if (a != 0.0) v += a * lam[o];
        out[o] = v;
    }
}

// out[i][j] = in[j][i] through a 64x64 LDS tile
__global__ void __launch_bounds__(256) k_transpose(int rows, int cols, const double *in, double *out)
{
    __shared__ double t[64][65];
    const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    for (int r = ly; r < 64; r += 4)
        if (r0 + r < rows && c0 + lx < cols) t[r][lx] = in[(size_t)(r0 + r) * cols + c0 + lx];
    __syncthreads();
    for (int c = ly; c < 64; c += 4)
        if (c0 + c < cols && r0 + lx < rows) out[(size_t)(c0 + c) * rows + r0 + lx] = t[lx][c];
}

// partial sums of x . (wa a + wb b), compensated, fixed order
__global__ void __launch_bounds__(256) k_dot(const double *x, const double *a, const double *b, double wa, double wb,
                                             size_t n, double *partials)
{
    __shared__ double ss[256], sc[256];
    double s = 0.0, c = 0.0;
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) {
        double v = wa * a[k];
        if (b != nullptr) v += wb * b[k];
        const double p = x[k] * v;
        const double t = s + p;
        c += fabs(s) >= fabs(p) ? (s - t) + p : (p - t) + s;
        s = t;
    }
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double p = ss[threadIdx.x + w], q = ss[threadIdx.x];
            const double t = q + p;
            sc[threadIdx.x] += sc[threadIdx.x + w] + (fabs(q) >= fabs(p) ? (q - t) + p : (p - t) + q);
            ss[threadIdx.x] = t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = ss[0];
        partials[2 * blockIdx.x + 1] = sc[0];
    }
}

// random diagonally dominant test systems for the autotuner
__global__ void k_fill_test(size_t n, double *bands, double *rhs)
{
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) {
        unsigned long long z = k * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const double r = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        bands[k] = 0.1 * r;
        bands[n + k] = -0.4 * r;
        bands[2 * n + k] = 2.0 + r;
        bands[3 * n + k] = -0.3 * r;
        bands[4 * n + k] = 0.2 * r;
        rhs[k] = r - 0.5;
    }
}

// A film 1 + 0.01 r and a right-hand side 1e-6 (r - 1/2), r uniform in [0, 1) from a
// counter-based hash, for timing the forward x sweeps.
__global__ void k_fill_film(size_t n, double *u, double *w)
{
    for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) {
        unsigned long long z = k * 0x9E3779B97F4A7C15ull + 0x2545F4914F6CDD1Dull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const double r = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        u[k] = 1.0 + 0.01 * r;
        w[k] = 1e-6 * (r - 0.5);
    }
}

} // namespace tf

// =========================================================================================
// host
// =========================================================================================
namespace {

tf_status afail(tf_status s, const std::string &msg)
{
    tf_detail::set_error(msg);
    return s;
}

#define TF_AHIP(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return afail(TF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

enum Variant { V_PARTITIONED = 0, V_THOMAS = 1, V_PCR = 2, V_LINE = 3, N_VARIANTS = 4 };
const char *kVariantNames[] = {"partitioned", "thomas", "pcr", "line"};

// A solver choice: the variant and, for Thomas, the workgroup size (lines per block).
struct Choice {
    int variant = V_PARTITIONED;
    int block = 64;
};

struct TuneKey {
    int length, batch, transposed;
    bool operator<(const TuneKey &o) const
    {
        return length != o.length ? length < o.length : (batch != o.batch ? batch < o.batch : transposed < o.transposed);
    }
};
struct TuneTable {
    std::mutex mu;
    std::map<TuneKey, Choice> best; // (length, batch, transposed) -> choice
};
TuneTable &tune_table()
{
    static TuneTable t;
    return t;
}
// Table entries of the forward x sweep (variant 0: partitioned, 1: whole-row) use this
// value in TuneKey::transposed.
constexpr int XSWEEP_KIND = 2;

// choice for a batch of `nl` lines of length `np` (plain or transposed solves): the
// autotuned entry of the same kind with the nearest (log-distance) shape, else a
// heuristic (one lane per line only pays when the lines alone fill the GPU). Cyclic
// reduction is only used for lines that fit in LDS.
Choice pick_variant(int np, int nl, bool trans)
{
    TuneTable &t = tune_table();
    std::lock_guard<std::mutex> lk(t.mu);
    double best_d = 1e30;
    Choice c;
    bool found = false;
    for (auto &kv : t.best) {
        if (kv.first.transposed != (int)trans) continue; // (also skips the x-sweep entries)
        const double d = std::fabs(std::log((double)kv.first.length / np)) + std::fabs(std::log((double)kv.first.batch / nl));
        if (d < best_d) { best_d = d; c = kv.second; found = true; }
    }
    if (found && best_d < 0.7 && !(c.variant == V_PCR && np > tf::PCR_MAX)
        && !(c.variant == V_LINE && !tf::sbline_supported(np)))
        return c;
    c.variant = nl >= 65536 ? V_THOMAS : V_PARTITIONED;
    c.block = 64;
    return c;
}

struct Scratch {
    double *rel = nullptr, *ext = nullptr, *chain = nullptr, *work = nullptr;
};

} // namespace

namespace tf {
// x-sweep variant for ny rows of nx cells in one launch: the tuned entry with the nearest
// shape, else the measured rule (the whole-row kernel while the launch has at most 2048
// rows: with few rows the partitioned solver's three launches are latency bound, with many
// its tile kernels stream faster); the whole-row kernel is only chosen where its 4-wave
// workgroups hold the row (nx <= 4096).
int xsweep_choice(int nx, int ny)
{
    if (!xrow_supported(nx) || nx > XR_ROW4_MAX_NX) return 0;
    TuneTable &t = tune_table();
    std::lock_guard<std::mutex> lk(t.mu);
    double best_d = 1e30;
    int v = -1;
    for (auto &kv : t.best) {
        if (kv.first.transposed != XSWEEP_KIND) continue;
        const double d = std::fabs(std::log((double)kv.first.length / nx)) + std::fabs(std::log((double)kv.first.batch / ny));
        if (d < best_d) { best_d = d; v = kv.second.variant; }
    }
    if (v >= 0 && best_d < 0.7) return v;
    return ny <= 2048 ? 1 : 0;
}
} // namespace tf

namespace {

// rowio: rhs and out line-major (transposed MODE 0 solves of the partitioned variant, and
// of the whole-line variant, whose bands are then line-major too).
tf_status sb_solve(Choice ch, bool trans, int mode, int nl, int np, const double *bands, const double *rhs,
                   double *out, unsigned long long *red, const Scratch &S, hipStream_t s, bool rowio = false,
                   const unsigned long long *stop = nullptr)
{
    // (stop: honoured by the whole-line solver only; the callers pass it for that variant)
    tf::SBParams P{nl, np, bands, rhs, out, S.rel, S.ext, red};
    if (rowio && ((ch.variant != V_PARTITIONED && ch.variant != V_LINE) || !trans || mode != 0))
        return afail(TF_EINVAL, "line-major solves need a transposed MODE 0 partitioned or whole-line solve");
    if (ch.variant == V_LINE) {
        if (!tf::sbline_supported(np)) return afail(TF_EINVAL, "the whole-line solver needs 4 <= n <= 4096");
        TF_AHIP(tf::launch_sbline(trans, !rowio, mode, nl, np, bands, rhs, out, red, s, stop));
        return TF_OK;
    }
    if (ch.variant == V_PCR) {
        if (np > tf::PCR_MAX) return afail(TF_EINVAL, "cyclic reduction needs lines of at most 2048 cells");
        const dim3 g(nl), b(tf::PCR_THREADS);
        if (!trans && mode == 0) tf::k_sb_pcr<false, 0><<<g, b, 0, s>>>(P);
        else if (!trans) tf::k_sb_pcr<false, 1><<<g, b, 0, s>>>(P);
        else if (mode == 0) tf::k_sb_pcr<true, 0><<<g, b, 0, s>>>(P);
        else tf::k_sb_pcr<true, 1><<<g, b, 0, s>>>(P);
        TF_AHIP(hipGetLastError());
        return TF_OK;
    }
    if (ch.variant == V_THOMAS) {
        const int bs = ch.block == 128 || ch.block == 256 ? ch.block : 64;
        const dim3 g((nl + bs - 1) / bs), b(bs);
        if (!trans && mode == 0) tf::k_sb_thomas<false, 0><<<g, b, 0, s>>>(P, S.work);
        else if (!trans) tf::k_sb_thomas<false, 1><<<g, b, 0, s>>>(P, S.work);
        else if (mode == 0) tf::k_sb_thomas<true, 0><<<g, b, 0, s>>>(P, S.work);
        else tf::k_sb_thomas<true, 1><<<g, b, 0, s>>>(P, S.work);
        TF_AHIP(hipGetLastError());
        return TF_OK;
    }
    const int ntile = ((nl + 63) / 64) * tf::seg_count(np);
    const dim3 g(ntile), b(tf::BLOCK);
    if (rowio) tf::k_sb_pass<false, true, 0, true><<<g, b, 0, s>>>(P);
    else if (trans) tf::k_sb_pass<false, true, 0><<<g, b, 0, s>>>(P);
    else tf::k_sb_pass<false, false, 0><<<g, b, 0, s>>>(P);
    TF_AHIP(hipGetLastError());
    tf::ChainParams C{nl, tf::seg_count(np), S.rel, S.chain, S.ext};
    TF_AHIP(tf::launch_chain(C, s));
    if (rowio) tf::k_sb_pass<true, true, 0, true><<<g, b, 0, s>>>(P);
    else if (trans && mode == 0) tf::k_sb_pass<true, true, 0><<<g, b, 0, s>>>(P);
    else if (trans) tf::k_sb_pass<true, true, 1><<<g, b, 0, s>>>(P);
    else if (mode == 0) tf::k_sb_pass<true, false, 0><<<g, b, 0, s>>>(P);
    else tf::k_sb_pass<true, false, 1><<<g, b, 0, s>>>(P);
    TF_AHIP(hipGetLastError());
    return TF_OK;
}

struct AdjBuffers {
    int nx = 0, ny = 0;
    double *bx = nullptr, *by = nullptr, *mu = nullptr, *r = nullptr, *rT = nullptr, *y = nullptr, *yT = nullptr;
    double *dk1 = nullptr, *dk0 = nullptr, *work = nullptr, *part = nullptr;
    double *hpart = nullptr;
    unsigned long long *red = nullptr, *hred = nullptr;
    int last_iters = 0; // Richardson iterations of the previous adjoint step (batch size)
};

std::mutex g_adj_mu;
std::map<const tf_grid *, AdjBuffers> g_adj;

void free_adj(AdjBuffers &b)
{
    double *ps[] = {b.bx, b.by, b.mu, b.r, b.rT, b.y, b.yT, b.dk1, b.dk0, b.work, b.part};
    for (double *p : ps) (void)hipFree(p);
    (void)hipFree(b.red);
    if (b.hpart) (void)hipHostFree(b.hpart);
    if (b.hred) (void)hipHostFree(b.hred);
    b = AdjBuffers{};
}

tf_status get_adj(const tf_grid *g, int nx, int ny, AdjBuffers **out)
{
    std::lock_guard<std::mutex> lk(g_adj_mu);
    AdjBuffers &b = g_adj[g];
    if (b.nx == nx && b.ny == ny && b.bx) {
        *out = &b;
        return TF_OK;
    }
    free_adj(b);
    const size_t N = (size_t)nx * ny;
    bool ok = hipMalloc(&b.bx, 5 * N * sizeof(double)) == hipSuccess && hipMalloc(&b.by, 5 * N * sizeof(double)) == hipSuccess
              && hipMalloc(&b.mu, N * sizeof(double)) == hipSuccess && hipMalloc(&b.r, N * sizeof(double)) == hipSuccess
              && hipMalloc(&b.rT, N * sizeof(double)) == hipSuccess && hipMalloc(&b.y, N * sizeof(double)) == hipSuccess
              && hipMalloc(&b.yT, N * sizeof(double)) == hipSuccess && hipMalloc(&b.dk1, N * sizeof(double)) == hipSuccess
              && hipMalloc(&b.dk0, N * sizeof(double)) == hipSuccess
              && hipMalloc(&b.work, 3 * N * sizeof(double)) == hipSuccess
              && hipMalloc(&b.part, 2 * 4096 * sizeof(double)) == hipSuccess
              && hipMalloc(&b.red, 8 * sizeof(unsigned long long)) == hipSuccess
              && hipHostMalloc(&b.hpart, 2 * 4096 * sizeof(double), hipHostMallocDefault) == hipSuccess
              && hipHostMalloc(&b.hred, 8 * sizeof(unsigned long long), hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_adj(b);
        return afail(TF_ENOMEM, "adjoint scratch allocation failed");
    }
    b.nx = nx;
    b.ny = ny;
    *out = &b;
    return TF_OK;
}

tf_status jdt(const tf_detail::GridView &v, const double *u, const double *mu, const double *lam, double a, double b,
              double gmul, double *out, unsigned long long *clr = nullptr, const unsigned long long *chk = nullptr,
              unsigned long long *ctl = nullptr, double tol = 0.0, int it = 0)
{
    const double ids = 1.0 / v.ds, ids2 = ids * ids;
    const dim3 grid((v.nx + tf::JT_X - 1) / tf::JT_X, (v.ny + tf::JT_Y - 1) / tf::JT_Y), blk(256);
    if (v.M.p32)
        tf::k_jdt<true><<<grid, blk, 0, v.stream>>>(v.nx, v.ny, ids, ids2, v.M, u, mu, lam, a, b, gmul, out, clr, chk,
                                                     ctl, tol, it);
    else
        tf::k_jdt<false><<<grid, blk, 0, v.stream>>>(v.nx, v.ny, ids, ids2, v.M, u, mu, lam, a, b, gmul, out, clr, chk,
                                                      ctl, tol, it);
    TF_AHIP(hipGetLastError());
    return TF_OK;
}

tf_status transpose(int rows, int cols, const double *in, double *out, hipStream_t s)
{
    tf::k_transpose<<<dim3((cols + 63) / 64, (rows + 63) / 64), dim3(256), 0, s>>>(rows, cols, in, out);
    TF_AHIP(hipGetLastError());
    return TF_OK;
}

// Enqueue x . (wa a + wb b) as per-block compensated partials copied to pinned host
// memory; dot_finish combines them after the caller has synchronised the stream.
tf_status dot_enqueue(const double *x, const double *a, const double *b, double wa, double wb, size_t n,
                      AdjBuffers &B, hipStream_t s, size_t *nblocks)
{
    size_t nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    tf::k_dot<<<dim3((unsigned)nb), dim3(256), 0, s>>>(x, a, b, wa, wb, n, B.part);
    TF_AHIP(hipGetLastError());
    TF_AHIP(hipMemcpyAsync(B.hpart, B.part, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
    *nblocks = nb;
    return TF_OK;
}

double dot_finish(const AdjBuffers &B, size_t nb)
{
    double sum = 0.0, c = 0.0;
    for (size_t k = 0; k < nb; ++k) {
        const double p = B.hpart[2 * k], t = sum + p;
        c += (std::fabs(sum) >= std::fabs(p) ? (sum - t) + p : (p - t) + sum) + B.hpart[2 * k + 1];
        sum = t;
    }
    return sum + c;
}

double bits_to_double(unsigned long long x)
{
    double d;
    std::memcpy(&d, &x, sizeof d);
    return d;
}

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string n = p.gcnArchName;
    const size_t c = n.find(':');
    return c == std::string::npos ? n : n.substr(0, c);
}

} // namespace

namespace tf_detail {
void release_adjoint(const tf_grid *g)
{
    std::lock_guard<std::mutex> lk(g_adj_mu);
    auto it = g_adj.find(g);
    if (it != g_adj.end()) {
        free_adj(it->second);
        g_adj.erase(it);
    }
}
} // namespace tf_detail

// ---- scratch of the entry point that allocates nothing --------------------------------
// tf_penta_solve_noalloc takes the interface records (partitioned variant) or the factor
// work array (Thomas variant) from this array instead of hipMalloc. Each GPU the library
// runs on holds its own copy until the process ends; host code reaches it only through the
// device address hipGetSymbolAddress returns (the symbol itself is a host-side stand-in).
static __device__ __align__(256) double scratch[TF_NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {}; // device address of `scratch`, per device

// Device address of the scratch array on the current device (looked up once per device).
tf_status noalloc_scratch(double **out)
{
    int dev = 0;
    TF_AHIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return afail(TF_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[dev] == nullptr) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return afail(TF_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_noalloc_ptr[dev] = (double *)ptr;
    }
    *out = g_noalloc_ptr[dev];
    return TF_OK;
}

// Scratch doubles a solve of nlines lines of n cells needs with a variant.
size_t scratch_need(int variant, int n, int nlines)
{
    const size_t recs = (size_t)tf::seg_count(n) * nlines;
    if (variant == V_PARTITIONED) return recs * (tf::NREL + tf::NEXT + tf::NCHAIN);
    if (variant == V_THOMAS) return 3 * (size_t)n * nlines;
    return 0; // cyclic reduction and the whole-line solver work in LDS
}
} // namespace

extern "C" {

tf_status tf_adjoint_step(tf_grid *g, const double *h_n, const double *h_np1, double dt, double *lambda_inout,
                          double *dL_dkappa_accum, double tol, int max_iter, int *iters_out)
{
    tf_detail::GridView v;
    if (g == nullptr || h_n == nullptr || h_np1 == nullptr || lambda_inout == nullptr)
        return afail(TF_EINVAL, "NULL argument");
    if (!tf_detail::grid_view(g, &v)) return afail(TF_ESTATE, "model not set");
    if (!(dt > 0.0) || !(tol > 0.0) || max_iter < 1) return afail(TF_EINVAL, "need dt > 0, tol > 0, max_iter >= 1");
    if (dL_dkappa_accum != nullptr && v.M.kind != tf::MODEL_POWER)
        return afail(TF_EINVAL, "dL/dkappa is defined for the power-law model only");
    AdjBuffers *Bp;
    tf_status st = get_adj(g, v.nx, v.ny, &Bp);
    if (st != TF_OK) return st;
    AdjBuffers &B = *Bp;
    const int nx = v.nx, ny = v.ny;
    const size_t N = (size_t)nx * ny;
    const double c = v.theta * dt;
    const double ids = 1.0 / v.ds, ids2 = ids * ids;
    const double k1 = c / v.ds, k3 = c / (v.ds * v.ds * v.ds * v.ds);
    hipStream_t s = v.stream;
    // the x solves take the grid's x-sweep variant: whole rows in one kernel (bands of
    // I + c J_x stored [j][i]) or else the tuned stored-band solver without that kernel
    // (bands stored [i][j]); the y solves take the tuned variant
    const bool rowx = v.xsweep == TF_XSWEEP_ROW && tf::sbline_supported(nx);
    // bands of I + c J_x and I + c J_y (stored [j][i]) at u^{n+1}
    {
        const dim3 gy((nx + 63) / 64, (ny + 3) / 4), gx((ny + 63) / 64, (nx + 3) / 4), blk(256);
        if (v.M.p32) {
            tf::k_bands_store<0, true><<<gy, blk, 0, s>>>(nx, ny, ids, ids2, k1, k3, v.M, h_np1, B.by);
            if (rowx) tf::k_bands_store<1, true, true><<<gy, blk, 0, s>>>(nx, ny, ids, ids2, k1, k3, v.M, h_np1, B.bx);
            else tf::k_bands_store<1, true><<<gx, blk, 0, s>>>(nx, ny, ids, ids2, k1, k3, v.M, h_np1, B.bx);
        } else {
            tf::k_bands_store<0, false><<<gy, blk, 0, s>>>(nx, ny, ids, ids2, k1, k3, v.M, h_np1, B.by);
            if (rowx) tf::k_bands_store<1, false, true><<<gy, blk, 0, s>>>(nx, ny, ids, ids2, k1, k3, v.M, h_np1, B.bx);
            else tf::k_bands_store<1, false><<<gx, blk, 0, s>>>(nx, ny, ids, ids2, k1, k3, v.M, h_np1, B.bx);
        }
        TF_AHIP(hipGetLastError());
    }
    Scratch S{v.rel, v.ext, v.chain, B.work};
    Choice vx = pick_variant(nx, ny, true);
    const Choice vy = pick_variant(ny, nx, true);
    if (vx.variant == V_LINE) vx = Choice{};
    // initial guess mu = lambda^{n+1} (the solution for dt -> 0; only the number of
    // iterations depends on it)
    TF_AHIP(hipMemcpyAsync(B.mu, lambda_inout, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    // Iteration i keeps its reduction record {max|z|, max|mu|} in red[2 (i % 2) ..]. When both
    // solves are whole-line kernels, whose launches can stand down on the device, the
    // iterations are enqueued in batches (one more than the previous step needed) and each
    // launch of J_D^T first tests the previous iteration's record (red[4..5]: stop word and
    // converged iteration): the host then waits once per batch instead of once per
    // iteration, and the iterates are those of a test after every iteration.
    const bool batched = rowx && vy.variant == V_LINE;
    unsigned long long *ctl = batched ? B.red + 4 : nullptr;
    if (batched) TF_AHIP(hipMemsetAsync(B.red + 4, 0, 2 * sizeof(unsigned long long), s));
    int it = 0;
    bool conv = false;
    while (it < max_iter && !conv) {
        const int nb = batched ? std::min(std::max(B.last_iters + 1, 2), max_iter - it) : 1;
        for (int k = 1; k <= nb; ++k) {
            const int i = it + k;
            unsigned long long *cur = B.red + 2 * (i & 1), *prev = B.red + 2 * ((i - 1) & 1);
            // r = lambda - (I + c J^T) mu (this kernel also zeroes the iteration's record)
            if ((st = jdt(v, h_np1, B.mu, lambda_inout, 1.0, -1.0, -c, B.r, cur, k > 1 ? prev : nullptr, ctl, tol,
                          i)) != TF_OK)
                return st;
            // (I + c J_x)^-T: rows as lines; the whole-row kernel and the partitioned solver
            // read r and write y row by row, the other variants work on the transposed layout
            if (rowx) {
                if ((st = sb_solve(Choice{V_LINE, 256}, true, 0, ny, nx, B.bx, B.r, B.y, nullptr, S, s, true, ctl)) !=
                    TF_OK)
                    return st;
            } else if (vx.variant == V_PARTITIONED) {
                if ((st = sb_solve(vx, true, 0, ny, nx, B.bx, B.r, B.y, nullptr, S, s, true)) != TF_OK) return st;
            } else {
                if ((st = transpose(ny, nx, B.r, B.rT, s)) != TF_OK) return st;
                if ((st = sb_solve(vx, true, 0, ny, nx, B.bx, B.rT, B.yT, nullptr, S, s)) != TF_OK) return st;
                if ((st = transpose(nx, ny, B.yT, B.y, s)) != TF_OK) return st;
            }
            // (I + c J_y)^-T: columns as lines; mu += z with max|z|, max|mu|
            if ((st = sb_solve(vy, true, 1, nx, ny, B.by, B.y, B.mu, cur, S, s, false, ctl)) != TF_OK) return st;
        }
        const int last = it + nb;
        TF_AHIP(hipMemcpyAsync(B.hred, B.red, 6 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        TF_AHIP(hipStreamSynchronize(s));
        if (batched && B.hred[4] != 0ull) {
            if (B.hred[4] == 2ull) return afail(TF_ENONPOS, "adjoint iteration produced NaN");
            it = (int)B.hred[5];
            conv = true;
            break;
        }
        const unsigned long long *rec = B.hred + 2 * (last & 1);
        const double zmax = bits_to_double(rec[0]), mmax = bits_to_double(rec[1]);
        if (!(zmax == zmax) || !(mmax == mmax)) return afail(TF_ENONPOS, "adjoint iteration produced NaN");
        it = last;
        conv = zmax <= tol * mmax;
    }
    if (conv) B.last_iters = it;
    if (iters_out) *iters_out = conv ? it : max_iter;
    if (!conv) return afail(TF_ENOCONV, "adjoint Richardson iteration did not converge");
    size_t dot_blocks = 0;
    // kappa gradient: dL/dkappa -= dt mu . [theta dD/dk(u^{n+1}) + (1 - theta) dD/dk(u^n)]
    if (dL_dkappa_accum != nullptr) {
        tf::Model Mk = v.M; // f1 with kappa = 1, f0 dropped
        Mk.kappa = 1.0;
        Mk.Cn = v.M.Cn / (v.M.kappa != 0.0 ? v.M.kappa : 1.0);
        Mk.Cm = v.M.Cm / (v.M.kappa != 0.0 ? v.M.kappa : 1.0);
        Mk.Dn = v.M.Dn / (v.M.kappa != 0.0 ? v.M.kappa : 1.0);
        Mk.Dm = v.M.Dm / (v.M.kappa != 0.0 ? v.M.kappa : 1.0);
        if (v.M.kappa == 0.0) {
            const double n = v.M.n, m = v.M.m, b = v.M.b;
            Mk.Cn = n * std::pow(b, n); Mk.Cm = m * std::pow(b, m);
            Mk.Dn = n * (n - 2.0) * std::pow(b, n); Mk.Dm = m * (m - 2.0) * std::pow(b, m);
        }
        TF_AHIP(tf::launch_flux_divergence_f1(nx, ny, ids, ids2, Mk, h_np1, B.dk1, s));
        if (v.theta < 1.0) TF_AHIP(tf::launch_flux_divergence_f1(nx, ny, ids, ids2, Mk, h_n, B.dk0, s));
        if ((st = dot_enqueue(B.mu, B.dk1, v.theta < 1.0 ? B.dk0 : nullptr, v.theta, 1.0 - v.theta, N, B, s,
                              &dot_blocks)) != TF_OK)
            return st;
    }
    // lambda^n = mu - (1 - theta) dt J_D(u^n)^T mu
    if (v.theta < 1.0) {
        if ((st = jdt(v, h_n, B.mu, nullptr, 0.0, 1.0, -(1.0 - v.theta) * dt, lambda_inout)) != TF_OK) return st;
    } else {
        TF_AHIP(hipMemcpyAsync(lambda_inout, B.mu, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    TF_AHIP(hipStreamSynchronize(s));
    if (dot_blocks > 0) *dL_dkappa_accum -= dt * dot_finish(B, dot_blocks);
    return TF_OK;
}

tf_status tf_adjoint_steps(tf_grid *g, int nsteps, const double *const *states, double dt, double *lambda_inout,
                           double *dL_dkappa_accum, double tol, int max_iter, int *iters_out)
{
    if (g == nullptr || nsteps < 0 || (nsteps > 0 && states == nullptr) || lambda_inout == nullptr)
        return afail(TF_EINVAL, "bad argument");
    int total = 0;
    tf_status st = TF_OK;
    for (int s = nsteps - 1; s >= 0 && st == TF_OK; --s) {
        int it = 0;
        st = tf_adjoint_step(g, states[s], states[s + 1], dt, lambda_inout, dL_dkappa_accum, tol, max_iter, &it);
        total += it;
    }
    if (iters_out) *iters_out = total;
    return st;
}

tf_status tf_jacobian_apply_t(tf_grid *g, const double *u, const double *mu, double *out)
{
    tf_detail::GridView v;
    if (g == nullptr || u == nullptr || mu == nullptr || out == nullptr) return afail(TF_EINVAL, "NULL argument");
    if (!tf_detail::grid_view(g, &v)) return afail(TF_ESTATE, "model not set");
    tf_status st;
    if ((st = jdt(v, u, mu, nullptr, 0.0, 0.0, 1.0, out)) != TF_OK) return st;
    TF_AHIP(hipStreamSynchronize(v.stream));
    return TF_OK;
}

tf_status tf_penta_solve(int nlines, int n, const double *bands, const double *rhs, double *x, int transposed,
                         int variant, void *stream)
{
    if (nlines < 1 || n < 2 || bands == nullptr || rhs == nullptr || x == nullptr || variant < -1 || variant > 3)
        return afail(TF_EINVAL, "bad argument");
    if (variant == V_PCR && n > tf::PCR_MAX) return afail(TF_EINVAL, "cyclic reduction needs n <= 2048");
    if (variant == V_LINE && !tf::sbline_supported(n)) return afail(TF_EINVAL, "the whole-line solver needs 4 <= n <= 4096");
    hipStream_t s = (hipStream_t)stream;
    const size_t recs = (size_t)tf::seg_count(n) * nlines;
    Scratch S;
    bool ok = hipMalloc(&S.rel, recs * tf::NREL * sizeof(double)) == hipSuccess
              && hipMalloc(&S.ext, recs * tf::NEXT * sizeof(double)) == hipSuccess
              && hipMalloc(&S.chain, recs * tf::NCHAIN * sizeof(double)) == hipSuccess
              && hipMalloc(&S.work, 3 * (size_t)n * nlines * sizeof(double)) == hipSuccess;
    tf_status st = TF_OK;
    if (!ok) st = afail(TF_ENOMEM, "scratch allocation failed");
    if (st == TF_OK) {
        Choice c;
        if (variant < 0) c = pick_variant(n, nlines, transposed != 0);
        else c.variant = variant;
        st = sb_solve(c, transposed != 0, 0, nlines, n, bands, rhs, x, nullptr, S, s);
        if (st == TF_OK && hipStreamSynchronize(s) != hipSuccess) st = afail(TF_EDEVICE, "synchronize failed");
    }
    (void)hipFree(S.rel);
    (void)hipFree(S.ext);
    (void)hipFree(S.chain);
    (void)hipFree(S.work);
    return st;
}

tf_status tf_penta_solve_noalloc(int nlines, int n, const double *bands, const double *rhs, double *x,
                                 int transposed, int variant, void *stream)
{
    if (nlines < 1 || n < 2 || bands == nullptr || rhs == nullptr || x == nullptr || variant < -1 || variant > 3)
        return afail(TF_EINVAL, "bad argument");
    if (variant == V_PCR && n > tf::PCR_MAX) return afail(TF_EINVAL, "cyclic reduction needs n <= 2048");
    if (variant == V_LINE && !tf::sbline_supported(n)) return afail(TF_EINVAL, "the whole-line solver needs 4 <= n <= 4096");
    Choice c;
    if (variant < 0) {
        c = pick_variant(n, nlines, transposed != 0);
        // an automatic choice that does not fit the scratch array falls back to one that does
        if (scratch_need(c.variant, n, nlines) > (size_t)TF_NOALLOC_SCRATCH_DOUBLES) {
            if (n <= tf::PCR_MAX) c.variant = V_PCR;
            else c.variant = V_PARTITIONED;
        }
    } else {
        c.variant = variant;
    }
    const size_t need = scratch_need(c.variant, n, nlines);
    if (need > (size_t)TF_NOALLOC_SCRATCH_DOUBLES)
        return afail(TF_EINVAL, "the solve needs " + std::to_string(need) + " doubles of scratch; the no-allocation "
                                "entry point holds " + std::to_string((size_t)TF_NOALLOC_SCRATCH_DOUBLES));
    double *base = nullptr;
    tf_status st = noalloc_scratch(&base);
    if (st != TF_OK) return st;
    const size_t recs = (size_t)tf::seg_count(n) * nlines;
    Scratch S;
    S.rel = base;
    S.ext = base + recs * tf::NREL;
    S.chain = base + recs * (tf::NREL + tf::NEXT);
    S.work = base;
    return sb_solve(c, transposed != 0, 0, nlines, n, bands, rhs, x, nullptr, S, (hipStream_t)stream);
}

tf_status tf_autotune(int length, int batch, int transposed, const char *cache_path)
{
    if (length < 2 || batch < 1) return afail(TF_EINVAL, "need length >= 2 and batch >= 1");
    const size_t N = (size_t)length * batch;
    double *bands = nullptr, *rhs = nullptr, *x = nullptr;
    Scratch S;
    const size_t recs = (size_t)tf::seg_count(length) * batch;
    hipStream_t s = nullptr;
    bool ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess
              && hipMalloc(&bands, 5 * N * sizeof(double)) == hipSuccess && hipMalloc(&rhs, N * sizeof(double)) == hipSuccess
              && hipMalloc(&x, N * sizeof(double)) == hipSuccess
              && hipMalloc(&S.rel, recs * tf::NREL * sizeof(double)) == hipSuccess
              && hipMalloc(&S.ext, recs * tf::NEXT * sizeof(double)) == hipSuccess
              && hipMalloc(&S.chain, recs * tf::NCHAIN * sizeof(double)) == hipSuccess
              && hipMalloc(&S.work, 3 * N * sizeof(double)) == hipSuccess;
    tf_status st = ok ? TF_OK : afail(TF_ENOMEM, "autotune allocation failed");
    // candidates: partitioned; Thomas with 64, 128, 256 lines per block; cyclic reduction
    // (lines of at most PCR_MAX cells); whole lines in one kernel (lines of 4 ..= 4096 cells)
    std::vector<Choice> cands;
    std::vector<std::string> names;
    cands.push_back({V_PARTITIONED, 64});
    names.push_back("partitioned");
    for (int bs : {64, 128, 256}) {
        cands.push_back({V_THOMAS, bs});
        names.push_back("thomas/" + std::to_string(bs));
    }
    if (length <= tf::PCR_MAX) {
        cands.push_back({V_PCR, tf::PCR_THREADS});
        names.push_back("pcr");
    }
    if (tf::sbline_supported(length)) {
        cands.push_back({V_LINE, 256});
        names.push_back("line");
    }
    std::vector<double> ms(cands.size(), 1e30);
    if (st == TF_OK) {
        tf::k_fill_test<<<dim3(1024), dim3(256), 0, s>>>(N, bands, rhs);
        hipEvent_t a, b;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        for (size_t v = 0; v < cands.size() && st == TF_OK; ++v) {
            std::vector<float> t;
            for (int r = 0; r < 6 && st == TF_OK; ++r) {
                (void)hipEventRecord(a, s);
                st = sb_solve(cands[v], transposed != 0, 0, batch, length, bands, rhs, x, nullptr, S, s);
                (void)hipEventRecord(b, s);
                (void)hipEventSynchronize(b);
                float e = 0.0f;
                (void)hipEventElapsedTime(&e, a, b);
                if (r > 0) t.push_back(e); // first run is a warm-up
            }
            std::sort(t.begin(), t.end());
            ms[v] = t.empty() ? 1e30 : t[t.size() / 2];
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    (void)hipFree(bands);
    (void)hipFree(rhs);
    (void)hipFree(x);
    (void)hipFree(S.rel);
    (void)hipFree(S.ext);
    (void)hipFree(S.chain);
    (void)hipFree(S.work);
    if (s) (void)hipStreamDestroy(s);
    if (st != TF_OK) return st;
    size_t best = 0;
    for (size_t v = 1; v < cands.size(); ++v)
        if (ms[v] < ms[best]) best = v;
    {
        TuneTable &t = tune_table();
        std::lock_guard<std::mutex> lk(t.mu);
        t.best[{length, batch, transposed != 0}] = cands[best];
    }
    if (cache_path != nullptr && cache_path[0] != '\0') {
        // one JSON object per line: {"arch", "length", "batch", "transposed", "variant", "block", "ms": {...}}
        std::ofstream f(cache_path, std::ios::app);
        if (!f) return afail(TF_EINVAL, std::string("cannot write ") + cache_path);
        std::ostringstream o;
        o << "{\"arch\": \"" << arch_name() << "\", \"length\": " << length << ", \"batch\": " << batch
          << ", \"transposed\": " << (transposed != 0 ? 1 : 0) << ", \"variant\": \"" << kVariantNames[cands[best].variant] << "\", \"block\": " << cands[best].block
          << ", \"ms\": {";
        char buf[64];
        for (size_t v = 0; v < cands.size(); ++v) {
            std::snprintf(buf, sizeof buf, "%.6f", ms[v]);
            o << (v ? ", " : "") << "\"" << names[v] << "\": " << buf;
        }
        o << "}}\n";
        f << o.str();
    }
    return TF_OK;
}

tf_status tf_autotune_xsweep(int length, int batch, const char *cache_path)
{
    if (length < 4 || batch < 4) return afail(TF_EINVAL, "need length >= 4 and batch >= 4");
    const size_t N = (size_t)length * batch;
    const size_t recs = (size_t)tf::seg_count(length) * batch;
    double *u = nullptr, *w = nullptr, *out = nullptr, *rel = nullptr, *ext = nullptr, *chain = nullptr;
    unsigned long long *res = nullptr;
    hipStream_t s = nullptr;
    bool ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess
              && hipMalloc(&u, N * sizeof(double)) == hipSuccess && hipMalloc(&w, N * sizeof(double)) == hipSuccess
              && hipMalloc(&out, N * sizeof(double)) == hipSuccess
              && hipMalloc(&rel, recs * tf::NREL * sizeof(double)) == hipSuccess
              && hipMalloc(&ext, recs * tf::NEXT * sizeof(double)) == hipSuccess
              && hipMalloc(&chain, recs * tf::NCHAIN * sizeof(double)) == hipSuccess
              && hipMalloc(&res, tf::RES_SPREAD * tf::RES_WORDS * sizeof(unsigned long long)) == hipSuccess;
    tf_status st = ok ? TF_OK : afail(TF_ENOMEM, "autotune allocation failed");
    // the n = 3, m = 2 power law of the benchmark films (kappa = 10, b = 0.1), ds = 0.67347,
    // backward Euler dt = 0.2
    tf::Model M{};
    M.kappa = 10.0; M.b = 0.1; M.n = 3; M.m = 2;
    M.Cn = 10.0 * 3.0 * 1e-3; M.Cm = 10.0 * 2.0 * 1e-2; M.Dn = 10.0 * 3.0 * 1.0 * 1e-3; M.Dm = 0.0;
    M.p32 = true; M.kind = tf::MODEL_POWER; M.cap = 1.0;
    tf::PassParams P{};
    const double ds = 0.67347, dt = 0.2;
    P.nx = length; P.ny = batch;
    P.ids2 = 1.0 / (ds * ds);
    P.f0s = P.ids2;
    P.ka = 0.5 * dt * P.ids2;
    P.K0 = 3.0 * P.ka * P.ids2;
    P.K1 = P.ka * M.Dn;
    P.M = M;
    P.res_spread = tf::RES_SPREAD;
    P.u = u; P.in2 = w; P.out = out; P.rel = rel; P.ext = ext; P.res = res;
    P.tiles_x = tf::seg_count(length);
    P.tiles_y = (batch + tf::TILE - 1) / tf::TILE;
    const tf::ChainParams C{batch, tf::seg_count(length), rel, chain, ext};
    auto run = [&](int v) -> hipError_t {
        if (v == 1) return tf::launch_xrow(P, s);
        tf::PassParams Q = P;
        Q.res = nullptr;
        hipError_t e = tf::launch_pass(1, false, Q, s);
        if (e == hipSuccess) e = tf::launch_chain(C, s);
        if (e == hipSuccess) e = tf::launch_pass(1, true, P, s);
        return e;
    };
    const int nv = tf::xrow_supported(length) ? 2 : 1;
    const char *names[2] = {"partitioned", "row"};
    double ms[2] = {1e30, 1e30};
    if (st == TF_OK) {
        tf::k_fill_film<<<dim3(1024), dim3(256), 0, s>>>(N, u, w);
        (void)hipMemsetAsync(res, 0, tf::RES_SPREAD * tf::RES_WORDS * sizeof(unsigned long long), s);
        hipEvent_t a, b;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        for (int v = 0; v < nv && st == TF_OK; ++v) {
            std::vector<float> t;
            for (int r = 0; r < 6 && st == TF_OK; ++r) {
                (void)hipEventRecord(a, s);
                const hipError_t e = run(v);
                (void)hipEventRecord(b, s);
                if (e != hipSuccess) {
                    st = afail(TF_EDEVICE, std::string("x-sweep launch: ") + hipGetErrorString(e));
                    break;
                }
                (void)hipEventSynchronize(b);
                float el = 0.0f;
                (void)hipEventElapsedTime(&el, a, b);
                if (r > 0) t.push_back(el); // first run is a warm-up
            }
            std::sort(t.begin(), t.end());
            ms[v] = t.empty() ? 1e30 : t[t.size() / 2];
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (st == TF_OK && hipStreamSynchronize(s) != hipSuccess) st = afail(TF_EDEVICE, "x-sweep timing failed");
    }
    (void)hipFree(u);
    (void)hipFree(w);
    (void)hipFree(out);
    (void)hipFree(rel);
    (void)hipFree(ext);
    (void)hipFree(chain);
    (void)hipFree(res);
    if (s) (void)hipStreamDestroy(s);
    if (st != TF_OK) return st;
    const int best = (nv > 1 && ms[1] < ms[0]) ? 1 : 0;
    {
        TuneTable &t = tune_table();
        std::lock_guard<std::mutex> lk(t.mu);
        Choice c;
        c.variant = best;
        t.best[{length, batch, XSWEEP_KIND}] = c;
    }
    if (cache_path != nullptr && cache_path[0] != '\0') {
        std::ofstream f(cache_path, std::ios::app);
        if (!f) return afail(TF_EINVAL, std::string("cannot write ") + cache_path);
        std::ostringstream o;
        o << "{\"arch\": \"" << arch_name() << "\", \"kind\": \"xsweep\", \"length\": " << length
          << ", \"batch\": " << batch << ", \"variant\": \"" << names[best] << "\", \"ms\": {";
        char buf[64];
        for (int v = 0; v < nv; ++v) {
            std::snprintf(buf, sizeof buf, "%.6f", ms[v]);
            o << (v ? ", " : "") << "\"" << names[v] << "\": " << buf;
        }
        o << "}}\n";
        f << o.str();
    }
    return TF_OK;
}

int tf_xsweep_choice(int nx, int ny) { return tf::xsweep_choice(nx, ny); }

tf_status tf_autotune_load(const char *cache_path)
{
    if (cache_path == nullptr) return afail(TF_EINVAL, "NULL path");
    std::ifstream f(cache_path);
    if (!f) return afail(TF_EINVAL, std::string("cannot read ") + cache_path);
    const std::string arch = arch_name();
    std::string line;
    int loaded = 0;
    TuneTable &t = tune_table();
    std::lock_guard<std::mutex> lk(t.mu);
    while (std::getline(f, line)) {
        auto field = [&](const char *key) -> std::string {
            const std::string k = std::string("\"") + key + "\": ";
            const size_t p = line.find(k);
            if (p == std::string::npos) return "";
            size_t q = p + k.size();
            if (line[q] == '"') {
                const size_t e = line.find('"', q + 1);
                return line.substr(q + 1, e - q - 1);
            }
            size_t e = q;
            while (e < line.size() && (std::isdigit((unsigned char)line[e]) || line[e] == '-')) ++e;
            return line.substr(q, e - q);
        };
        if (field("arch") != arch) continue;
        const std::string L = field("length"), Bt = field("batch"), V = field("variant"), Bs = field("block");
        const std::string Tr = field("transposed");
        if (L.empty() || Bt.empty()) continue;
        Choice c;
        if (field("kind") == "xsweep") {
            c.variant = V == "row" ? 1 : 0;
            t.best[{std::stoi(L), std::stoi(Bt), XSWEEP_KIND}] = c;
            ++loaded;
            continue;
        }
        c.variant = V == "thomas" ? V_THOMAS : (V == "pcr" ? V_PCR : (V == "line" ? V_LINE : V_PARTITIONED));
        c.block = Bs.empty() ? 64 : std::stoi(Bs);
        t.best[{std::stoi(L), std::stoi(Bt), Tr.empty() ? 0 : (std::stoi(Tr) != 0)}] = c;
        ++loaded;
    }
    return loaded > 0 ? TF_OK : afail(TF_EINVAL, "no entries for this GPU architecture in the cache");
}

int tf_autotune_choice(int length, int batch, int transposed)
{
    return pick_variant(length, batch, transposed != 0).variant;
}

} // extern "C"
