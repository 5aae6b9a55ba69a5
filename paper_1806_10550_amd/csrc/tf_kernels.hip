// HIP kernels (gfx950, FP64) of the ADI-Newton thin-film step.
//
// One Newton iteration (Lam, Cummings & Kondic, arXiv:1806.10550, eqs.
// JacobianSystem1-3) is two line sweeps:
//   y sweep: (I + c J_y(u_k)) w = -G(u_k)      one pentadiagonal system per grid column
//   x sweep: (I + c J_x(u_k)) v = w            one pentadiagonal system per grid row
//            u_{k+1} = u_k + v, e = max|v/u_k| (eq. NewtonError)
// Every sweep is a partitioned (SPIKE-like) solve in three kernels:
//   k_pass<.., SOLVE=false>  per 64x64 tile: stage u in LDS, assemble coefficients,
//                            residual and bands in registers, eliminate each line
//                            segment with its outer unknowns kept symbolic, and emit
//                            the segment's boundary relations (20 doubles per line);
//   k_chain                  per line: solve the small block system that couples
//                            neighbouring segments (2 unknowns on each side);
//   k_pass<.., SOLVE=true>   per tile: redo the elimination with the factors held in
//                            registers, plug in the segment's outer unknowns and
//                            back-substitute; write w (y sweep) or u_{k+1} (x sweep).
// No band matrix is ever stored: coefficients are recomputed from the u tile.
#include "tf_internal.h"

namespace tf {

// Reciprocal from the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r); accurate to about one ulp for normal x.
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

__device__ __forceinline__ double ipow(double r, double h, int k)
{
    const double base = k >= 0 ? r : h;
    const int e = k >= 0 ? k : -k;
    double acc = 1.0;
    for (int i = 0; i < e; ++i) acc *= base;
    return acc;
}

// f0 = h^3, f0' = 3h^2, f1 = kappa h^3 f'(h), f1' (see Model).
template <bool P32>
__device__ __forceinline__ void model_coefs(const Model &M, double u, double &f0, double &f1,
                                            double &f0p, double &f1p)
{
    const double r = rcp(u);
    const double u2 = u * u;
    f0 = u2 * u;
    f0p = 3.0 * u2;
    if (P32) {
        f1 = M.Cm - M.Cn * r;
        f1p = M.Dn * (r * r);
    } else {
        f1 = M.Cm * ipow(r, u, M.m - 2) - M.Cn * ipow(r, u, M.n - 2);
        f1p = M.Dn * ipow(r, u, M.n - 1) - M.Dm * ipow(r, u, M.m - 1);
    }
}

struct Cell {
    double u, lap, f0, f1, f0p, f1p;
};

// Even reflection across the boundary faces (no-flux ghosts), clamped so that a
// ragged tile never reads outside the grid.
__device__ __forceinline__ int crefl(int k, int n)
{
    if (k < 0) k = -1 - k;
    if (k >= n) k = 2 * n - 1 - k;
    return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

// LDS u tile: (line l, position p) in tile-local coordinates, -HALO <= l, p < TILE+HALO.
// DIR 0 (y sweep): lines are grid columns (x), positions rows (y).
// DIR 1 (x sweep): lines are grid rows (y), positions columns (x).
template <int DIR>
__device__ __forceinline__ double uat(const double *sU, int l, int p)
{
    return DIR == 0 ? sU[(p + HALO) * UPITCH + (l + HALO)] : sU[(l + HALO) * UPITCH + (p + HALO)];
}

template <int DIR, bool P32>
__device__ __forceinline__ Cell cell_at(const double *sU, const Model &M, double ids2, int l, int p)
{
    Cell c;
    c.u = uat<DIR>(sU, l, p);
    double xp, xm, yp, ym;
    if (DIR == 0) {
        xp = uat<DIR>(sU, l + 1, p); xm = uat<DIR>(sU, l - 1, p);
        yp = uat<DIR>(sU, l, p + 1); ym = uat<DIR>(sU, l, p - 1);
    } else {
        xp = uat<DIR>(sU, l, p + 1); xm = uat<DIR>(sU, l, p - 1);
        yp = uat<DIR>(sU, l + 1, p); ym = uat<DIR>(sU, l - 1, p);
    }
    c.lap = (xp + xm + yp + ym - 4.0 * c.u) * ids2;
    model_coefs<P32>(M, c.u, c.f0, c.f1, c.f0p, c.f1p);
    return c;
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous run
// of tiles so that neighbouring tiles share halos in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// ---- 2x2 / 2x5 helpers for the interface chain --------------------------------------
struct M2 { double a, b, c, d; }; // [[a b] [c d]]

__device__ __forceinline__ M2 mul(const M2 &x, const M2 &y)
{
    return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}
__device__ __forceinline__ M2 inv_i_minus(const M2 &x) // (I - x)^-1
{
    const double a = 1.0 - x.a, b = -x.b, c = -x.c, d = 1.0 - x.d;
    const double r = rcp(a * d - b * c);
    return {d * r, -b * r, -c * r, a * r};
}

// Relation record of one segment for one line: with (l1, l2) the two cells before the
// segment and (r1, r2) the two cells after it,
//   top pair    T[i] = T[i][0] + T[i][1] l1 + T[i][2] l2 + T[i][3] r1 + T[i][4] r2
//   bottom pair B[i] = ...
// stored as NREL doubles: T[0][0..4], T[1][0..4], B[0][0..4], B[1][0..4].
struct Rel {
    double T[2][5], B[2][5];
};

// Numeric interface chain over Q segments with outer boundary values (l, r):
// eliminates forward keeping T_q = tau_q + N_q T_{q+1}, B_q = bt_q + M_q T_{q+1}.
// Outputs the boundary values of every segment: lo[q] = B_{q-1}, hi[q] = T_{q+1}.
template <int QMAX>
__device__ __forceinline__ void chain_numeric(const Rel *R, int Q, double l1, double l2, double r1,
                                              double r2, double lo[QMAX][2], double hi[QMAX][2])
{
    double tau[QMAX][2], bt[QMAX][2];
    M2 N[QMAX], Mm[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        if (q >= Q) break;
        const Rel &S = R[q];
        const M2 Tl = {S.T[0][1], S.T[0][2], S.T[1][1], S.T[1][2]};
        const M2 Tr = {S.T[0][3], S.T[0][4], S.T[1][3], S.T[1][4]};
        const M2 Bl = {S.B[0][1], S.B[0][2], S.B[1][1], S.B[1][2]};
        const M2 Br = {S.B[0][3], S.B[0][4], S.B[1][3], S.B[1][4]};
        if (q == 0) {
            tau[0][0] = S.T[0][0] + Tl.a * l1 + Tl.b * l2;
            tau[0][1] = S.T[1][0] + Tl.c * l1 + Tl.d * l2;
            N[0] = Tr;
            bt[0][0] = S.B[0][0] + Bl.a * l1 + Bl.b * l2;
            bt[0][1] = S.B[1][0] + Bl.c * l1 + Bl.d * l2;
            Mm[0] = Br;
        } else {
            const M2 K = inv_i_minus(mul(Tl, Mm[q - 1]));
            const double s0 = S.T[0][0] + Tl.a * bt[q - 1][0] + Tl.b * bt[q - 1][1];
            const double s1 = S.T[1][0] + Tl.c * bt[q - 1][0] + Tl.d * bt[q - 1][1];
            tau[q][0] = K.a * s0 + K.b * s1;
            tau[q][1] = K.c * s0 + K.d * s1;
            N[q] = mul(K, Tr);
            const M2 &Mp = Mm[q - 1];
            const double v0 = bt[q - 1][0] + Mp.a * tau[q][0] + Mp.b * tau[q][1];
            const double v1 = bt[q - 1][1] + Mp.c * tau[q][0] + Mp.d * tau[q][1];
            bt[q][0] = S.B[0][0] + Bl.a * v0 + Bl.b * v1;
            bt[q][1] = S.B[1][0] + Bl.c * v0 + Bl.d * v1;
            const M2 BM = mul(mul(Bl, Mp), N[q]);
            Mm[q] = {BM.a + Br.a, BM.b + Br.b, BM.c + Br.c, BM.d + Br.d};
        }
    }
    double tn0 = r1, tn1 = r2;
#pragma unroll
    for (int q = QMAX - 1; q >= 0; --q) {
        if (q >= Q) continue;
        hi[q][0] = tn0;
        hi[q][1] = tn1;
        const double t0 = tau[q][0] + N[q].a * tn0 + N[q].b * tn1;
        const double t1 = tau[q][1] + N[q].c * tn0 + N[q].d * tn1;
        if (q + 1 < Q) {
            lo[q + 1][0] = bt[q][0] + Mm[q].a * tn0 + Mm[q].b * tn1;
            lo[q + 1][1] = bt[q][1] + Mm[q].c * tn0 + Mm[q].d * tn1;
        }
        tn0 = t0;
        tn1 = t1;
    }
    lo[0][0] = l1;
    lo[0][1] = l2;
}

// Symbolic interface chain over Q sub-segments: returns the relation record of the
// whole segment (top pair of the first sub-segment, bottom pair of the last) in terms
// of the segment's outer boundary values.
template <int QMAX>
__device__ __forceinline__ void chain_symbolic(const Rel *R, int Q, Rel &out)
{
    // forms over (1, l1, l2, r1, r2)
    double tau[QMAX][2][5], bt[QMAX][2][5];
    M2 N[QMAX], Mm[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        if (q >= Q) break;
        const Rel &S = R[q];
        const M2 Tl = {S.T[0][1], S.T[0][2], S.T[1][1], S.T[1][2]};
        const M2 Tr = {S.T[0][3], S.T[0][4], S.T[1][3], S.T[1][4]};
        const M2 Bl = {S.B[0][1], S.B[0][2], S.B[1][1], S.B[1][2]};
        const M2 Br = {S.B[0][3], S.B[0][4], S.B[1][3], S.B[1][4]};
        if (q == 0) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                tau[0][i][0] = S.T[i][0]; tau[0][i][1] = S.T[i][1]; tau[0][i][2] = S.T[i][2];
                tau[0][i][3] = 0.0; tau[0][i][4] = 0.0;
                bt[0][i][0] = S.B[i][0]; bt[0][i][1] = S.B[i][1]; bt[0][i][2] = S.B[i][2];
                bt[0][i][3] = 0.0; bt[0][i][4] = 0.0;
            }
            N[0] = Tr;
            Mm[0] = Br;
        } else {
            const M2 K = inv_i_minus(mul(Tl, Mm[q - 1]));
            double s[2][5];
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                s[0][j] = (j == 0 ? S.T[0][0] : 0.0) + Tl.a * bt[q - 1][0][j] + Tl.b * bt[q - 1][1][j];
                s[1][j] = (j == 0 ? S.T[1][0] : 0.0) + Tl.c * bt[q - 1][0][j] + Tl.d * bt[q - 1][1][j];
            }
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                tau[q][0][j] = K.a * s[0][j] + K.b * s[1][j];
                tau[q][1][j] = K.c * s[0][j] + K.d * s[1][j];
            }
            N[q] = mul(K, Tr);
            const M2 &Mp = Mm[q - 1];
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                const double v0 = bt[q - 1][0][j] + Mp.a * tau[q][0][j] + Mp.b * tau[q][1][j];
                const double v1 = bt[q - 1][1][j] + Mp.c * tau[q][0][j] + Mp.d * tau[q][1][j];
                bt[q][0][j] = (j == 0 ? S.B[0][0] : 0.0) + Bl.a * v0 + Bl.b * v1;
                bt[q][1][j] = (j == 0 ? S.B[1][0] : 0.0) + Bl.c * v0 + Bl.d * v1;
            }
            const M2 BM = mul(mul(Bl, Mp), N[q]);
            Mm[q] = {BM.a + Br.a, BM.b + Br.b, BM.c + Br.c, BM.d + Br.d};
        }
    }
    // T_{Q} is the outer right pair: the form (r1, r2)
    double tn[2][5] = {{0, 0, 0, 1, 0}, {0, 0, 0, 0, 1}};
#pragma unroll
    for (int q = QMAX - 1; q >= 0; --q) {
        if (q >= Q) continue;
        if (q == Q - 1) {
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                out.B[0][j] = bt[q][0][j] + Mm[q].a * tn[0][j] + Mm[q].b * tn[1][j];
                out.B[1][j] = bt[q][1][j] + Mm[q].c * tn[0][j] + Mm[q].d * tn[1][j];
            }
        }
        double t[2][5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            t[0][j] = tau[q][0][j] + N[q].a * tn[0][j] + N[q].b * tn[1][j];
            t[1][j] = tau[q][1][j] + N[q].c * tn[0][j] + N[q].d * tn[1][j];
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            tn[0][j] = t[0][j];
            tn[1][j] = t[1][j];
        }
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        out.T[0][j] = tn[0][j];
        out.T[1][j] = tn[1][j];
    }
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ unsigned wave_or(unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

// ------------------------------------------------------------------------------------
// Tile pass. DIR 0: y sweep (columns), DIR 1: x sweep (rows). SOLVE false: emit the
// tile's segment relations; SOLVE true: finish the solve with the chained boundaries.
// ------------------------------------------------------------------------------------
template <int DIR, bool SOLVE, bool P32>
__global__ void __launch_bounds__(BLOCK) k_pass(PassParams p)
{
    __shared__ double sU[TW * UPITCH];
    __shared__ double sB[NSUB * NREL * 64];
    __shared__ double sRed[NSUB][2];
    __shared__ unsigned sFlag[NSUB];
    static_assert(NSUB * NREL * 64 >= TILE * WPITCH, "second LDS region too small");

    const int nx = p.nx, ny = p.ny;
    const int ntiles = p.tiles_x * p.tiles_y;
    const int t = xcd_tile(blockIdx.x, ntiles);
    const int tx = t % p.tiles_x, ty = t / p.tiles_x;
    const int x0 = seg_start(tx, nx), x1 = seg_start(tx + 1, nx);
    const int y0 = seg_start(ty, ny), y1 = seg_start(ty + 1, ny);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    if (p.res_clear != nullptr && blockIdx.x == 0 && tid < RES_WORDS) p.res_clear[tid] = 0ull;

    for (int idx = tid; idx < TW * TW; idx += BLOCK) {
        const int ly = idx / TW, lx = idx - ly * TW;
        const int gx = crefl(x0 - HALO + lx, nx), gy = crefl(y0 - HALO + ly, ny);
        sU[ly * UPITCH + lx] = p.u[(size_t)gy * nx + gx];
    }
    for (int idx = tid; idx < TILE * TILE; idx += BLOCK) {
        const int ly = idx >> 6, lx = idx & 63;
        const int gx = min(x0 + lx, nx - 1), gy = min(y0 + ly, ny - 1);
        sB[ly * WPITCH + lx] = p.in2[(size_t)gy * nx + gx];
    }
    __syncthreads();

    const int lbase = DIR == 0 ? x0 : y0;
    const int nlt = DIR == 0 ? x1 - x0 : y1 - y0;   // lines in this tile
    const int pbase = DIR == 0 ? y0 : x0;
    const int npos = DIR == 0 ? y1 - y0 : x1 - x0;  // segment length
    const int Nl = DIR == 0 ? nx : ny;
    const int Np = DIR == 0 ? ny : nx;
    const int qseg = DIR == 0 ? ty : tx;
    const int gl = lbase + lane;
    const bool active = lane < nlt;
    const int nsub = min(NSUB, npos / 2);
    const int ps = (wave * npos) / nsub;
    const int len = wave < nsub ? ((wave + 1) * npos) / nsub - ps : 0;
    const double ids = p.ids, ids2 = p.ids2, k1 = p.k1, k3 = p.k3;

    double fa[SUB], fb[SUB], fz[SUB], fph[SUB], fps[SUB], fu[SUB];
    Rel mine;
    double rmax = 0.0;
    unsigned flags = 0;

    if (len > 0) {
        Cell cm = cell_at<DIR, P32>(sU, p.M, ids2, lane, ps - 1);
        Cell c0 = cell_at<DIR, P32>(sU, p.M, ids2, lane, ps);
        double al1 = 0.0, be1 = 0.0, al2 = 0.0, be2 = 0.0;
        // rows s-2 and s-1 stand for the outer unknowns l1 and l2
        double z1 = 0.0, ph1 = 0.0, ps1 = 1.0, z2 = 0.0, ph2 = 1.0, ps2 = 0.0;
        double g1 = 0.0, g2 = 0.0, h1 = 0.0, h2 = 0.0;
        double sgz = 0.0, sgph = 0.0, sgps = 0.0, shz = 0.0, shph = 0.0, shps = 0.0;
#pragma unroll
        for (int k = 0; k < SUB; ++k) {
            if (k < len) {
                const int lp = ps + k;
                const int gp = pbase + lp;
                const Cell cp = cell_at<DIR, P32>(sU, p.M, ids2, lane, lp + 1);
                const bool fm = gp > 0, fpl = gp < Np - 1;
                // faces lp-1/2 (m) and lp+1/2 (p) along the line: mean coefficients,
                // full-Laplacian and value differences
                const double Am = 0.5 * (cm.f0 + c0.f0), Bm = 0.5 * (cm.f1 + c0.f1);
                const double Ap = 0.5 * (c0.f0 + cp.f0), Bp = 0.5 * (c0.f1 + cp.f1);
                const double Lm = (c0.lap - cm.lap) * ids, Gm = (c0.u - cm.u) * ids;
                const double Lp = (cp.lap - c0.lap) * ids, Gp = (cp.u - c0.u) * ids;
                double rhs;
                if (DIR == 0) {
                    // residual -G(u_k) = -(u_k - b^n + theta dt D(u_k)); D uses the x
                    // faces of this cell too
                    const Cell aw = cell_at<DIR, P32>(sU, p.M, ids2, lane - 1, lp);
                    const Cell ae = cell_at<DIR, P32>(sU, p.M, ids2, lane + 1, lp);
                    const double Fw = gl > 0 ? 0.5 * (aw.f0 + c0.f0) * ((c0.lap - aw.lap) * ids)
                                                   + 0.5 * (aw.f1 + c0.f1) * ((c0.u - aw.u) * ids)
                                             : 0.0;
                    const double Fe = gl < Nl - 1 ? 0.5 * (c0.f0 + ae.f0) * ((ae.lap - c0.lap) * ids)
                                                        + 0.5 * (c0.f1 + ae.f1) * ((ae.u - c0.u) * ids)
                                                  : 0.0;
                    const double Fs = fm ? Am * Lm + Bm * Gm : 0.0;
                    const double Fn = fpl ? Ap * Lp + Bp * Gp : 0.0;
                    const double D = (Fe - Fw + Fn - Fs) * ids;
                    const double G = c0.u - sB[lp * WPITCH + lane] + p.cD * D;
                    rhs = -G;
                    if (active && !SOLVE) {
                        rmax = fmax(rmax, fabs(G));
                        if (G != G) flags |= FLAG_NAN;
                    }
                } else {
                    rhs = sB[lane * WPITCH + lp];
                }
                // bands of I + c J along the line (split Jacobian of the face fluxes)
                double a = 0.0, b = 0.0, c = 1.0, d = 0.0, e = 0.0;
                if (fpl) {
                    const double kA = k3 * Ap;
                    b -= kA;
                    c += 3.0 * kA + k1 * (0.5 * c0.f0p * Lp + 0.5 * c0.f1p * Gp - Bp * ids);
                    d += -3.0 * kA + k1 * (0.5 * cp.f0p * Lp + 0.5 * cp.f1p * Gp + Bp * ids);
                    e += kA;
                }
                if (fm) {
                    const double kA = k3 * Am;
                    a += kA;
                    b += -3.0 * kA - k1 * (0.5 * cm.f0p * Lm + 0.5 * cm.f1p * Gm - Bm * ids);
                    c += 3.0 * kA - k1 * (0.5 * c0.f0p * Lm + 0.5 * c0.f1p * Gm + Bm * ids);
                    d -= kA;
                }
                // fold ghost columns back (even reflection of the perturbation)
                if (gp == 0) { c += b; d += a; b = 0.0; a = 0.0; }
                else if (gp == 1) { b += a; a = 0.0; }
                if (gp == Np - 1) { c += d; b += e; d = 0.0; e = 0.0; }
                else if (gp == Np - 2) { d += e; e = 0.0; }
                // LU elimination step; the right-hand side carries the symbolic outer
                // unknowns (z: constant part, ph: coefficient of l1, ps: of l2)
                const double gam = b - a * al2;
                const double mu = c - a * be2 - gam * al1;
                const double rm = rcp(mu);
                const double al = (d - gam * be1) * rm;
                const double be = e * rm;
                const double z = (rhs - a * z2 - gam * z1) * rm;
                const double ph = (-a * ph2 - gam * ph1) * rm;
                const double pss = (-a * ps2 - gam * ps1) * rm;
                // rows s and s+1 of the inverse of the unit upper factor
                const double g = k == 0 ? 1.0 : -al1 * g1 - be2 * g2;
                const double h = k == 1 ? 1.0 : (k == 0 ? 0.0 : -al1 * h1 - be2 * h2);
                sgz += g * z; sgph += g * ph; sgps += g * pss;
                shz += h * z; shph += h * ph; shps += h * pss;
                if (SOLVE) {
                    fa[k] = al; fb[k] = be; fz[k] = z; fph[k] = ph; fps[k] = pss; fu[k] = c0.u;
                }
                g2 = g1; g1 = g; h2 = h1; h1 = h;
                al2 = al1; be2 = be1; al1 = al; be1 = be;
                z2 = z1; ph2 = ph1; ps2 = ps1; z1 = z; ph1 = ph; ps1 = pss;
                cm = c0;
                c0 = cp;
            }
        }
        // bottom pair: x_{e-1} = Z_{e-1} - al1 r1 - be1 r2, x_{e-2} = Z_{e-2} - be2 r1 - al2 x_{e-1}
        mine.B[1][0] = z1; mine.B[1][1] = ph1; mine.B[1][2] = ps1; mine.B[1][3] = -al1; mine.B[1][4] = -be1;
        mine.B[0][0] = z2 - al2 * z1; mine.B[0][1] = ph2 - al2 * ph1; mine.B[0][2] = ps2 - al2 * ps1;
        mine.B[0][3] = -be2 + al2 * al1; mine.B[0][4] = al2 * be1;
        // top pair: x_s = sum_k g_k Zt_k, x_{s+1} = sum_k h_k Zt_k
        mine.T[0][0] = sgz; mine.T[0][1] = sgph; mine.T[0][2] = sgps;
        mine.T[0][3] = -g2 * be2 - g1 * al1; mine.T[0][4] = -g1 * be1;
        mine.T[1][0] = shz; mine.T[1][1] = shph; mine.T[1][2] = shps;
        mine.T[1][3] = -h2 * be2 - h1 * al1; mine.T[1][4] = -h1 * be1;
    }

    if (!SOLVE && DIR == 0 && p.res != nullptr) {
        const double wm = wave_max(rmax);
        const unsigned wf = wave_or(flags);
        if (lane == 0) { sRed[wave][0] = wm; sFlag[wave] = wf; }
    }
    __syncthreads(); // all sweeps done: sB may be reused for the relation exchange
    if (len > 0) {
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
        if (DIR == 0 && p.res != nullptr && tid == 0) {
            double m = 0.0;
            unsigned f = 0;
            for (int w = 0; w < NSUB; ++w) { m = fmax(m, sRed[w][0]); f |= sFlag[w]; }
            atomicMax(&p.res[RES_RMAX], (unsigned long long)__double_as_longlong(m));
            if (f) atomicOr(&p.res[RES_FLAGS], (unsigned long long)f);
        }
        if (wave == 0 && active) {
            Rel R[NSUB];
#pragma unroll
            for (int q = 0; q < NSUB; ++q) {
                if (q >= nsub) break;
                const double *src = sB + (size_t)q * NREL * 64 + lane;
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 5; ++j) {
                        R[q].T[i][j] = src[(i * 5 + j) * 64];
                        R[q].B[i][j] = src[(10 + i * 5 + j) * 64];
                    }
            }
            Rel seg;
            chain_symbolic<NSUB>(R, nsub, seg);
            double *o = p.rel + (size_t)qseg * NREL * Nl + gl;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 5; ++j) {
                    o[(size_t)(i * 5 + j) * Nl] = seg.T[i][j];
                    o[(size_t)(10 + i * 5 + j) * Nl] = seg.B[i][j];
                }
        }
        return;
    }

    // ---- SOLVE: boundary values of this wave's sub-segment, then back-substitution
    double xs[SUB];
    double emax = 0.0;
    if (len > 0) {
        Rel R[NSUB];
#pragma unroll
        for (int q = 0; q < NSUB; ++q) {
            if (q >= nsub) break;
            const double *src = sB + (size_t)q * NREL * 64 + lane;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 5; ++j) {
                    R[q].T[i][j] = src[(i * 5 + j) * 64];
                    R[q].B[i][j] = src[(10 + i * 5 + j) * 64];
                }
        }
        const double *ex = p.ext + (size_t)qseg * NEXT * Nl + min(gl, Nl - 1);
        const double l1 = ex[0], l2 = ex[(size_t)Nl], r1 = ex[(size_t)2 * Nl], r2 = ex[(size_t)3 * Nl];
        double lo[NSUB][2], hi[NSUB][2];
        chain_numeric<NSUB>(R, nsub, l1, l2, r1, r2, lo, hi);
        double wl1 = lo[0][0], wl2 = lo[0][1], x1 = hi[0][0], x2 = hi[0][1];
#pragma unroll
        for (int q = 1; q < NSUB; ++q)
            if (q == wave) { wl1 = lo[q][0]; wl2 = lo[q][1]; x1 = hi[q][0]; x2 = hi[q][1]; }
#pragma unroll
        for (int k = SUB - 1; k >= 0; --k) {
            if (k < len) {
                const double x = fz[k] + fph[k] * wl1 + fps[k] * wl2 - fa[k] * x1 - fb[k] * x2;
                xs[k] = x;
                x2 = x1;
                x1 = x;
            }
        }
    }
    __syncthreads(); // relation records consumed: sU becomes the output staging tile

    if (DIR == 0) {
        // w is stored straight from registers: lanes cover consecutive x
        if (len > 0 && active) {
#pragma unroll
            for (int k = 0; k < SUB; ++k)
                if (k < len) p.out[(size_t)(pbase + ps + k) * nx + gl] = xs[k];
        }
        return;
    } else {
        if (len > 0 && active) {
#pragma unroll
            for (int k = 0; k < SUB; ++k) {
                if (k < len) {
                    const double v = xs[k];
                    const double un = fu[k] + v;
                    const double q = fabs(v) * rcp(fabs(fu[k]));
                    emax = fmax(emax, q);
                    if (!(un > 0.0)) flags |= (un != un || v != v) ? FLAG_NAN : FLAG_NONPOS;
                    sU[lane * UPITCH + ps + k] = un;
                }
            }
        }
        const double wm = wave_max(emax);
        const unsigned wf = wave_or(flags);
        if (lane == 0) { sRed[wave][0] = wm; sFlag[wave] = wf; }
        __syncthreads();
        for (int idx = tid; idx < TILE * TILE; idx += BLOCK) {
            const int ly = idx >> 6, lx = idx & 63;
            if (ly < nlt && lx < npos) p.out[(size_t)(y0 + ly) * nx + x0 + lx] = sU[ly * UPITCH + lx];
        }
        if (tid == 0 && p.res != nullptr) {
            double m = 0.0;
            unsigned f = 0;
            for (int w = 0; w < NSUB; ++w) { m = fmax(m, sRed[w][0]); f |= sFlag[w]; }
            atomicMax(&p.res[RES_EMAX], (unsigned long long)__double_as_longlong(m));
            if (f) atomicOr(&p.res[RES_FLAGS], (unsigned long long)f);
        }
    }
}

// ------------------------------------------------------------------------------------
// Interface chain: per line, block elimination over the P segments (outer boundary
// values are zero at the two ends of the line), then back-substitution giving every
// segment its two left and two right neighbouring values.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_chain(ChainParams c)
{
    const int line = blockIdx.x * 64 + threadIdx.x;
    if (line >= c.nlines) return;
    const size_t NL = (size_t)c.nlines;
    double tau0 = 0.0, tau1 = 0.0, bt0 = 0.0, bt1 = 0.0;
    M2 N = {0, 0, 0, 0}, Mm = {0, 0, 0, 0};
    for (int q = 0; q < c.P; ++q) {
        const double *r = c.rel + (size_t)q * NREL * NL + line;
        double T[2][5], B[2][5];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                T[i][j] = r[(size_t)(i * 5 + j) * NL];
                B[i][j] = r[(size_t)(10 + i * 5 + j) * NL];
            }
        const M2 Tl = {T[0][1], T[0][2], T[1][1], T[1][2]};
        const M2 Tr = {T[0][3], T[0][4], T[1][3], T[1][4]};
        const M2 Bl = {B[0][1], B[0][2], B[1][1], B[1][2]};
        const M2 Br = {B[0][3], B[0][4], B[1][3], B[1][4]};
        if (q == 0) {
            tau0 = T[0][0]; tau1 = T[1][0]; N = Tr;
            bt0 = B[0][0]; bt1 = B[1][0]; Mm = Br;
        } else {
            const M2 K = inv_i_minus(mul(Tl, Mm));
            const double s0 = T[0][0] + Tl.a * bt0 + Tl.b * bt1;
            const double s1 = T[1][0] + Tl.c * bt0 + Tl.d * bt1;
            const double nt0 = K.a * s0 + K.b * s1, nt1 = K.c * s0 + K.d * s1;
            const M2 nN = mul(K, Tr);
            const double v0 = bt0 + Mm.a * nt0 + Mm.b * nt1;
            const double v1 = bt1 + Mm.c * nt0 + Mm.d * nt1;
            const M2 BM = mul(mul(Bl, Mm), nN);
            tau0 = nt0; tau1 = nt1; N = nN;
            bt0 = B[0][0] + Bl.a * v0 + Bl.b * v1;
            bt1 = B[1][0] + Bl.c * v0 + Bl.d * v1;
            Mm = {BM.a + Br.a, BM.b + Br.b, BM.c + Br.c, BM.d + Br.d};
        }
        double *w = c.chain + (size_t)q * NCHAIN * NL + line;
        w[0] = tau0; w[NL] = tau1; w[2 * NL] = N.a; w[3 * NL] = N.b; w[4 * NL] = N.c; w[5 * NL] = N.d;
        w[6 * NL] = bt0; w[7 * NL] = bt1; w[8 * NL] = Mm.a; w[9 * NL] = Mm.b; w[10 * NL] = Mm.c;
        w[11 * NL] = Mm.d;
    }
    double tn0 = 0.0, tn1 = 0.0;
    for (int q = c.P - 1; q >= 0; --q) {
        const double *w = c.chain + (size_t)q * NCHAIN * NL + line;
        const double t0 = w[0] + w[2 * NL] * tn0 + w[3 * NL] * tn1;
        const double t1 = w[NL] + w[4 * NL] * tn0 + w[5 * NL] * tn1;
        double *e = c.ext + (size_t)q * NEXT * NL + line;
        e[2 * NL] = tn0;
        e[3 * NL] = tn1;
        if (q > 0) {
            const double *v = c.chain + (size_t)(q - 1) * NCHAIN * NL + line;
            e[0] = v[6 * NL] + v[8 * NL] * t0 + v[9 * NL] * t1;
            e[NL] = v[7 * NL] + v[10 * NL] * t0 + v[11 * NL] * t1;
        } else {
            e[0] = 0.0;
            e[NL] = 0.0;
        }
        tn0 = t0;
        tn1 = t1;
    }
}

// ------------------------------------------------------------------------------------
// out = alpha * add + beta * D(u) per cell (flux-difference operator; add may be null).
// Used for b^n = u^n - (1 - theta) dt D(u^n) and for testing D.
// ------------------------------------------------------------------------------------
template <bool P32>
__device__ __forceinline__ void cell_g(const double *u, int nx, int ny, int i, int j, const Model &M,
                                       double ids2, double &uc, double &lap, double &f0, double &f1)
{
    const int im = crefl(i - 1, nx), ip = crefl(i + 1, nx), jm = crefl(j - 1, ny), jp = crefl(j + 1, ny);
    const int ic = crefl(i, nx), jc = crefl(j, ny);
    uc = u[(size_t)jc * nx + ic];
    lap = (u[(size_t)jc * nx + ip] + u[(size_t)jc * nx + im] + u[(size_t)jp * nx + ic]
           + u[(size_t)jm * nx + ic] - 4.0 * uc) * ids2;
    double f0p, f1p;
    model_coefs<P32>(M, uc, f0, f1, f0p, f1p);
}

template <bool P32>
__global__ void __launch_bounds__(256) k_flux_divergence(int nx, int ny, double ids, double ids2, Model M,
                                                         const double *u, double alpha, double beta,
                                                         const double *add, double *out)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= nx || j >= ny) return;
    double uc, lc, f0c, f1c;
    cell_g<P32>(u, nx, ny, i, j, M, ids2, uc, lc, f0c, f1c);
    double F[4];
    const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
    const bool inside[4] = {i > 0, i < nx - 1, j > 0, j < ny - 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double un, ln, f0n, f1n;
        cell_g<P32>(u, nx, ny, i + di[k], j + dj[k], M, ids2, un, ln, f0n, f1n);
        // flux through the face towards neighbour k, oriented along +x / +y
        const bool lower = (k == 0 || k == 2);
        const double A = lower ? 0.5 * (f0n + f0c) : 0.5 * (f0c + f0n);
        const double B = lower ? 0.5 * (f1n + f1c) : 0.5 * (f1c + f1n);
        const double dl = lower ? (lc - ln) : (ln - lc);
        const double du = lower ? (uc - un) : (un - uc);
        F[k] = inside[k] ? A * (dl * ids) + B * (du * ids) : 0.0;
    }
    const double D = (F[1] - F[0] + F[3] - F[2]) * ids;
    const size_t o = (size_t)j * nx + i;
    out[o] = (add != nullptr ? alpha * add[o] : 0.0) + beta * D;
}

// ------------------------------------------------------------------------------------
// Mass diagnostic: per-block compensated (Neumaier) sum, minimum and NaN flag, reduced
// in a fixed tree order; the host adds the block records in index order.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void two_sum_acc(double &s, double &c, double x)
{
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

__global__ void __launch_bounds__(256) k_mass(const double *u, size_t n, double *partials)
{
    __shared__ double ss[256], sc[256], sm[256], sn[256];
    double s = 0.0, c = 0.0, m = __builtin_inf(), nanf = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const double x = u[i];
        if (x != x) nanf = 1.0;
        two_sum_acc(s, c, x);
        m = fmin(m, x);
    }
    ss[threadIdx.x] = s; sc[threadIdx.x] = c; sm[threadIdx.x] = m; sn[threadIdx.x] = nanf;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double a = ss[threadIdx.x], ca = sc[threadIdx.x] + sc[threadIdx.x + w];
            two_sum_acc(a, ca, ss[threadIdx.x + w]);
            ss[threadIdx.x] = a;
            sc[threadIdx.x] = ca;
            sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + w]);
            sn[threadIdx.x] = fmax(sn[threadIdx.x], sn[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[4 * blockIdx.x + 0] = ss[0];
        partials[4 * blockIdx.x + 1] = sc[0];
        partials[4 * blockIdx.x + 2] = sm[0];
        partials[4 * blockIdx.x + 3] = sn[0];
    }
}

// ---- launchers -----------------------------------------------------------------------
hipError_t launch_pass(int dir, bool solve, const PassParams &p, hipStream_t s)
{
    const dim3 grid(p.tiles_x * p.tiles_y), block(BLOCK);
    if (p.M.p32) {
        if (dir == 0 && !solve) k_pass<0, false, true><<<grid, block, 0, s>>>(p);
        else if (dir == 0) k_pass<0, true, true><<<grid, block, 0, s>>>(p);
        else if (!solve) k_pass<1, false, true><<<grid, block, 0, s>>>(p);
        else k_pass<1, true, true><<<grid, block, 0, s>>>(p);
    } else {
        if (dir == 0 && !solve) k_pass<0, false, false><<<grid, block, 0, s>>>(p);
        else if (dir == 0) k_pass<0, true, false><<<grid, block, 0, s>>>(p);
        else if (!solve) k_pass<1, false, false><<<grid, block, 0, s>>>(p);
        else k_pass<1, true, false><<<grid, block, 0, s>>>(p);
    }
    return hipGetLastError();
}

hipError_t launch_chain(const ChainParams &c, hipStream_t s)
{
    k_chain<<<dim3((c.nlines + 63) / 64), dim3(64), 0, s>>>(c);
    return hipGetLastError();
}

hipError_t launch_flux_divergence(int nx, int ny, double ids, double ids2, const Model &M, const double *u,
                                  double alpha, double beta, const double *add, double *out, hipStream_t s)
{
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4), block(256);
    if (M.p32) k_flux_divergence<true><<<grid, block, 0, s>>>(nx, ny, ids, ids2, M, u, alpha, beta, add, out);
    else k_flux_divergence<false><<<grid, block, 0, s>>>(nx, ny, ids, ids2, M, u, alpha, beta, add, out);
    return hipGetLastError();
}

int mass_blocks(size_t n)
{
    size_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_mass(const double *u, size_t n, double *partials, int nblocks, hipStream_t s)
{
    k_mass<<<dim3(nblocks), dim3(256), 0, s>>>(u, n, partials);
    return hipGetLastError();
}

} // namespace tf
