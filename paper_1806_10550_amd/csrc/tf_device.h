// Device helpers shared by the forward sweeps (tf_kernels.hip) and the adjoint /
// stored-band solvers (tf_adjoint.hip): model coefficients, cell and face quantities,
// the reciprocal, ghost reflection, and the interface-chain algebra.
#pragma once

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

// Reciprocal with one Newton-Raphson step (within a few ulp; measured at most 11 on gfx950),
// for the pivots of the line solves: they only precondition the Newton iteration, whose fixed
// point does not depend on them.
__device__ __forceinline__ double rcp_pivot(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double ipow(double r, double h, int k)
{
    const double base = k >= 0 ? r : h;
    const int e = k >= 0 ? k : -k;
    double acc = 1.0;
    for (int i = 0; i < e; ++i) acc *= base;
    return acc;
}

// x^k for 0 <= k < 16 by binary powering with a fixed number of steps (no data-dependent
// loop, so the sweep kernels keep their registers).
__device__ __forceinline__ double pow16(double x, int k)
{
    double acc = 1.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        acc = (k & 1) ? acc * x : acc;
        x *= x;
        k >>= 1;
    }
    return acc;
}

// Pi'(h) and Pi''(h) of the NLC and polymer models (see Model), r = 1/h. NLC, with
// q = m(h)/h = g(h) s(h), s = h / (h^2 + beta^2):
//   Pi'  = K(-3 b^3 h^-4 + 2 b^2 h^-3) + N q q',
//   Pi'' = K(12 b^3 h^-5 - 6 b^2 h^-4) + N (q'^2 + q q'').
// g = (1 + tanh z)/2 = 1/(1 + e), e = exp(-2z), z = (h - 2b)/w, so that
//   tanh z = g (1 - e),  1 - tanh^2 z = 4 e g^2,  g' = (1 - tanh^2 z)/(2w),
//   g'' = -(1 - tanh^2 z) tanh z / w^2
// (one exponential and one reciprocal; every factor stays accurate when g is near 0 or 1).
__device__ __forceinline__ void nlc_derivs(const Model &M, double h, double r, double &pip, double &pipp)
{
    const double r2 = r * r, r4 = r2 * r2, r5 = r4 * r;
    {
        const double mz2 = fmin(-2.0 * (h - 2.0 * M.b) * M.iw, 700.0);
        const double e = exp(mz2);
        const double g = rcp(1.0 + e);
        const double s2 = 4.0 * e * (g * g), th = g * (1.0 - e);
        const double gp = 0.5 * s2 * M.iw, gpp = -s2 * th * (M.iw * M.iw);
        const double rd = rcp(h * h + M.beta2);
        const double sv = h * rd, sp = (M.beta2 - h * h) * rd * rd, spp = 2.0 * h * (h * h - 3.0 * M.beta2) * rd * rd * rd;
        const double q = g * sv, qp = gp * sv + g * sp, qpp = gpp * sv + 2.0 * gp * sp + g * spp;
        const double b2 = M.b * M.b, b3 = b2 * M.b;
        pip = M.K * (-3.0 * b3 * r4 + 2.0 * b2 * r2 * r) + M.N * q * qp;
        pipp = M.K * (12.0 * b3 * r5 - 6.0 * b2 * r4) + M.N * (qp * qp + q * qpp);
    }
}

__device__ __forceinline__ void polymer_derivs(const Model &M, double h, double r, double &pip, double &pipp)
{
    const double r2 = r * r, r4 = r2 * r2, r5 = r4 * r;
    {
        const double e = rcp(h + M.d), e2 = e * e, e4 = e2 * e2;
        const double r10 = r5 * r5;
        pip = -9.0 * M.C8 * r10 + 3.0 * M.a2 * r4 - 3.0 * M.c2 * e4;
        pipp = 90.0 * M.C8 * r10 * r - 12.0 * M.a2 * r5 + 12.0 * M.c2 * e4 * e;
    }
}

__device__ __forceinline__ void disjoining_derivs(const Model &M, double h, double r, double &pip, double &pipp)
{
    if (M.kind == MODEL_NLC) nlc_derivs(M, h, r, pip, pipp);
    else polymer_derivs(M, h, r, pip, pipp);
}

// f0 = cap h^3, f0' = 3 cap h^2, f1 = h^3 Pi'(h), f1' = 3 h^2 Pi' + h^3 Pi'' (see Model);
// f0 = c0, f1 = c1 for the linear model.
template <bool P32>
__device__ __forceinline__ void model_coefs(const Model &M, double u, double &f0, double &f1,
                                            double &f0p, double &f1p)
{
    if (!P32 && M.kind == MODEL_LINEAR) {
        f0 = M.cap;
        f1 = M.Cm;
        f0p = 0.0;
        f1p = 0.0;
        return;
    }
    const double r = rcp(u);
    const double u2 = u * u;
    f0 = M.cap * (u2 * u);
    f0p = 3.0 * M.cap * u2;
    if (P32) {
        f1 = M.Cm - M.Cn * r;
        f1p = M.Dn * (r * r);
    } else if (M.kind == MODEL_POWER) {
        f1 = M.Cm * ipow(r, u, M.m - 2) - M.Cn * ipow(r, u, M.n - 2);
        f1p = M.Dn * ipow(r, u, M.n - 1) - M.Dm * ipow(r, u, M.m - 1);
    } else {
        double pip, pipp;
        disjoining_derivs(M, u, r, pip, pipp);
        f1 = (u2 * u) * pip;
        f1p = 3.0 * u2 * pip + (u2 * u) * pipp;
    }
}

struct Cell {
    double u, lap, f0, f1, f0p, f1p; // f0p, f1p hold f0'/2 and f1'/2
};


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
    c.f0p *= 0.5; // the bands use f0'/2 and f1'/2
    c.f1p *= 0.5;
    return c;
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

// Relation records (NREL doubles per (segment, line)) and chain records (NCHAIN) in global
// memory hold the fields of a record in pairs: in a block of records of NL lines, field f of
// line l sits at 2 (f / 2) NL + 2 l + f % 2, so that a lane moves two fields with one 16-byte
// access and the accesses of a wave are contiguous. `r` points at the block advanced by 2 l.
// (Boundary records, NEXT doubles, keep one field per array: field f of line l at f NL + l.)
__device__ __forceinline__ double2 rec_get2(const double *r, size_t NL, int k)
{
    return *reinterpret_cast<const double2 *>(r + 2 * (size_t)k * NL);
}
__device__ __forceinline__ void rec_put2(double *r, size_t NL, int k, double a, double b)
{
    *reinterpret_cast<double2 *>(r + 2 * (size_t)k * NL) = make_double2(a, b);
}

// Field f (record order T[0][0..4], T[1][0..4], B[0][0..4], B[1][0..4]) of a relation record.
__device__ __forceinline__ double &rel_field(Rel &S, int f)
{
    return f < 10 ? S.T[f / 5][f % 5] : S.B[(f - 10) / 5][(f - 10) % 5];
}

// A relation record to / from global memory (paired layout above).
__device__ __forceinline__ void rel_store(double *r, size_t NL, Rel S)
{
#pragma unroll
    for (int k = 0; k < NREL / 2; ++k) rec_put2(r, NL, k, rel_field(S, 2 * k), rel_field(S, 2 * k + 1));
}
__device__ __forceinline__ void rel_fetch(const double *r, size_t NL, Rel &S)
{
#pragma unroll
    for (int k = 0; k < NREL / 2; ++k) {
        const double2 v = rec_get2(r, NL, k);
        rel_field(S, 2 * k) = v.x;
        rel_field(S, 2 * k + 1) = v.y;
    }
}

// Relation record q of this lane from the LDS exchange area.
__device__ __forceinline__ void load_rel(const double *sB, int q, int lane, Rel &S)
{
    const double *src = sB + (size_t)q * NREL * 64 + lane;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            S.T[i][j] = src[(i * 5 + j) * 64];
            S.B[i][j] = src[(10 + i * 5 + j) * 64];
        }
}

// Interface chain over the Q sub-segments of a tile (forward block elimination):
// with B_{q-1} = bt_{q-1} + M_{q-1} T_q from the previous step, sub-segment q gives
//   T_q = tau_q + N_q T_{q+1},  tau_q = K (t_q + Tl_q bt_{q-1}),  N_q = K Tr_q,
//   K = (I - Tl_q M_{q-1})^-1,
//   B_q = bt_q + M_q T_{q+1},   bt_q = b_q + Bl_q (bt_{q-1} + M_{q-1} tau_q),
//   M_q = Bl_q M_{q-1} N_q + Br_q.
// The recurrences below carry only what later steps need, so T_0 (and the boundary
// values a wave needs) follow from forward accumulation: T_0 = sum_q N_0..N_{q-1} tau_q
// + N_0..N_{Q-1} T_Q.

// Symbolic version: quantities are affine forms over (1, l1, l2, r1, r2), the tile's
// outer boundary values. The record of sub-segment 0 comes in registers, those of
// sub-segments 1..Q-1 from the LDS exchange area `rest`. Returns the tile's relation
// record (T_0, B_{Q-1}).
__device__ __forceinline__ void chain_symbolic(const Rel &first, const double *rest, int lane, int Q, Rel &out)
{
    double bt[2][5], acc[2][5];
    M2 Mm = {0, 0, 0, 0}, P = {1, 0, 0, 1};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) { bt[i][j] = 0.0; acc[i][j] = 0.0; }
#pragma unroll
    for (int q = 0; q < NSUB; ++q) {
        if (q >= Q) break;
        Rel S;
        if (q == 0) S = first;
        else load_rel(rest, q - 1, lane, S);
        const M2 Tl = {S.T[0][1], S.T[0][2], S.T[1][1], S.T[1][2]};
        const M2 Tr = {S.T[0][3], S.T[0][4], S.T[1][3], S.T[1][4]};
        const M2 Bl = {S.B[0][1], S.B[0][2], S.B[1][1], S.B[1][2]};
        const M2 Br = {S.B[0][3], S.B[0][4], S.B[1][3], S.B[1][4]};
        double tau[2][5];
        M2 N;
        if (q == 0) {
            // B_{-1} is the outer pair (l1, l2)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                tau[i][0] = S.T[i][0]; tau[i][1] = S.T[i][1]; tau[i][2] = S.T[i][2]; tau[i][3] = 0.0; tau[i][4] = 0.0;
                bt[i][0] = S.B[i][0]; bt[i][1] = S.B[i][1]; bt[i][2] = S.B[i][2]; bt[i][3] = 0.0; bt[i][4] = 0.0;
            }
            N = Tr;
            Mm = Br;
        } else {
            const M2 K = inv_i_minus(mul(Tl, Mm));
            N = mul(K, Tr);
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                const double s0 = (j == 0 ? S.T[0][0] : 0.0) + Tl.a * bt[0][j] + Tl.b * bt[1][j];
                const double s1 = (j == 0 ? S.T[1][0] : 0.0) + Tl.c * bt[0][j] + Tl.d * bt[1][j];
                tau[0][j] = K.a * s0 + K.b * s1;
                tau[1][j] = K.c * s0 + K.d * s1;
                const double v0 = bt[0][j] + Mm.a * tau[0][j] + Mm.b * tau[1][j];
                const double v1 = bt[1][j] + Mm.c * tau[0][j] + Mm.d * tau[1][j];
                bt[0][j] = (j == 0 ? S.B[0][0] : 0.0) + Bl.a * v0 + Bl.b * v1;
                bt[1][j] = (j == 0 ? S.B[1][0] : 0.0) + Bl.c * v0 + Bl.d * v1;
            }
            const M2 BM = mul(mul(Bl, Mm), N);
            Mm = {BM.a + Br.a, BM.b + Br.b, BM.c + Br.c, BM.d + Br.d};
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            acc[0][j] += P.a * tau[0][j] + P.b * tau[1][j];
            acc[1][j] += P.c * tau[0][j] + P.d * tau[1][j];
        }
        P = mul(P, N);
    }
    // T_Q is the outer right pair: the forms r1, r2
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            out.T[i][j] = acc[i][j];
            out.B[i][j] = bt[i][j];
        }
    out.T[0][3] += P.a; out.T[0][4] += P.b; out.T[1][3] += P.c; out.T[1][4] += P.d;
    out.B[0][3] += Mm.a; out.B[0][4] += Mm.b; out.B[1][3] += Mm.c; out.B[1][4] += Mm.d;
}

// Numeric version with the outer values known: returns the boundary values of
// sub-segment w, lo = B_{w-1} (the outer l for w = 0) and hi = T_{w+1} (outer r for the
// last sub-segment).
template <bool SKIP_LAST_B = false>
__device__ __forceinline__ void chain_numeric(const double *sB, int lane, int Q, int w, double l1, double l2,
                                              double r1, double r2, double &lo1, double &lo2, double &hi1,
                                              double &hi2)
{
    double bt0 = 0.0, bt1 = 0.0;
    M2 Mm = {0, 0, 0, 0};
    double sbt0 = 0.0, sbt1 = 0.0, stau0 = 0.0, stau1 = 0.0; // bt_{w-1}, tau_w
    M2 sM = {0, 0, 0, 0}, sN = {0, 0, 0, 0};                 // M_{w-1}, N_w
    double acc0 = 0.0, acc1 = 0.0;
    M2 P = {1, 0, 0, 1};
#pragma unroll
    for (int q = 0; q < NSUB; ++q) {
        if (q >= Q) break;
        // the bottom pair of the last sub-segment is never used (SKIP_LAST_B: not exchanged)
        Rel S;
        if (!SKIP_LAST_B) {
            load_rel(sB, q, lane, S);
        } else {
            const double *src = sB + (size_t)q * NREL * 64 + lane;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 5; ++j) {
                    S.T[i][j] = src[(i * 5 + j) * 64];
                    S.B[i][j] = q < Q - 1 ? src[(10 + i * 5 + j) * 64] : 0.0;
                }
        }
        const M2 Tl = {S.T[0][1], S.T[0][2], S.T[1][1], S.T[1][2]};
        const M2 Tr = {S.T[0][3], S.T[0][4], S.T[1][3], S.T[1][4]};
        const M2 Bl = {S.B[0][1], S.B[0][2], S.B[1][1], S.B[1][2]};
        const M2 Br = {S.B[0][3], S.B[0][4], S.B[1][3], S.B[1][4]};
        double tau0, tau1;
        M2 N;
        if (q == 0) {
            tau0 = S.T[0][0] + Tl.a * l1 + Tl.b * l2;
            tau1 = S.T[1][0] + Tl.c * l1 + Tl.d * l2;
            N = Tr;
            bt0 = S.B[0][0] + Bl.a * l1 + Bl.b * l2;
            bt1 = S.B[1][0] + Bl.c * l1 + Bl.d * l2;
            Mm = Br;
        } else {
            if (q == w) { sbt0 = bt0; sbt1 = bt1; sM = Mm; }
            const M2 K = inv_i_minus(mul(Tl, Mm));
            const double s0 = S.T[0][0] + Tl.a * bt0 + Tl.b * bt1;
            const double s1 = S.T[1][0] + Tl.c * bt0 + Tl.d * bt1;
            tau0 = K.a * s0 + K.b * s1;
            tau1 = K.c * s0 + K.d * s1;
            N = mul(K, Tr);
            const double v0 = bt0 + Mm.a * tau0 + Mm.b * tau1;
            const double v1 = bt1 + Mm.c * tau0 + Mm.d * tau1;
            bt0 = S.B[0][0] + Bl.a * v0 + Bl.b * v1;
            bt1 = S.B[1][0] + Bl.c * v0 + Bl.d * v1;
            const M2 BM = mul(mul(Bl, Mm), N);
            Mm = {BM.a + Br.a, BM.b + Br.b, BM.c + Br.c, BM.d + Br.d};
        }
        if (q == w) { stau0 = tau0; stau1 = tau1; sN = N; }
        if (q > w) {
            acc0 += P.a * tau0 + P.b * tau1;
            acc1 += P.c * tau0 + P.d * tau1;
            P = mul(P, N);
        }
    }
    // T_{w+1} (the outer r when w is the last sub-segment)
    hi1 = acc0 + P.a * r1 + P.b * r2;
    hi2 = acc1 + P.c * r1 + P.d * r2;
    if (w == 0) {
        lo1 = l1;
        lo2 = l2;
    } else {
        const double t0 = stau0 + sN.a * hi1 + sN.b * hi2;
        const double t1 = stau1 + sN.c * hi1 + sN.d * hi2;
        lo1 = sbt0 + sM.a * t0 + sM.b * t1;
        lo2 = sbt1 + sM.c * t0 + sM.d * t1;
    }
}

// Neumaier's compensated accumulation: s + c carries the running sum, c the rounding errors
// of the additions (each recovered exactly by the two-sum identity).
__device__ __forceinline__ void two_sum_acc(double &s, double &c, double x)
{
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

// Combine two compensated partial sums (s, c) += (s2, c2); symmetric in its operands, so a
// butterfly over the lanes of a wave leaves the same value in every lane.
__device__ __forceinline__ void comp_add(double &s, double &c, double s2, double c2)
{
    double cc = c + c2;
    two_sum_acc(s, cc, s2);
    c = cc;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
// Maximum that keeps a NaN (fmax drops it): used where a NaN must reach the host.
__device__ __forceinline__ double max_nan(double a, double b) { return (b != b || b > a) ? b : a; }
__device__ __forceinline__ double wave_max_nan(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max_nan(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ unsigned wave_or(unsigned v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

struct FaceQ {
    double kA, P, Q, F; // k3 A, k1 (f0'_L Lam + f1'_L Gam)/2 - k1 B/ds, the same with R and +B, flux
};

template <bool FLUX>
__device__ __forceinline__ FaceQ face_q(const Cell &L, const Cell &R, bool interior, double ids, double k1,
                                        double k3)
{
    FaceQ f;
    const double A = 0.5 * (L.f0 + R.f0), B = 0.5 * (L.f1 + R.f1);
    const double Lam = (R.lap - L.lap) * ids, Gam = (R.u - L.u) * ids;
    const double Bi = B * ids;
    f.kA = interior ? k3 * A : 0.0;
    f.P = interior ? k1 * (L.f0p * Lam + L.f1p * Gam - Bi) : 0.0;
    f.Q = interior ? k1 * (R.f0p * Lam + R.f1p * Gam + Bi) : 0.0;
    f.F = (FLUX && interior) ? A * Lam + B * Gam : 0.0;
    return f;
}

} // namespace tf
