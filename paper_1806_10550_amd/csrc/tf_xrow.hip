// Whole-row x sweep (gfx950, FP64): the second half of one ADI-Newton iteration
// (Lam, Cummings & Kondic, arXiv:1806.10550, eqs. JacobianSystem2-3, NewtonError),
//   (I + c J_x(u_k)) v = w   per grid row,   u_{k+1} = u_k + v,   e = max|v/u_k|,
// in ONE kernel that reads u_k and w once and writes u_{k+1} once.
//
// A workgroup owns whole rows (one row of up to 8192 cells, or several shorter rows).
// Each lane owns a sub-segment of at most XR_CPL consecutive cells of its row:
//   phase 1  stage u_k(row) and u_k(row-1) + u_k(row+1) in LDS; every lane assembles the
//            five bands of its sub-segment and eliminates it with its outer unknowns (the
//            two cells before and the two after) kept symbolic -> a relation record
//            expressing its first and last cell pairs in those outer unknowns;
//   tree     the records of a row are merged pairwise in LDS (log2 levels): merging two
//            neighbouring blocks eliminates the two cell pairs at their junction; the
//            junction's solution, affine in the merged block's outer pairs, stays in the
//            right child's slot. Walking back down gives every sub-segment its outer pairs;
//   back-substitution  every lane finishes its sub-segment from the factors of phase 1
//            (held in registers; one of the five arrays waits in the u row's LDS while
//            the tree runs) and its outer pairs;
//   output   v through LDS, u_{k+1} = u_k + v, max|v/u_k|, h <= 0 / NaN flags and the
//            mass diagnostic of u_{k+1} in one coalesced store loop.
// No band, factor or interface record goes to HBM: 24 algorithmic bytes per cell (u_k is
// read twice, the second time for the update, mostly from L2).
#include "tf_sweep.h"

namespace tf {

bool xrow_supported(int nx)
{
    if (nx < 4 || nx > XR_MAX_NX) return false;
    const XRowGeom g = xrow_geom(nx);
    return g.W <= g.waves && g.R * (g.pu + g.p2) <= xr_lds(g.waves);
}

// Bands of row p of I + c J_x from the faces p-1/2 (fm) and p+1/2 (fp).
struct Band {
    double a, b, c, d, e;
};
__device__ __forceinline__ Band xr_band(const FaceS &fm, const FaceS &fp)
{
    Band B;
    B.a = fm.kA;
    B.b = __builtin_fma(-3.0, fm.kA, -fp.kA) - fm.P;
    B.c = __builtin_fma(3.0, fp.kA + fm.kA, 1.0) + (fp.P - fm.Q);
    B.d = __builtin_fma(-3.0, fp.kA, fp.Q) - fm.kA;
    B.e = fp.kA;
    return B;
}
// Ghost columns folded back (even reflection of the perturbation) at the row ends.
__device__ __forceinline__ void fold_left(Band &B, int pos) // pos: 0 or 1
{
    if (pos == 0) { B.c += B.b; B.d += B.a; B.b = 0.0; B.a = 0.0; }
    else { B.b += B.a; B.a = 0.0; }
}
__device__ __forceinline__ void fold_right(Band &B, int pos) // pos: nx-1 (0) or nx-2 (1)
{
    if (pos == 0) { B.c += B.d; B.b += B.e; B.d = 0.0; B.e = 0.0; }
    else { B.d += B.e; B.e = 0.0; }
}

// Orders this wave's LDS writes before its later LDS reads by other lanes of the same wave:
// the wave's LDS operations complete in issue order once the counter drains, and the empty
// asm statement keeps the compiler from moving memory accesses across the point.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_s_waitcnt(0xc07f); // lgkmcnt(0)
    __asm__ volatile("" ::: "memory");
}

// ---- record algebra of the row tree ---------------------------------------------------
// A block [a, e] of sub-segments has the record
//   T_a = t + Tl Bo + Tr To,   B_e = b + Bl Bo + Br To
// with Bo = B_{a-1} (the last pair before the block) and To = T_{e+1} (the first pair after
// it); a leaf record is the relation record (Rel) of one sub-segment. Records live in LDS
// as structure of arrays: field f of slot s at rec[f * S + s] (the Rel order T[0][0..4],
// T[1][0..4], B[0][0..4], B[1][0..4]).
__device__ __forceinline__ void rec_load(const double *rec, int S, int s, Rel &R)
{
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            R.T[i][j] = rec[(i * 5 + j) * S + s];
            R.B[i][j] = rec[(10 + i * 5 + j) * S + s];
        }
}
__device__ __forceinline__ M2 madd(const M2 &x, const M2 &y) { return {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d}; }
// Merge of the blocks in slots a (left, [a, m]) and c = m+1 (right, [c, e]): the junction
// pairs Bm = B_m and Tm = T_c solve
//   Bm = bL + BlL Bo + BrL Tm,   Tm = tR + TlR Bm + TrR To,
// so with K = (I - BrL TlR)^-1:  Bm = K (bL + BrL tR) + K BlL Bo + K BrL TrR To and
// Tm = tR + TlR Bm + TrR To. The merged record goes to slot a; the junction forms (Bm in
// the B fields, Tm in the T fields) to slot c.
__device__ __forceinline__ M2 ld_m2(const double *rec, int S, int s, int f) // fields f, f+1, f+5, f+6
{
    return {rec[f * S + s], rec[(f + 1) * S + s], rec[(f + 5) * S + s], rec[(f + 6) * S + s]};
}
__device__ __forceinline__ void st_form(double *rec, int S, int s, int f0, double c0, double c1, const M2 &L,
                                        const M2 &Rr) // fields f0 .. f0 + 9 (one pair form)
{
    double *r = rec + s;
    r[(f0 + 0) * S] = c0; r[(f0 + 1) * S] = L.a; r[(f0 + 2) * S] = L.b; r[(f0 + 3) * S] = Rr.a; r[(f0 + 4) * S] = Rr.b;
    r[(f0 + 5) * S] = c1; r[(f0 + 6) * S] = L.c; r[(f0 + 7) * S] = L.d; r[(f0 + 8) * S] = Rr.c; r[(f0 + 9) * S] = Rr.d;
}
__device__ __forceinline__ void rec_merge(double *rec, int S, int a, int c)
{
    // junction: B fields of slot a (left) and T fields of slot c (right)
    const M2 BrL = ld_m2(rec, S, a, 13), TlR = ld_m2(rec, S, c, 1);
    const double bL0 = rec[10 * S + a], bL1 = rec[15 * S + a], tR0 = rec[0 * S + c], tR1 = rec[5 * S + c];
    const M2 K = inv_i_minus(mul(BrL, TlR));
    const double s0 = bL0 + BrL.a * tR0 + BrL.b * tR1;
    const double s1 = bL1 + BrL.c * tR0 + BrL.d * tR1;
    const double b0 = K.a * s0 + K.b * s1, b1 = K.c * s0 + K.d * s1;
    const M2 TrR = ld_m2(rec, S, c, 3), BlL = ld_m2(rec, S, a, 11);
    const M2 b_l = mul(K, BlL), b_r = mul(K, mul(BrL, TrR));
    const double t0 = tR0 + TlR.a * b0 + TlR.b * b1, t1 = tR1 + TlR.c * b0 + TlR.d * b1;
    const M2 t_l = mul(TlR, b_l), t_r = madd(mul(TlR, b_r), TrR);
    // merged record: T from slot a's T fields, B from slot c's B fields
    {
        const M2 TlL = ld_m2(rec, S, a, 1), TrL = ld_m2(rec, S, a, 3);
        const double tL0 = rec[0 * S + a], tL1 = rec[5 * S + a];
        st_form(rec, S, a, 0, tL0 + TrL.a * t0 + TrL.b * t1, tL1 + TrL.c * t0 + TrL.d * t1, madd(TlL, mul(TrL, t_l)),
                mul(TrL, t_r));
    }
    {
        const M2 BlR = ld_m2(rec, S, c, 11), BrR = ld_m2(rec, S, c, 13);
        const double bR0 = rec[10 * S + c], bR1 = rec[15 * S + c];
        st_form(rec, S, a, 10, bR0 + BlR.a * b0 + BlR.b * b1, bR1 + BlR.c * b0 + BlR.d * b1, mul(BlR, b_l),
                madd(mul(BlR, b_r), BrR));
    }
    // junction forms: Tm in the T fields, Bm in the B fields of slot c
    st_form(rec, S, c, 0, t0, t1, t_l, t_r);
    st_form(rec, S, c, 10, b0, b1, b_l, b_r);
}

// Down the tree: the block in slot a with outer pairs (Bo, To) in rec[0..3][a] splits at
// c; the junction forms in slot c give Bm and Tm, and the children get (Bo, Tm) in slot a
// and (Bm, To) in slot c (fields 0..3 of a slot hold its outer pairs on the way down).
__device__ __forceinline__ void rec_split(double *rec, int S, int a, int c)
{
    const double bo0 = rec[0 * S + a], bo1 = rec[1 * S + a], to0 = rec[2 * S + a], to1 = rec[3 * S + a];
    Rel J;
    rec_load(rec, S, c, J);
    const double tm0 = J.T[0][0] + J.T[0][1] * bo0 + J.T[0][2] * bo1 + J.T[0][3] * to0 + J.T[0][4] * to1;
    const double tm1 = J.T[1][0] + J.T[1][1] * bo0 + J.T[1][2] * bo1 + J.T[1][3] * to0 + J.T[1][4] * to1;
    const double bm0 = J.B[0][0] + J.B[0][1] * bo0 + J.B[0][2] * bo1 + J.B[0][3] * to0 + J.B[0][4] * to1;
    const double bm1 = J.B[1][0] + J.B[1][1] * bo0 + J.B[1][2] * bo1 + J.B[1][3] * to0 + J.B[1][4] * to1;
    rec[2 * S + a] = tm0;
    rec[3 * S + a] = tm1;
    rec[0 * S + c] = bm0;
    rec[1 * S + c] = bm1;
    rec[2 * S + c] = to0;
    rec[3 * S + c] = to1;
}

// LU step at position k of a lane's sub-segment with the outer unknowns l1 = x_{p0-2},
// l2 = x_{p0-1} kept symbolic (z: constant part, ph: coefficient of l1, ps: of l2); the
// factors of every position stay in the arrays for the back-substitution.
template <int CPL>
__device__ __forceinline__ void xr_elim(int k, const Band &B, double rhs, double (&fa)[CPL], double (&fb)[CPL],
                                        double (&fz)[CPL], double (&fph)[CPL], double (&fps)[CPL])
{
    const double al2 = k >= 2 ? fa[k - 2] : 0.0, be2 = k >= 2 ? fb[k - 2] : 0.0;
    const double al1 = k >= 1 ? fa[k - 1] : 0.0, be1 = k >= 1 ? fb[k - 1] : 0.0;
    const double z2 = k >= 2 ? fz[k - 2] : 0.0, z1 = k >= 1 ? fz[k - 1] : 0.0;
    // rows p0-2 and p0-1 stand for the outer unknowns l1 (ph = 1) and l2 (ps = 1)
    const double ph2 = k >= 2 ? fph[k - 2] : (k == 0 ? 1.0 : 0.0), ph1 = k >= 1 ? fph[k - 1] : 0.0;
    const double ps2 = k >= 2 ? fps[k - 2] : (k == 1 ? 1.0 : 0.0), ps1 = k >= 1 ? fps[k - 1] : 1.0;
    const double gam = B.b - B.a * al2;
    const double mu = B.c - B.a * be2 - gam * al1;
    const double rm = rcp_pivot(mu);
    fa[k] = (B.d - gam * be1) * rm;
    fb[k] = B.e * rm;
    fz[k] = (rhs - B.a * z2 - gam * z1) * rm;
    fph[k] = (-B.a * ph2 - gam * ph1) * rm;
    fps[k] = (-B.a * ps2 - gam * ps1) * rm;
}

// The relation record of slot s from the factors of its sub-segment (Rel layout, field f at
// rec[f * S + s]). Top pair: x_{p0} = sum_k g_k Z_k, x_{p0+1} = sum_k h_k Z_k with g, h the
// first two rows of the inverse of the unit upper factor (g_k = -al_{k-1} g_{k-1} -
// be_{k-2} g_{k-2}) and Z_k = z_k + ph_k l1 + ps_k l2 the eliminated right-hand sides;
// bottom pair x_{e-1} = Z_{e-1} - al1 r1 - be1 r2, x_{e-2} = Z_{e-2} - al2 x_{e-1} - be2 r1.
template <int CPL>
__device__ __forceinline__ void xr_record(double *rec, int S, int s, const double (&fa)[CPL], const double (&fb)[CPL],
                                          const double (&fz)[CPL], const double (&fph)[CPL], const double (&fps)[CPL])
{
    double g1 = 0.0, g2 = 0.0, h1 = 0.0, h2 = 0.0;
    double sgz = 0.0, sgph = 0.0, sgps = 0.0, shz = 0.0, shph = 0.0, shps = 0.0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const double gg = k == 0 ? 1.0 : -fa[k - 1] * g1 - (k >= 2 ? fb[k - 2] : 0.0) * g2;
        const double hh = k == 1 ? 1.0 : (k == 0 ? 0.0 : -fa[k - 1] * h1 - (k >= 2 ? fb[k - 2] : 0.0) * h2);
        sgz += gg * fz[k]; sgph += gg * fph[k]; sgps += gg * fps[k];
        shz += hh * fz[k]; shph += hh * fph[k]; shps += hh * fps[k];
        g2 = g1; g1 = gg; h2 = h1; h1 = hh;
    }
    constexpr int L = CPL - 1;
    double *r = rec + s;
    r[0 * S] = sgz; r[1 * S] = sgph; r[2 * S] = sgps;
    r[3 * S] = -g2 * fb[L - 1] - g1 * fa[L]; r[4 * S] = -g1 * fb[L];
    r[5 * S] = shz; r[6 * S] = shph; r[7 * S] = shps;
    r[8 * S] = -h2 * fb[L - 1] - h1 * fa[L]; r[9 * S] = -h1 * fb[L];
    r[10 * S] = fz[L - 1] - fa[L - 1] * fz[L];
    r[11 * S] = fph[L - 1] - fa[L - 1] * fph[L];
    r[12 * S] = fps[L - 1] - fa[L - 1] * fps[L];
    r[13 * S] = -fb[L - 1] + fa[L - 1] * fa[L];
    r[14 * S] = fa[L - 1] * fb[L];
    r[15 * S] = fz[L]; r[16 * S] = fph[L]; r[17 * S] = fps[L]; r[18 * S] = -fa[L]; r[19 * S] = -fb[L];
}

// Tree over the S records of a row (called by every thread of the workgroup; tr: the
// thread's index within its row group, row_ok: the group holds a row). Level l merges the
// blocks starting at slots b * 2^l and b * 2^l + 2^(l-1); merge b is done by thread b of the
// row group, so only the first waves work at the low levels and wave 0 alone at the top
// (nm <= 64 merges: no workgroup barrier needed there, only ordering of this wave's LDS
// accesses). On return, fields 0..3 of slot s hold the outer pairs of sub-segment s.
__device__ __forceinline__ void xr_tree(double *rec, int S, int tr, bool row_ok)
{
    int levels = 0;
    while ((1 << levels) < S) ++levels;
    auto nmerge = [&](int l) { const int half = 1 << (l - 1); return (S - half + 2 * half - 1) / (2 * half); };
    int lw = levels + 1; // first level done by wave 0 alone
    for (int l = 1; l <= levels; ++l)
        if (nmerge(l) <= 64) { lw = l; break; }
    for (int l = 1; l < lw; ++l) {
        const int half = 1 << (l - 1);
        if (row_ok && tr < nmerge(l)) rec_merge(rec, S, tr * 2 * half, tr * 2 * half + half);
        __syncthreads();
    }
    if (row_ok && tr < 64) {
        for (int l = lw; l <= levels; ++l) {
            const int half = 1 << (l - 1);
            if (tr < nmerge(l)) rec_merge(rec, S, tr * 2 * half, tr * 2 * half + half);
            wave_lds_sync();
        }
        // the row's outer pairs are the ghost-folded ends: zero
        if (tr == 0) { rec[0 * S] = 0.0; rec[1 * S] = 0.0; rec[2 * S] = 0.0; rec[3 * S] = 0.0; }
        wave_lds_sync();
        for (int l = levels; l >= lw; --l) {
            const int half = 1 << (l - 1);
            if (tr < nmerge(l)) rec_split(rec, S, tr * 2 * half, tr * 2 * half + half);
            wave_lds_sync();
        }
    }
    __syncthreads();
    for (int l = lw - 1; l >= 1; --l) {
        const int half = 1 << (l - 1);
        if (row_ok && tr < nmerge(l)) rec_split(rec, S, tr * 2 * half, tr * 2 * half + half);
        __syncthreads();
    }
}

// Back-substitution of slot s from its outer pairs (fields 0..3 of the slot after the tree);
// the coefficient ps of l2 waits in the LDS slot of each position (parked there before the
// tree) and the solution replaces it.
template <int CPL>
__device__ __forceinline__ void xr_backsub(const double *rec, int S, int s, double *slots,
                                           const double (&fa)[CPL], const double (&fb)[CPL], const double (&fz)[CPL],
                                           const double (&fph)[CPL])
{
    // slots: this lane's block (position k at slots[k]); positions before the row are
    // identity rows and solve to zero
    const double l1 = rec[0 * S + s], l2 = rec[1 * S + s];
    double x1 = rec[2 * S + s], x2 = rec[3 * S + s];
#pragma unroll
    for (int k = CPL - 1; k >= 0; --k) {
        double *slot = slots + k;
        const double v = fz[k] + fph[k] * l1 + *slot * l2 - fa[k] * x1 - fb[k] * x2;
        *slot = v;
        x2 = x1;
        x1 = v;
    }
}

// ---- the kernel body -------------------------------------------------------------------
// Lane s of a row owns the XR_CPL positions p0 + k, p0 = nx - XR_CPL (S - s), k < XR_CPL.
// Positions before the row (only in lane 0, when XR_CPL does not divide nx) are identity
// rows with a zero right-hand side: the ghost folds at the left end leave the first real
// row without a coupling to them, so they solve to zero and change nothing. Every lane
// thus runs the same fixed-length loop; the row ends fall on lanes whose p0 <= 1 (left)
// and on positions XR_CPL-2, XR_CPL-1 of lane S-1 (right).
template <int KM>
__device__ __forceinline__ void xrow_body(const PassParams &p, const XRowGeom &g, int rowblock, double *lds)
{
    constexpr int CPL = XR_CPL;
    const int nx = p.nx, ny = p.ny;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rg = wave / g.W;                       // row group of this wave (uniform)
    const int s = (wave - rg * g.W) * 64 + lane;     // slot (sub-segment) of this lane in its row
    const int nthr = 64 * g.W;                       // threads of a row group
    const int tr = s;                                // thread index within the row group
    const int j = rowblock * g.R + rg;               // grid row of this row group
    const bool row_ok = rg < g.R && j < ny;
    double *const sU = lds + (size_t)rg * (g.pu + g.p2);
    double *const sX = sU + g.pu;                    // u_N + u_S, then the tree
    const double ka = p.ka;
    const int S = g.S;
    const int sh = CPL * S - nx;                     // staged index w = q + sh

    // ---- stage u(j) at w = -2 .. 16 S + 1 (two ghost cells each side) and u(j-1) + u(j+1)
    // at w = -1 .. 16 S (one); positions before lane 0's ghosts hold the first ghost's value.
    // Every global load of a thread is issued before its first LDS store.
    if (row_ok) {
        const double *uc = p.u + (size_t)j * nx;
        const double *un = p.u + (size_t)crefl(j - 1, ny) * nx;
        const double *us = p.u + (size_t)crefl(j + 1, ny) * nx;
        double vu[XR_STAGE], vx[XR_STAGE];
#pragma unroll
        for (int k = 0; k < XR_STAGE; ++k) {
            const int i = tr + k * nthr;            // w = i - 2 (u row), i - 1 (X row)
            if (i < CPL * S + 4) vu[k] = uc[crefl(max(i - 2 - sh, -2), nx)];
            if (i < CPL * S + 2) {
                const int c = crefl(max(i - 1 - sh, -1), nx);
                vx[k] = us[c] + un[c];
            }
        }
#pragma unroll
        for (int k = 0; k < XR_STAGE; ++k) {
            const int i = tr + k * nthr;
            if (i < CPL * S + 4) sU[xr_at(i - 2)] = vu[k];
            if (i < CPL * S + 2) sX[xr_at(i - 1)] = vx[k];
        }
    }
    const bool act = row_ok && s < S;
    const int p0 = nx - CPL * (S - s);
    const bool lnear = p0 <= 1;                      // holds a left-end position (or padding)
    const bool re = s == S - 1;                      // holds the right end at k = CPL-2, CPL-1
    // right-hand side w of this lane's cells (padding positions read cell 0)
    double wr[CPL];
    if (act) {
        const double *wrow = p.in2 + (size_t)j * nx;
#pragma unroll
        for (int k = 0; k < CPL; ++k) wr[k] = wrow[max(p0 + k, 0)];
    }
    __syncthreads();

    // u and ds^2 times the 5-point Laplacian at position p0 + t of this lane (t >= -1)
    const int base = xr_base(s);
    auto U = [&](int t) { return sU[base + xr_off(t)]; };
    auto cell = [&](int t) {
        const double uq = U(t);
        return cell_core<KM>(p, uq, __builtin_fma(-4.0, uq, (U(t + 1) + U(t - 1)) + sX[base + xr_off(t)]));
    };
    // phase 1: assemble and eliminate the sub-segment with its outer unknowns l1 = x_{p0-2},
    // l2 = x_{p0-1} kept symbolic (z: constant part, ph: coefficient of l1, ps: of l2); the
    // factors stay in registers for the back-substitution
    double fa[CPL], fb[CPL], fz[CPL], fph[CPL], fps[CPL];
    if (act) {
        CellS c0 = cell(0);
        FaceS fm = face_s<false>(cell(-1), c0, true, ka); // re-formed below at x = 0
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const int gp = p0 + k;
            const CellS cp = cell(k + 1);
            const FaceS fp = face_s<false>(c0, cp, !(re && k == CPL - 1), ka);
            Band B = xr_band(fm, fp);
            double rhs = wr[k];
            if (re && k >= CPL - 2) fold_right(B, CPL - 1 - k);
            if (lnear) {
                if (gp < 0) {
                    B = {0.0, 0.0, 1.0, 0.0, 0.0};
                    rhs = 0.0;
                } else if (gp == 0) {
                    // the face x = 0 carries no flux
                    B = xr_band(FaceS{0.0, 0.0, 0.0, 0.0}, fp);
                    if (re && k >= CPL - 2) fold_right(B, CPL - 1 - k);
                    fold_left(B, 0);
                } else if (gp == 1) {
                    fold_left(B, 1);
                }
            }
            xr_elim(k, B, rhs, fa, fb, fz, fph, fps);
            c0 = cp;
            fm = fp;
        }
    }
    __syncthreads(); // the staged rows are consumed: X becomes the record tree and the u
                     // row's space holds one factor array until the back-substitution
    double *const rec = sX;
    if (act) {
        xr_record(rec, S, s, fa, fb, fz, fph, fps);
#pragma unroll
        for (int k = 0; k < CPL; ++k) sU[base + k] = fps[k];
    }
    __syncthreads();
    xr_tree(rec, S, tr, row_ok);
    // back-substitution from the outer pairs; v replaces the parked factor in the u row
    if (act) xr_backsub(rec, S, s, sU + base, fa, fb, fz, fph);
    __syncthreads();

    // output: u_{k+1} = u_k + v, update ratio, flags, mass diagnostic (coalesced)
    double emax = 0.0;
    unsigned flags = 0;
    const bool diag = p.mass != nullptr;
    double ms = 0.0, mc = 0.0, mmin = __builtin_inf();
    if (row_ok) {
        double *orow = p.out + (size_t)j * nx;
        const double *urow = p.u + (size_t)j * nx;
        double uk[XR_STAGE];
#pragma unroll
        for (int k = 0; k < XR_STAGE; ++k) {
            const int i = tr + k * nthr;
            uk[k] = urow[min(i, nx - 1)];
        }
#pragma unroll
        for (int k = 0; k < XR_STAGE; ++k) {
            const int i = tr + k * nthr;
            if (i < nx) {
                const double v = sU[xr_at(i + sh)];
                const double un = uk[k] + v;
                emax = fmax(emax, fabs(v) * rcp(fabs(uk[k])));
                if (!(un > 0.0)) flags |= (un != un || v != v) ? FLAG_NAN : FLAG_NONPOS;
                orow[i] = un;
                if (diag) {
                    two_sum_acc(ms, mc, un);
                    mmin = fmin(mmin, un);
                }
            }
        }
    }
    const double wm = wave_max(emax);
    const unsigned wf = wave_or(flags);
    if (lane == 0 && p.res != nullptr) {
        unsigned long long *rs = p.res + (size_t)((blockIdx.x * 8 + wave) % p.res_spread) * RES_WORDS;
        atomicMax(&rs[RES_EMAX], (unsigned long long)__double_as_longlong(wm));
        if (wf) atomicOr(&rs[RES_FLAGS], (unsigned long long)wf);
    }
    if (diag) {
        // fixed-order butterfly over the lanes, then the waves in order: the record of the
        // workgroup does not depend on scheduling
        __shared__ double sM[3 * XR_WAVES];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            comp_add(ms, mc, __shfl_xor(ms, o), __shfl_xor(mc, o));
            mmin = fmin(mmin, __shfl_xor(mmin, o));
        }
        if (lane == 0) {
            sM[3 * wave] = ms;
            sM[3 * wave + 1] = mc;
            sM[3 * wave + 2] = mmin;
        }
        __syncthreads();
        if (tid == 0) {
            const int nw = blockDim.x >> 6;
            double sm = sM[0], c = sM[1], m = sM[2];
            for (int w = 1; w < nw; ++w) {
                comp_add(sm, c, sM[3 * w], sM[3 * w + 1]);
                m = fmin(m, sM[3 * w + 2]);
            }
            double *o = p.mass + 4 * (size_t)rowblock;
            o[0] = sm;
            o[1] = c;
            o[2] = m;
            o[3] = 0.0;
        }
    }
}

template <int KM, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_xrow(PassParams p, XRowGeom g, int nblocks)
{
    __shared__ double lds[xr_lds(WAVES)];
    const int rb = xcd_tile(blockIdx.x, nblocks);
    xrow_body<KM>(p, g, rb, lds);
}

template <int KM>
static void launch_xrow_km(const PassParams &p, const XRowGeom &g, hipStream_t s)
{
    const int nb = (p.ny + g.R - 1) / g.R;
    const dim3 grid(nb), block(64 * g.W * g.R);
    if (g.waves == 4) k_xrow<KM, 4><<<grid, block, 0, s>>>(p, g, nb);
    else k_xrow<KM, XR_WAVES><<<grid, block, 0, s>>>(p, g, nb);
}

// Ensemble version: block -> (film, row block) from the work list; the film's geometry,
// model, dt and buffer rotation come from the device tables. Every film on this path has
// rows of at most XR_ROW4_MAX_NX cells (4-wave workgroups). Films that are not iterating
// exit at once (before any barrier: the test is uniform over the block).
template <int KM>
__global__ void __launch_bounds__(256) k_xrow_ens(EnsParams e)
{
    __shared__ double lds[xr_lds(4)];
    const int t = xcd_tile(blockIdx.x, e.nitems);
    const int f = e.items[2 * t], rb = e.items[2 * t + 1];
    FilmState *st = e.state + f;
    if (!st->active) return;
    const FilmDesc d = e.desc[f];
    double *B[3] = {e.buf0, e.buf1, e.buf2};
    PassParams p{};
    p.nx = d.nx;
    p.ny = d.ny;
    p.ids2 = 1.0 / (d.ds * d.ds);
    p.f0s = p.ids2 * d.M.cap;
    p.ka = 0.5 * e.theta * st->dt * p.ids2;
    p.K0 = 3.0 * p.ka * p.ids2 * d.M.cap;
    p.K1 = p.ka * d.M.Dn;
    p.M = d.M;
    p.u = B[st->it] + d.off;
    p.in2 = e.w + d.off;
    p.out = B[st->nxt] + d.off;
    p.res = st->red;
    p.res_spread = ENS_RES_SPREAD;
    xrow_body<KM>(p, xrow_geom(d.nx), rb, lds);
}

hipError_t launch_xrow_ens(int km, const EnsParams &e, hipStream_t s)
{
    const dim3 grid(e.nitems), block(256);
    switch (km) {
    case KM_P32: k_xrow_ens<KM_P32><<<grid, block, 0, s>>>(e); break;
    case KM_POWER: k_xrow_ens<KM_POWER><<<grid, block, 0, s>>>(e); break;
    case KM_LINEAR: k_xrow_ens<KM_LINEAR><<<grid, block, 0, s>>>(e); break;
    case KM_NLC: k_xrow_ens<KM_NLC><<<grid, block, 0, s>>>(e); break;
    default: k_xrow_ens<KM_POLYMER><<<grid, block, 0, s>>>(e); break;
    }
    return hipGetLastError();
}

// ---- stored-band whole-line solve -------------------------------------------------------
// A x = r (TRANS: A^T x = r) for nl lines of np cells with the five bands a..e of A stored
// per line: line-major (PM false: element (line j, position i) at j np + i; the row solves
// of the adjoint's preconditioner) or position-major (PM true: at i nl + j; the layout of
// tf_penta_solve and of the adjoint's column solves), bands back to back (band k at
// k nl np). MODE 0: out = x; MODE 1: out += x and red[0], red[1] take max|x|, max|out|
// (atomic maxima of the bit patterns). One kernel instead of the partitioned solver's three:
// the elimination, relation records, tree and back-substitution are those of the forward
// whole-row sweep. Row p of A^T is (e_{p-2}, d_{p-1}, c_p, b_{p+1}, a_{p+2}); entries that
// reach outside the line are taken as zero. Padding positions before the line (lane 0, when
// XR_CPL does not divide np) are identity rows with a zero right-hand side, and the first
// real rows have no coupling to them.
template <bool TRANS, bool PM, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_sbline(int nl, int np, const double *bands, const double *rhs, double *out, unsigned long long *red, XRowGeom g,
         int nblocks, const unsigned long long *stop)
{
    if (stop != nullptr && *stop != 0ull) return; // a converged iteration (the whole workgroup leaves)
    __shared__ double lds[xr_lds(4)];
    __shared__ double sRed[4][2];
    constexpr int CPL = XR_CPL;
    const int rb = xcd_tile(blockIdx.x, nblocks);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rg = wave / g.W;                       // line group of this wave (uniform)
    const int s = (wave - rg * g.W) * 64 + lane;     // slot (sub-segment) of this lane in its line
    const int nthr = 64 * g.W;
    const int j = rb * g.R + rg;
    const bool row_ok = rg < g.R && j < nl;
    double *const sV = lds + (size_t)rg * (g.pu + g.p2); // parked factor, then the solution
    double *const rec = sV + g.pu;
    const int S = g.S;
    const bool act = row_ok && s < S;
    const int p0 = np - CPL * (S - s);
    const size_t N = (size_t)nl * np;
    // element (position q, this line), 0 <= q < np
    auto at = [&](int q) -> size_t { return PM ? (size_t)q * nl + j : (size_t)j * np + q; };
    double fa[CPL], fb[CPL], fz[CPL], fph[CPL], fps[CPL];
    if (act) {
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const int q = p0 + k;
            const bool real = q >= 0;
            // every load stays inside the line (clamped position); entries outside it are
            // selected away afterwards
            double va, vb, vc, vd, ve;
            if (TRANS) {
                va = bands[4 * N + at(max(q - 2, 0))];
                vb = bands[3 * N + at(max(q - 1, 0))];
                vc = bands[2 * N + at(max(q, 0))];
                vd = bands[N + at(min(max(q + 1, 0), np - 1))];
                ve = bands[at(min(max(q + 2, 0), np - 1))];
            } else {
                const size_t o = at(max(q, 0));
                va = bands[o]; vb = bands[N + o]; vc = bands[2 * N + o]; vd = bands[3 * N + o]; ve = bands[4 * N + o];
            }
            const double rr = rhs[at(max(q, 0))];
            Band B;
            B.a = q >= 2 ? va : 0.0;
            B.b = q >= 1 ? vb : 0.0;
            B.c = real ? vc : 1.0;
            B.d = real && q + 1 < np ? vd : 0.0;
            B.e = real && q + 2 < np ? ve : 0.0;
            xr_elim(k, B, real ? rr : 0.0, fa, fb, fz, fph, fps);
        }
        xr_record(rec, S, s, fa, fb, fz, fph, fps);
#pragma unroll
        for (int k = 0; k < CPL; ++k) sV[xr_base(s) + k] = fps[k];
    }
    __syncthreads();
    xr_tree(rec, S, s, row_ok);
    if (act) xr_backsub(rec, S, s, sV + xr_base(s), fa, fb, fz, fph);
    __syncthreads();
    double xm = 0.0, om = 0.0;
    if (row_ok) {
        for (int i = s; i < np; i += nthr) {
            const double x = sV[xr_at(i + CPL * S - np)];
            const size_t o = at(i);
            if (MODE == 0) {
                out[o] = x;
            } else {
                const double v = out[o] + x;
                out[o] = v;
                xm = max_nan(xm, fabs(x));
                om = max_nan(om, fabs(v));
            }
        }
    }
    if (MODE == 1) {
        const double wx = wave_max_nan(xm), wo = wave_max_nan(om);
        if (lane == 0) { sRed[wave][0] = wx; sRed[wave][1] = wo; }
        __syncthreads();
        if (tid == 0) {
            double a = 0.0, b = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a = max_nan(a, sRed[w][0]); b = max_nan(b, sRed[w][1]); }
            atomicMax(&red[0], (unsigned long long)__double_as_longlong(a));
            atomicMax(&red[1], (unsigned long long)__double_as_longlong(b));
        }
    }
}

bool sbline_supported(int np) { return np <= XR_ROW4_MAX_NX && xrow_supported(np); }

hipError_t launch_sbline(bool trans, bool pm, int mode, int nl, int np, const double *bands, const double *rhs,
                         double *out, unsigned long long *red, hipStream_t s, const unsigned long long *stop)
{
    if (nl < 1 || !sbline_supported(np) || (mode == 1 && red == nullptr) || (!pm && (!trans || mode != 0)))
        return hipErrorInvalidValue;
    const XRowGeom g = xrow_geom(np); // 4-wave workgroups for lines of at most XR_ROW4_MAX_NX cells
    const int nb = (nl + g.R - 1) / g.R;
    const dim3 grid(nb), block(64 * g.W * g.R);
    if (!pm) k_sbline<true, false, 0><<<grid, block, 0, s>>>(nl, np, bands, rhs, out, red, g, nb, stop);
    else if (trans && mode == 0) k_sbline<true, true, 0><<<grid, block, 0, s>>>(nl, np, bands, rhs, out, red, g, nb, stop);
    else if (trans) k_sbline<true, true, 1><<<grid, block, 0, s>>>(nl, np, bands, rhs, out, red, g, nb, stop);
    else if (mode == 0) k_sbline<false, true, 0><<<grid, block, 0, s>>>(nl, np, bands, rhs, out, red, g, nb, stop);
    else k_sbline<false, true, 1><<<grid, block, 0, s>>>(nl, np, bands, rhs, out, red, g, nb, stop);
    return hipGetLastError();
}

int xrow_blocks(int nx, int ny)
{
    const XRowGeom g = xrow_geom(nx);
    return (ny + g.R - 1) / g.R;
}

hipError_t launch_xrow(const PassParams &p, hipStream_t s)
{
    if (!xrow_supported(p.nx)) return hipErrorInvalidValue;
    const XRowGeom g = xrow_geom(p.nx);
    switch (p.M.kind) {
    case MODEL_LINEAR: launch_xrow_km<KM_LINEAR>(p, g, s); break;
    case MODEL_NLC: launch_xrow_km<KM_NLC>(p, g, s); break;
    case MODEL_POLYMER: launch_xrow_km<KM_POLYMER>(p, g, s); break;
    default:
        if (p.M.p32) launch_xrow_km<KM_P32>(p, g, s);
        else launch_xrow_km<KM_POWER>(p, g, s);
    }
    return hipGetLastError();
}

} // namespace tf
