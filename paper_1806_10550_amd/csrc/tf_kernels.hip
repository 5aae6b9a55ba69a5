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
#include "tf_device.h"

namespace tf {

#ifndef K3_WAVES_PER_EU
#define K3_WAVES_PER_EU 2
#endif
#ifndef K1_UNROLL
#define K1_UNROLL 1
#endif
#ifndef K1Y_FAST_UNROLL
#define K1Y_FAST_UNROLL 8
#endif

// ------------------------------------------------------------------------------------
// Tile pass. DIR 0: y sweep (columns), DIR 1: x sweep (rows). SOLVE false: emit the
// tile's segment relations; SOLVE true: finish the solve with the chained boundaries.
// y-sweep tiles own LT0 = 62 columns: lanes 0 and 63 carry the neighbouring columns so
// that the x faces of the residual come from lane shuffles.
// ------------------------------------------------------------------------------------
// Elimination sweep of one wave over its sub-segment [ps, ps+len) for all 64 lanes:
// assembles, per position, the cell coefficients, the residual (y sweep) and the five
// bands of I + c J, and runs the LU step with the sub-segment's outer unknowns kept
// symbolic. FAST: interior tile with 16 positions per wave, no domain boundary inside
// (no folded ghost columns, no zero-flux faces, no per-lane boundary selects).
template <int DIR, bool SOLVE, bool P32, bool FAST>
__device__ __forceinline__ void sweep(const double *sU, const double *sB, const PassParams &p, int lane, int ps,
                                      int len, int pbase, int Np, int gl, int Nl, bool owned, double *fa,
                                      double *fb, double *fz, double *fph, double *fps, Rel &mine,
                                      double &rmax, unsigned &flags)
{
    const double ids = p.ids, ids2 = p.ids2, k1 = p.k1, k3 = p.k3;
    {
        const Cell cm = cell_at<DIR, P32>(sU, p.M, ids2, lane, ps - 1);
        Cell c0 = cell_at<DIR, P32>(sU, p.M, ids2, lane, ps);
        FaceQ fm = face_q<DIR == 0>(cm, c0, FAST || pbase + ps > 0, ids, k1, k3);
        double al1 = 0.0, be1 = 0.0, al2 = 0.0, be2 = 0.0;
        // rows s-2 and s-1 stand for the outer unknowns l1 and l2
        double z1 = 0.0, ph1 = 0.0, ps1 = 1.0, z2 = 0.0, ph2 = 1.0, ps2 = 0.0;
        double g1 = 0.0, g2 = 0.0, h1 = 0.0, h2 = 0.0;
        double sgz = 0.0, sgph = 0.0, sgps = 0.0, shz = 0.0, shph = 0.0, shps = 0.0;
        // the solve pass keeps per-position factors in registers (full unroll); the
        // relations pass needs none and, off the interior path, is only partly unrolled
        constexpr int UNR = SOLVE ? SUB : (FAST ? (DIR == 0 ? K1Y_FAST_UNROLL : SUB) : K1_UNROLL);
#pragma unroll UNR
        for (int k = 0; k < SUB; ++k) {
            if (FAST || k < len) {
                const int lp = ps + k;
                const int gp = pbase + lp;          // wave-uniform
                const Cell cp = cell_at<DIR, P32>(sU, p.M, ids2, lane, lp + 1);
                const FaceQ fp = face_q<DIR == 0>(c0, cp, FAST || gp < Np - 1, ids, k1, k3);
                double rhs;
                if (DIR == 0) {
                    // -G(u_k) = -(u_k - b^n + theta dt D(u_k)); the x faces of this cell
                    // use the neighbouring lanes' cell values
                    const double eu = __shfl_down(c0.u, 1), el = __shfl_down(c0.lap, 1);
                    const double e0 = __shfl_down(c0.f0, 1), e1 = __shfl_down(c0.f1, 1);
                    const double Fe0 = 0.5 * (c0.f0 + e0) * ((el - c0.lap) * ids) + 0.5 * (c0.f1 + e1) * ((eu - c0.u) * ids);
                    const double Fe = (FAST || gl < Nl - 1) ? Fe0 : 0.0;
                    const double Fwr = __shfl_up(Fe, 1);
                    const double Fw = (FAST || gl > 0) ? Fwr : 0.0;
                    const double D = (Fe - Fw + fp.F - fm.F) * ids;
                    const double G = c0.u - sB[lp * WPITCH + lane] + p.cD * D;
                    rhs = -G;
                    if (!SOLVE && owned) {
                        rmax = fmax(rmax, fabs(G));
                        if (G != G) flags |= FLAG_NAN;
                    }
                } else {
                    rhs = sB[lane * WPITCH + lp];
                }
                // bands of I + c J along the line from the two face records
                double a = fm.kA;
                double b = -fp.kA - 3.0 * fm.kA - fm.P;
                double c = 1.0 + 3.0 * fp.kA + fp.P + 3.0 * fm.kA - fm.Q;
                double d = -3.0 * fp.kA + fp.Q - fm.kA;
                double e = fp.kA;
                if (!FAST) {
                    // fold ghost columns back (even reflection of the perturbation)
                    if (gp == 0) { c += b; d += a; b = 0.0; a = 0.0; }
                    else if (gp == 1) { b += a; a = 0.0; }
                    if (gp == Np - 1) { c += d; b += e; d = 0.0; e = 0.0; }
                    else if (gp == Np - 2) { d += e; e = 0.0; }
                }
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
                    fa[k] = al; fb[k] = be; fz[k] = z; fph[k] = ph; fps[k] = pss;
                }
                g2 = g1; g1 = g; h2 = h1; h1 = h;
                al2 = al1; be2 = be1; al1 = al; be1 = be;
                z2 = z1; ph2 = ph1; ps2 = ps1; z1 = z; ph1 = ph; ps1 = pss;
                c0 = cp;
                fm = fp;
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
}

template <int DIR, bool SOLVE, bool P32>
__device__ __forceinline__ void tile_body(const PassParams &p, int tx, int ty)
{
    __shared__ double sU[TW * UPITCH];
    __shared__ double sB[NSUB * NREL * 64];
    __shared__ double sRed[NSUB];
    __shared__ unsigned sFlag[NSUB];
    static_assert(NSUB * NREL * 64 >= TILE * WPITCH, "second LDS region too small");

    const int nx = p.nx, ny = p.ny;
    int x0, x1, y0, y1;
    if (DIR == 0) {
        x0 = tx * LT0; x1 = min(x0 + LT0, nx);
        y0 = seg_start(ty, ny); y1 = seg_start(ty + 1, ny);
    } else {
        x0 = seg_start(tx, nx); x1 = seg_start(tx + 1, nx);
        y0 = ty * TILE; y1 = min(y0 + TILE, ny);
    }
    const int bxo = DIR == 0 ? x0 - 1 : x0;  // grid x of lane/position 0 of the tile
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;


    {
        // issue every global load of the tile before the first LDS store
        constexpr int NU = (TW * TW + BLOCK - 1) / BLOCK, NB = TILE * TILE / BLOCK;
        double vu[NU], vb[NB];
#pragma unroll
        for (int r = 0; r < NU; ++r) {
            const int idx = tid + r * BLOCK;
            const int ly = min(idx / TW, TW - 1), lx = idx - (idx / TW) * TW;
            const int gx = crefl(bxo - HALO + lx, nx), gy = crefl(y0 - HALO + ly, ny);
            vu[r] = idx < TW * TW ? p.u[(size_t)gy * nx + gx] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int idx = tid + r * BLOCK;
            const int ly = idx >> 6, lx = idx & 63;
            const int gx = crefl(bxo + lx, nx), gy = min(y0 + ly, ny - 1);
            vb[r] = p.in2[(size_t)gy * nx + gx];
        }
#pragma unroll
        for (int r = 0; r < NU; ++r) {
            const int idx = tid + r * BLOCK;
            const int ly = idx / TW, lx = idx - ly * TW;
            if (idx < TW * TW) sU[ly * UPITCH + lx] = vu[r];
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            const int idx = tid + r * BLOCK;
            sB[(idx >> 6) * WPITCH + (idx & 63)] = vb[r];
        }
    }
    __syncthreads();

    const int lane0 = DIR == 0 ? 1 : 0;                 // first lane that owns a line
    const int nlt = DIR == 0 ? x1 - x0 : y1 - y0;       // lines owned by the tile
    const bool owned = lane >= lane0 && lane < lane0 + nlt;
    const int gl = (DIR == 0 ? x0 - 1 : y0) + lane;     // grid line of this lane
    const int pbase = DIR == 0 ? y0 : x0;
    const int npos = DIR == 0 ? y1 - y0 : x1 - x0;      // segment length
    const int Nl = DIR == 0 ? nx : ny;
    const int Np = DIR == 0 ? ny : nx;
    const int qseg = DIR == 0 ? ty : tx;
    const int nsub = min(NSUB, npos / 2);
    const int ps = (wave * npos) / nsub;
    const int len = wave < nsub ? ((wave + 1) * npos) / nsub - ps : 0;
    double fa[SUB], fb[SUB], fz[SUB], fph[SUB], fps[SUB];
    Rel mine;
    double rmax = 0.0;
    unsigned flags = 0;

    // interior tiles take the specialised path (wave-uniform branch)
    const bool fast = npos == TILE && pbase >= 2 && pbase + TILE <= Np - 2
                      && (DIR == 1 || (x0 > 0 && x0 + LT0 < nx && nlt == LT0));
    if (len > 0) {
        if (fast)
            sweep<DIR, SOLVE, P32, true>(sU, sB, p, lane, ps, len, pbase, Np, gl, Nl, owned, fa, fb, fz, fph, fps,
                                         mine, rmax, flags);
        else
            sweep<DIR, SOLVE, P32, false>(sU, sB, p, lane, ps, len, pbase, Np, gl, Nl, owned, fa, fb, fz, fph, fps,
                                          mine, rmax, flags);
    }

    if (!SOLVE && DIR == 0 && p.res != nullptr) {
        const double wm = wave_max(rmax);
        const unsigned wf = wave_or(flags);
        if (lane == 0) { sRed[wave] = wm; sFlag[wave] = wf; }
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
            for (int w = 0; w < NSUB; ++w) { m = fmax(m, sRed[w]); f |= sFlag[w]; }
            atomicMax(&p.res[RES_RMAX], (unsigned long long)__double_as_longlong(m));
            if (f) atomicOr(&p.res[RES_FLAGS], (unsigned long long)f);
        }
        if (wave == 0 && owned) {
            Rel seg;
            chain_symbolic(sB, lane, nsub, seg);
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
    double wl1 = 0.0, wl2 = 0.0, xr1 = 0.0, xr2 = 0.0;
    if (len > 0) {
        const double *ex = p.ext + (size_t)qseg * NEXT * Nl + min(max(gl, 0), Nl - 1);
        const double l1 = ex[0], l2 = ex[(size_t)Nl], r1 = ex[(size_t)2 * Nl], r2 = ex[(size_t)3 * Nl];
        chain_numeric(sB, lane, nsub, wave, l1, l2, r1, r2, wl1, wl2, xr1, xr2);
    }

    if (DIR == 0) {
        // w goes straight from registers to memory: lanes cover consecutive x
        if (len > 0) {
#pragma unroll
            for (int k = SUB - 1; k >= 0; --k) {
                if (k < len) {
                    const double x = fz[k] + fph[k] * wl1 + fps[k] * wl2 - fa[k] * xr1 - fb[k] * xr2;
                    if (owned) p.out[(size_t)(pbase + ps + k) * nx + gl] = x;
                    xr2 = xr1;
                    xr1 = x;
                }
            }
        }
        return;
    } else {
        __syncthreads(); // relation records consumed: sB becomes the output staging tile
        double emax = 0.0;
        if (len > 0) {
#pragma unroll
            for (int k = SUB - 1; k >= 0; --k) {
                if (k < len) {
                    const double v = fz[k] + fph[k] * wl1 + fps[k] * wl2 - fa[k] * xr1 - fb[k] * xr2;
                    xr2 = xr1;
                    xr1 = v;
                    const double uk = uat<DIR>(sU, lane, ps + k);
                    const double un = uk + v;
                    if (owned) {
                        emax = fmax(emax, fabs(v) * rcp(fabs(uk)));
                        if (!(un > 0.0)) flags |= (un != un || v != v) ? FLAG_NAN : FLAG_NONPOS;
                    }
                    sB[lane * WPITCH + ps + k] = un;
                }
            }
        }
        const double wm = wave_max(emax);
        const unsigned wf = wave_or(flags);
        if (lane == 0) { sRed[wave] = wm; sFlag[wave] = wf; }
        __syncthreads();
        for (int idx = tid; idx < TILE * TILE; idx += BLOCK) {
            const int ly = idx >> 6, lx = idx & 63;
            if (ly < nlt && lx < npos) p.out[(size_t)(y0 + ly) * nx + x0 + lx] = sB[ly * WPITCH + lx];
        }
        if (tid == 0 && p.res != nullptr) {
            double m = 0.0;
            unsigned f = 0;
            for (int w = 0; w < NSUB; ++w) { m = fmax(m, sRed[w]); f |= sFlag[w]; }
            atomicMax(&p.res[RES_EMAX], (unsigned long long)__double_as_longlong(m));
            if (f) atomicOr(&p.res[RES_FLAGS], (unsigned long long)f);
        }
    }
}

#define TF_PASS_ATTR                                                                         \
    __launch_bounds__(BLOCK)                                                                 \
    __attribute__((amdgpu_waves_per_eu(SOLVE ? K3_WAVES_PER_EU : 2, SOLVE ? K3_WAVES_PER_EU : 2)))

template <int DIR, bool SOLVE, bool P32>
__global__ void TF_PASS_ATTR k_pass(PassParams p)
{
    if (p.res_clear != nullptr && blockIdx.x == 0 && threadIdx.x < RES_WORDS) p.res_clear[threadIdx.x] = 0ull;
    const int t = xcd_tile(blockIdx.x, p.tiles_x * p.tiles_y);
    tile_body<DIR, SOLVE, P32>(p, t % p.tiles_x, t / p.tiles_x);
}

// Ensemble version: block -> (film, tile) from the work list; the film's geometry,
// model, dt and buffer rotation come from the device tables, so one launch (and one
// captured graph) serves every film. Films that are not iterating exit at once.
template <int DIR, bool SOLVE, bool P32>
__global__ void TF_PASS_ATTR k_pass_ens(EnsParams e)
{
    const int t = xcd_tile(blockIdx.x, e.nitems);
    const int f = e.items[3 * t], tx = e.items[3 * t + 1], ty = e.items[3 * t + 2];
    FilmState *s = e.state + f;
    if (!s->active) return;
    const FilmDesc d = e.desc[f];
    double *B[3] = {e.buf0, e.buf1, e.buf2};
    PassParams p{};
    p.nx = d.nx;
    p.ny = d.ny;
    p.ids = 1.0 / d.ds;
    p.ids2 = 1.0 / (d.ds * d.ds);
    const double c = e.theta * s->dt;
    p.k1 = c / d.ds;
    p.k3 = c / (d.ds * d.ds * d.ds * d.ds);
    p.cD = c;
    p.M = d.M;
    p.u = B[s->it] + d.off;
    p.in2 = DIR == 0 ? B[s->cur] + d.off : e.w + d.off;
    p.out = DIR == 0 ? e.w + d.off : B[s->nxt] + d.off;
    p.rel = e.rel + d.roff * NREL;
    p.ext = e.ext + d.roff * NEXT;
    p.res = s->red;
    tile_body<DIR, SOLVE, P32>(p, tx, ty);
}

// ------------------------------------------------------------------------------------
// Interface chain: per line, block elimination over the P segments (outer boundary
// values are zero at the two ends of the line), then back-substitution giving every
// segment its two left and two right neighbouring values.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void load_rec(const double *r, size_t NL, double (&T)[2][5], double (&B)[2][5])
{
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            T[i][j] = r[(size_t)(i * 5 + j) * NL];
            B[i][j] = r[(size_t)(10 + i * 5 + j) * NL];
        }
}

__device__ __forceinline__ void chain_body(const ChainParams &c, int line)
{
    const size_t NL = (size_t)c.nlines;
    const size_t RS = (size_t)NREL * NL; // stride between segment records
    double tau0 = 0.0, tau1 = 0.0, bt0 = 0.0, bt1 = 0.0;
    M2 N = {0, 0, 0, 0}, Mm = {0, 0, 0, 0};
    // records are loaded two segments ahead of their use to hide memory latency
    double T[2][5], B[2][5], Tn[2][5], Bn[2][5], Tnn[2][5], Bnn[2][5];
    const double *base = c.rel + line;
    load_rec(base, NL, T, B);
    if (c.P > 1) load_rec(base + RS, NL, Tn, Bn);
    for (int q = 0; q < c.P; ++q) {
        if (q + 2 < c.P) load_rec(base + (size_t)(q + 2) * RS, NL, Tnn, Bnn);
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
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                T[i][j] = Tn[i][j]; B[i][j] = Bn[i][j];
                Tn[i][j] = Tnn[i][j]; Bn[i][j] = Bnn[i][j];
            }
    }
    // backward substitution; the chain records of segments q and q-1 are read ahead
    double tn0 = 0.0, tn1 = 0.0;
    const double *cb = c.chain + line;
    const size_t CS = (size_t)NCHAIN * NL;
    double cq[6], cp[6], cpp[6]; // (tau0, tau1, N) of q; (bt0, bt1, M) of q-1
    auto ld_t = [&](int q, double *o) {
        const double *w = cb + (size_t)q * CS;
        for (int k = 0; k < 6; ++k) o[k] = w[(size_t)k * NL];
    };
    auto ld_b = [&](int q, double *o) {
        const double *w = cb + (size_t)q * CS + 6 * NL;
        for (int k = 0; k < 6; ++k) o[k] = w[(size_t)k * NL];
    };
    ld_t(c.P - 1, cq);
    if (c.P > 1) ld_b(c.P - 2, cp);
    for (int q = c.P - 1; q >= 0; --q) {
        double nq[6] = {0, 0, 0, 0, 0, 0};
        if (q > 0) ld_t(q - 1, nq);
        if (q > 1) ld_b(q - 2, cpp);
        const double t0 = cq[0] + cq[2] * tn0 + cq[3] * tn1;
        const double t1 = cq[1] + cq[4] * tn0 + cq[5] * tn1;
        double *e = c.ext + (size_t)q * NEXT * NL + line;
        e[2 * NL] = tn0;
        e[3 * NL] = tn1;
        if (q > 0) {
            e[0] = cp[0] + cp[2] * t0 + cp[3] * t1;
            e[NL] = cp[1] + cp[4] * t0 + cp[5] * t1;
        } else {
            e[0] = 0.0;
            e[NL] = 0.0;
        }
        tn0 = t0;
        tn1 = t1;
        for (int k = 0; k < 6; ++k) { cq[k] = nq[k]; cp[k] = cpp[k]; }
    }
}

__global__ void __launch_bounds__(64) k_chain(ChainParams c)
{
    const int line = blockIdx.x * 64 + threadIdx.x;
    if (line < c.nlines) chain_body(c, line);
}

// Ensemble version: block -> (film, block of 64 lines); dir 0 chains the y sweep.
__global__ void __launch_bounds__(64) k_chain_ens(EnsParams e, int dir)
{
    const int f = e.items[2 * blockIdx.x], lb = e.items[2 * blockIdx.x + 1];
    const FilmState *s = e.state + f;
    if (!s->active) return;
    const FilmDesc d = e.desc[f];
    ChainParams c{dir == 0 ? d.nx : d.ny, dir == 0 ? d.Py : d.Px, e.rel + d.roff * NREL, e.chain + d.roff * NCHAIN,
                  e.ext + d.roff * NEXT};
    const int line = lb * 64 + threadIdx.x;
    if (line < c.nlines) chain_body(c, line);
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

template <bool P32, bool NOF0>
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
        const double A = NOF0 ? 0.0 : (lower ? 0.5 * (f0n + f0c) : 0.5 * (f0c + f0n));
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


// ------------------------------------------------------------------------------------
// Ensemble control (Fig. FlowChartTime per film, on the device). One block; after
// every iteration each iterating film reads its reduction record and either accepts,
// continues, or rejects the attempt (shrinking dt when adaptive). The number of films
// still iterating is left in active_count for the host.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_ens_control(FilmState *st, int nfilms, EnsScheme S, int *active_count)
{
    __shared__ int cnt[256];
    int mine = 0;
    for (int f = threadIdx.x; f < nfilms; f += 256) {
        FilmState &s = st[f];
        if (!s.active) continue;
        const double e = __longlong_as_double((long long)s.red[RES_EMAX]);
        const double r = __longlong_as_double((long long)s.red[RES_RMAX]);
        const unsigned long long flags = s.red[RES_FLAGS];
        s.red[RES_EMAX] = 0ull;
        s.red[RES_RMAX] = 0ull;
        s.red[RES_FLAGS] = 0ull;
        s.k += 1;
        s.total += 1;
        s.e_last = e;
        s.r_last = r;
        bool fail = false;
        if (flags != 0ull) {
            fail = true;                       // an iterate left the admissible set
        } else if (e < S.tol) {                // accept u^{n+1} = u_{k+1}
            s.cur = s.nxt;
            s.newton = s.k;
            s.dt_used = s.dt;
            s.t += s.dt;
            s.successes += 1;
            if (S.adaptive && s.successes >= S.grow_after) {
                s.dt = fmin(s.dt * S.dt_grow, S.dt_max);
                s.successes = 0;
            }
            s.active = 0;
            s.status = 0;
        } else if (s.k >= S.max_newton) {
            fail = true;
        } else {                               // continue from u_{k+1}
            s.it = s.nxt;
            s.nxt = 3 - s.cur - s.it;
        }
        if (fail) {
            s.rejections += 1;
            s.successes = 0;
            s.dt_used = s.dt;
            if (!S.adaptive) {
                s.active = 0;
                s.status = 4; // TF_ENOCONV
            } else {
                s.dt *= S.dt_shrink;
                if (s.dt < S.dt_min) {
                    s.active = 0;
                    s.status = 4;
                } else {                       // retry from u^n
                    s.k = 0;
                    s.it = s.cur;
                    s.nxt = s.cur == 0 ? 1 : 0;
                }
            }
        }
        if (s.active) ++mine;
    }
    cnt[threadIdx.x] = mine;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) active_count[0] = cnt[0];
}

__global__ void __launch_bounds__(256) k_ens_begin(FilmState *st, int nfilms)
{
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (f >= nfilms) return;
    FilmState &s = st[f];
    if (s.status != 0) return;
    s.active = 1;
    s.k = 0;
    s.it = s.cur;
    s.nxt = s.cur == 0 ? 1 : 0;
    s.rejections = 0;
    s.red[RES_EMAX] = 0ull;
    s.red[RES_RMAX] = 0ull;
    s.red[RES_FLAGS] = 0ull;
}

// Copy every film's accepted state back into buffer 0 (the caller's).
__global__ void __launch_bounds__(256) k_ens_commit(const FilmDesc *desc, FilmState *st, double *buf0, double *buf1,
                                                    double *buf2)
{
    const int f = blockIdx.x;
    const int cur = st[f].cur;
    if (cur != 0) {
        const FilmDesc d = desc[f];
        const double *src = (cur == 1 ? buf1 : buf2) + d.off;
        double *dst = buf0 + d.off;
        const size_t n = (size_t)d.nx * d.ny;
        for (size_t i = threadIdx.x; i < n; i += 256) dst[i] = src[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) st[f].cur = 0;
}

// Mark films whose state holds h <= 0 or NaN (TF_ENONPOS).
__global__ void __launch_bounds__(256) k_ens_validate(const FilmDesc *desc, FilmState *st, const double *buf0)
{
    __shared__ int bad[256];
    const int f = blockIdx.x;
    const FilmDesc d = desc[f];
    const double *u = buf0 + d.off;
    const size_t n = (size_t)d.nx * d.ny;
    int b = 0;
    for (size_t i = threadIdx.x; i < n; i += 256)
        if (!(u[i] > 0.0)) b = 1;
    bad[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) bad[threadIdx.x] |= bad[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && bad[0]) {
        st[f].status = 5; // TF_ENONPOS
        st[f].active = 0;
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
    if (M.p32) k_flux_divergence<true, false><<<grid, block, 0, s>>>(nx, ny, ids, ids2, M, u, alpha, beta, add, out);
    else k_flux_divergence<false, false><<<grid, block, 0, s>>>(nx, ny, ids, ids2, M, u, alpha, beta, add, out);
    return hipGetLastError();
}

hipError_t launch_flux_divergence_f1(int nx, int ny, double ids, double ids2, const Model &M, const double *u,
                                     double *out, hipStream_t s)
{
    const dim3 grid((nx + 63) / 64, (ny + 3) / 4), block(256);
    if (M.p32) k_flux_divergence<true, true><<<grid, block, 0, s>>>(nx, ny, ids, ids2, M, u, 0.0, 1.0, nullptr, out);
    else k_flux_divergence<false, true><<<grid, block, 0, s>>>(nx, ny, ids, ids2, M, u, 0.0, 1.0, nullptr, out);
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

namespace tf {

hipError_t launch_pass_ens(int dir, bool solve, bool p32, const EnsParams &e, hipStream_t s)
{
    const dim3 grid(e.nitems), block(BLOCK);
    if (p32) {
        if (dir == 0 && !solve) k_pass_ens<0, false, true><<<grid, block, 0, s>>>(e);
        else if (dir == 0) k_pass_ens<0, true, true><<<grid, block, 0, s>>>(e);
        else if (!solve) k_pass_ens<1, false, true><<<grid, block, 0, s>>>(e);
        else k_pass_ens<1, true, true><<<grid, block, 0, s>>>(e);
    } else {
        if (dir == 0 && !solve) k_pass_ens<0, false, false><<<grid, block, 0, s>>>(e);
        else if (dir == 0) k_pass_ens<0, true, false><<<grid, block, 0, s>>>(e);
        else if (!solve) k_pass_ens<1, false, false><<<grid, block, 0, s>>>(e);
        else k_pass_ens<1, true, false><<<grid, block, 0, s>>>(e);
    }
    return hipGetLastError();
}

hipError_t launch_chain_ens(const EnsParams &e, int dir, hipStream_t s)
{
    k_chain_ens<<<dim3(e.nitems), dim3(64), 0, s>>>(e, dir);
    return hipGetLastError();
}

hipError_t launch_ens_control(FilmState *st, int nfilms, const EnsScheme &S, int *active_count, hipStream_t s)
{
    k_ens_control<<<dim3(1), dim3(256), 0, s>>>(st, nfilms, S, active_count);
    return hipGetLastError();
}

hipError_t launch_ens_begin(FilmState *st, int nfilms, hipStream_t s)
{
    k_ens_begin<<<dim3((nfilms + 255) / 256), dim3(256), 0, s>>>(st, nfilms);
    return hipGetLastError();
}

hipError_t launch_ens_commit(const FilmDesc *desc, FilmState *st, int nfilms, double *buf0, double *buf1,
                             double *buf2, hipStream_t s)
{
    k_ens_commit<<<dim3(nfilms), dim3(256), 0, s>>>(desc, st, buf0, buf1, buf2);
    return hipGetLastError();
}

hipError_t launch_ens_validate(const FilmDesc *desc, FilmState *st, int nfilms, const double *buf0, hipStream_t s)
{
    k_ens_validate<<<dim3(nfilms), dim3(256), 0, s>>>(desc, st, buf0);
    return hipGetLastError();
}

} // namespace tf
