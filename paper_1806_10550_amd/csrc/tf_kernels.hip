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
#include "tf_sweep.h"

namespace tf {

#ifndef K3_WAVES_PER_EU
#define K3_WAVES_PER_EU 2
#endif
#ifndef K1Y_WAVES_PER_EU
#define K1Y_WAVES_PER_EU 4
#endif
#ifndef K1X_WAVES_PER_EU
#define K1X_WAVES_PER_EU 3
#endif
#ifndef K1_UNROLL
#define K1_UNROLL 1
#endif
#ifndef K1Y_FAST_UNROLL
#define K1Y_FAST_UNROLL 2
#endif
#ifndef K1X_FAST_UNROLL
#define K1X_FAST_UNROLL 4
#endif

// ------------------------------------------------------------------------------------
// Tile pass. DIR 0: y sweep (columns), DIR 1: x sweep (rows). SOLVE false: emit the
// tile's segment relations; SOLVE true: finish the solve with the chained boundaries.
// A tile owns 64 lines (one per lane). The x faces of the y sweep's residual come from
// lane shuffles; the fluxes through the two faces on the tile's x edges are formed once per
// position before the sweeps and enter the b^n of lanes 0 and 63.
// ------------------------------------------------------------------------------------
// Value of the next (lane + 1) / previous (lane - 1) lane of the wave by whole-wave DPP
// shifts (VALU moves, no LDS permute); the edge lanes get 0 (the y sweep replaces what
// they would need by the tile-edge correction of b^n).
__device__ __forceinline__ double dpp_shift(double v, int ctrl)
{
    // bound_ctrl set: a lane whose source lies outside the wave reads 0, so no "old" value
    // has to be materialised first
    const long long b = __double_as_longlong(v);
    const int lo = ctrl == 0x130 ? __builtin_amdgcn_mov_dpp((int)b, 0x130, 0xf, 0xf, true)
                                 : __builtin_amdgcn_mov_dpp((int)b, 0x138, 0xf, 0xf, true);
    const int hi = ctrl == 0x130 ? __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xf, 0xf, true)
                                 : __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_next(double v) { return dpp_shift(v, 0x130); } // wave_shl:1
__device__ __forceinline__ double lane_prev(double v) { return dpp_shift(v, 0x138); } // wave_shr:1

// Cell quantities at (line l, position q) of the LDS u tile.
template <int DIR, int KM>
__device__ __forceinline__ CellS cell_s(const double *sU, const PassParams &p, int l, int q)
{
    const double u = uat<DIR>(sU, l, q);
    double xp, xm, yp, ym;
    if (DIR == 0) {
        xp = uat<DIR>(sU, l + 1, q); xm = uat<DIR>(sU, l - 1, q);
        yp = uat<DIR>(sU, l, q + 1); ym = uat<DIR>(sU, l, q - 1);
    } else {
        xp = uat<DIR>(sU, l, q + 1); xm = uat<DIR>(sU, l, q - 1);
        yp = uat<DIR>(sU, l + 1, q); ym = uat<DIR>(sU, l - 1, q);
    }
    return cell_core<KM>(p, u, __builtin_fma(-4.0, u, (xp + xm) + (yp + ym)));
}

// Elimination sweep of one wave over its sub-segment [ps, ps+len) for all 64 lanes:
// assembles, per position, the cell quantities, the residual (y sweep) and the five
// bands of I + c J, and runs the LU step with the sub-segment's outer unknowns kept
// symbolic. FAST: interior tile with 16 positions per wave, no domain boundary inside
// (no folded ghost columns, no zero-flux faces, no per-lane boundary selects).
template <int DIR, bool SOLVE, int KM, bool FAST>
__device__ __forceinline__ void sweep(const double *sU, double *sB, const double *sCorr, const double *bcol,
                                      const PassParams &p, int lane, int ps, int len, int pbase, int Np, int gl, int Nl,
                                      bool owned, double *fa,
                                      double *fb, double *fz, double *fph, double *fps, Rel &mine,
                                      double &rmax, unsigned &flags)
{
    const double ka = p.ka;
    // x relations pass: w read straight from global memory (each lane walks its row)
    constexpr bool WG = DIR == 1 && !SOLVE;
    // y relations pass: b^n corrections of this lane (lanes 0 and 63; the others read zeros)
    const double *corr = sCorr + (lane == 0 ? 0 : (lane == TILE - 1 ? TILE : 2 * TILE));
    // y sweep: lane 63 takes zero flux through its right face (the tile edge; its b^n carries
    // the flux there)
    const bool feok = DIR == 0 && (FAST || gl < Nl - 1) && lane != TILE - 1;
    {
        const CellS cm = cell_s<DIR, KM>(sU, p, lane, ps - 1);
        CellS c0 = cell_s<DIR, KM>(sU, p, lane, ps);
        FaceS fm = face_s<DIR == 0>(cm, c0, FAST || pbase + ps > 0, ka);
        double al1 = 0.0, be1 = 0.0, al2 = 0.0, be2 = 0.0;
        // rows s-2 and s-1 stand for the outer unknowns l1 and l2
        double z1 = 0.0, ph1 = 0.0, ps1 = 1.0, z2 = 0.0, ph2 = 1.0, ps2 = 0.0;
        double g1 = 0.0, g2 = 0.0, h1 = 0.0, h2 = 0.0;
        double sgz = 0.0, sgph = 0.0, sgps = 0.0, shz = 0.0, shph = 0.0, shps = 0.0;
        // the solve pass keeps per-position factors in registers (full unroll); the
        // relations pass needs none and, off the interior path, is only partly unrolled
        constexpr int UNR = SOLVE ? SUB : (FAST ? (DIR == 0 ? K1Y_FAST_UNROLL : K1X_FAST_UNROLL) : K1_UNROLL);
#pragma unroll UNR
        for (int k = 0; k < SUB; ++k) {
            if (FAST || k < len) {
                const int lp = ps + k;
                const int gp = pbase + lp;          // wave-uniform
                const CellS cp = cell_s<DIR, KM>(sU, p, lane, lp + 1);
                const FaceS fp = face_s<DIR == 0>(c0, cp, FAST || gp < Np - 1, ka);
                double rhs;
                if (DIR == 0) {
                    // -G(u_k) = -(u_k - b^n + theta dt D(u_k)); the x faces of this cell
                    // use the neighbouring lanes' cell values
                    const double eu = lane_next(c0.u), el = lane_next(c0.lap);
                    const double e0 = lane_next(c0.f0), e1 = lane_next(c0.f1);
                    const double Fe0 = __builtin_fma(c0.f0 + e0, el - c0.lap, (c0.f1 + e1) * (eu - c0.u));
                    const double Fe = feok ? Fe0 : 0.0;
                    const double Fwr = lane_prev(Fe);
                    const double Fw = (FAST || gl > 0) ? Fwr : 0.0;
                    const double D = (Fe - Fw) + (fp.F - fm.F);
                    // b^n with the edge correction (in the staged tile for the solve pass)
                    const double bn = SOLVE ? sB[lp * WPITCH + lane] : bcol[(size_t)gp * p.nx] + corr[lp];
                    const double G = __builtin_fma(ka, D, c0.u - bn);
                    rhs = -G;
                    if (!SOLVE && owned) {
                        rmax = fmax(rmax, fabs(G));
                        if (G != G) flags |= FLAG_NAN;
                    }
                } else {
                    rhs = WG ? bcol[k] : sB[lane * WPITCH + lp];
                }
                // bands of I + c J along the line from the two face records
                double a = fm.kA;
                double b = __builtin_fma(-3.0, fm.kA, -fp.kA) - fm.P;
                double c = __builtin_fma(3.0, fp.kA + fm.kA, 1.0) + (fp.P - fm.Q);
                double d = __builtin_fma(-3.0, fp.kA, fp.Q) - fm.kA;
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
                const double rm = rcp_pivot(mu);
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
                    fa[k] = al; fb[k] = be; fz[k] = z; fph[k] = ph;
                    // y solve: the coefficient of l2 is parked in the LDS slot of the b^n value
                    // just consumed (only this wave reads its positions' slots)
                    if (DIR == 0) sB[lp * WPITCH + lane] = pss;
                    else fps[k] = pss;
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

// Stage the haloed u tile and (STAGE_B) the tile of the second input (b^n or w) in LDS.
// Tile row ly holds grid row y0 - HALO + ly (u) or y0 + ly (second input); tile column lx
// holds grid column bxo - HALO + lx (u) or bxo + lx. Every load covers (part of) one grid row, so its row
// address is wave-uniform and only the column offset is per lane; all global loads are
// issued before the first LDS store. Only the u cells the sweeps read are staged:
// rows 0..67 (y sweep) or 1..66 (x sweep) of all 68 columns.
template <int DIR, bool STAGE_B>
__device__ __forceinline__ void stage_tile(const PassParams &p, double *sU, double *sB, int bxo, int y0, int wave,
                                           int lane)
{
    constexpr int LX0 = HALO;                     // tile column of lane 0 in a row load
    constexpr int RU0 = DIR == 0 ? 0 : 1;         // first u tile row read by the sweeps
    constexpr int NRU = DIR == 0 ? TW : TW - 2;   // u tile rows read by the sweeps
    constexpr int KU = (NRU + NSUB - 1) / NSUB;   // row loads per wave
    constexpr int KB = TILE / NSUB;
    // the columns outside the lanes' span: 2 on each side of every row
    constexpr int XPR = 2 * HALO;
    constexpr int NX = NRU * XPR;
    constexpr int KX = (NX + BLOCK - 1) / BLOCK;  // packed extra loads per wave
    const int nx = p.nx, ny = p.ny;
    const unsigned cu = (unsigned)crefl(bxo - HALO + LX0 + lane, nx);
    const unsigned cb = (unsigned)crefl(bxo + lane, nx);
    double vu[KU], vb[KB], vx[KX];
#pragma unroll
    for (int k = 0; k < KU; ++k) {
        const int ly = RU0 + wave + NSUB * k;
        if (ly < RU0 + NRU) {
            const int gy = crefl(y0 - HALO + ly, ny);
            vu[k] = (p.u + (size_t)gy * nx)[cu];
        }
    }
#pragma unroll
    for (int k = 0; k < KB; ++k) {
        if (STAGE_B) {
            const int gy = min(y0 + wave + NSUB * k, ny - 1);
            vb[k] = (p.in2 + (size_t)gy * nx)[cb];
        }
    }
    int xoff[KX];
#pragma unroll
    for (int k = 0; k < KX; ++k) {
        const int idx = (wave + NSUB * k) * 64 + lane;
        xoff[k] = -1;
        if (idx < NX) {
            const int ly = RU0 + idx / XPR, q = idx % XPR;
            const int lx = q < HALO ? q : TILE + q;
            const int gy = crefl(y0 - HALO + ly, ny), gx = crefl(bxo - HALO + lx, nx);
            vx[k] = p.u[(size_t)gy * nx + gx];
            xoff[k] = ly * UPITCH + lx;
        }
    }
#pragma unroll
    for (int k = 0; k < KU; ++k) {
        const int ly = RU0 + wave + NSUB * k;
        if (ly < RU0 + NRU) sU[ly * UPITCH + LX0 + lane] = vu[k];
    }
#pragma unroll
    for (int k = 0; k < KB; ++k)
        if (STAGE_B) sB[(wave + NSUB * k) * WPITCH + lane] = vb[k];
#pragma unroll
    for (int k = 0; k < KX; ++k)
        if (xoff[k] >= 0) sU[xoff[k]] = vx[k];
}

template <int DIR, bool SOLVE, int KM>
__device__ __forceinline__ void tile_body(const PassParams &p, int tx, int ty)
{
    // LDS: the u tile, then (solve passes) the tile of the second input (b^n, w) which
    // is later reused for the relation exchange and (x solve) the output tile. The
    // relations passes exchange in the u tile once the sweeps are done; they read their
    // right-hand side straight from global memory (y: lanes cover consecutive x; x: each
    // lane walks its row), which keeps their LDS footprint at one tile, so that three or
    // four workgroups fit on a CU.
    constexpr int NU = TW * UPITCH, NX = NSUB * NREL * 64, NW = TILE * WPITCH;
    constexpr bool STAGE_B = SOLVE;
    // y solve: the b^n tile keeps the parked factors, so its exchange goes to the u tile
    // (without the never-used bottom pair of the last sub-segment)
    constexpr bool XU = DIR == 0 && SOLVE;
    constexpr int NLDS = XU ? NU + NW : (SOLVE ? NU + NX : (STAGE_B ? NU + NW : NU));
    static_assert(NX >= NW && NU >= (NSUB - 1) * NREL * 64 + 10 * 64, "LDS regions too small");
    __shared__ double lds[NLDS];
    __shared__ double sRed[NSUB];
    __shared__ unsigned sFlag[NSUB];
    // y relations pass: b^n corrections of lane 0, lane 63 and (zeros) the other lanes
    __shared__ double sCorr[DIR == 0 && !SOLVE ? 3 * TILE : 1];
    double *const sU = lds;
    double *const sB = lds + NU;                 // second input, then exchange / output
    double *const xch = (SOLVE && !XU) ? sB : lds; // relation exchange

    const int nx = p.nx, ny = p.ny;
    int x0, x1, y0, y1;
    if (DIR == 0) {
        x0 = tx * TILE; x1 = min(x0 + TILE, nx);
        y0 = seg_start(ty, ny); y1 = seg_start(ty + 1, ny);
    } else {
        x0 = seg_start(tx, nx); x1 = seg_start(tx + 1, nx);
        y0 = ty * TILE; y1 = min(y0 + TILE, ny);
    }
    const int bxo = x0;  // grid x of lane/position 0 of the tile
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    stage_tile<DIR, STAGE_B>(p, sU, sB, bxo, y0, wave, lane);
    __syncthreads();

    const int nlt = DIR == 0 ? x1 - x0 : y1 - y0;       // lines owned by the tile
    const bool owned = lane < nlt;
    const int gl = (DIR == 0 ? x0 : y0) + lane;         // grid line of this lane
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

    // y sweep: the residual's x faces come from lane shuffles, so lanes 0 and 63 see zero flux
    // through the tile's edge faces x0-1 | x0 and x0+63 | x0+64. That is made up for in b^n
    // (G = u - b^n + ka D): at every position of the tile the edge face's flux F is formed
    // here with the in-wave arithmetic, and ka F (lane 0) or -ka F (lane 63) is added to the
    // lane's b^n, in the staged tile (solve) or as the sweep reads it (relations), the same
    // sum in both passes. Faces on the domain edge carry no flux and take no correction; a
    // flat film gets F = 0 and stays exact.
    if (DIR == 0) {
        if (tid < 2 * TILE) {
            const bool right = tid >= TILE;
            const int l = right ? TILE - 1 : -1, q = tid & (TILE - 1);
            if (q < npos) {
                const CellS L = cell_s<DIR, KM>(sU, p, l, q), R = cell_s<DIR, KM>(sU, p, l + 1, q);
                const double F = __builtin_fma(L.f0 + R.f0, R.lap - L.lap, (L.f1 + R.f1) * (R.u - L.u));
                const bool inner = right ? x1 < nx : x0 > 0;
                const double c = !inner ? 0.0 : (right ? -(p.ka * F) : p.ka * F);
                if (SOLVE && inner) sB[q * WPITCH + (right ? TILE - 1 : 0)] += c;
                if (!SOLVE) sCorr[tid] = c;
            }
        } else if (!SOLVE && tid < 3 * TILE) {
            sCorr[tid] = 0.0;
        }
        __syncthreads();
    }

    // interior tiles take the specialised path (wave-uniform branch)
    const bool fast = npos == TILE && pbase >= 2 && pbase + TILE <= Np - 2
                      && (DIR == 1 || (x0 > 0 && x1 < nx));
    // per-lane column of b^n for the y relations pass (read from global memory)
    const double *bcol = DIR == 0 ? p.in2 + crefl(bxo + lane, nx)
                                  : p.in2 + (size_t)min(y0 + lane, ny - 1) * nx + (x0 + ps);
    if (len > 0) {
        if (fast)
            sweep<DIR, SOLVE, KM, true>(sU, sB, sCorr, bcol, p, lane, ps, len, pbase, Np, gl, Nl, owned, fa, fb, fz, fph,
                                         fps, mine, rmax, flags);
        else
            sweep<DIR, SOLVE, KM, false>(sU, sB, sCorr, bcol, p, lane, ps, len, pbase, Np, gl, Nl, owned, fa, fb, fz, fph,
                                          fps, mine, rmax, flags);
    }

    if (!SOLVE && DIR == 0 && p.res != nullptr) {
        const double wm = wave_max(rmax);
        const unsigned wf = wave_or(flags);
        if (lane == 0) { sRed[wave] = wm; sFlag[wave] = wf; }
    }
    // solve pass: the tile's outer boundary values (from the chain) are loaded now, so
    // that their latency overlaps the relation exchange
    double l1 = 0.0, l2 = 0.0, r1 = 0.0, r2 = 0.0;
    if (SOLVE && len > 0) {
        const double *ex = p.ext + (size_t)qseg * NEXT * Nl;
        const unsigned gc = (unsigned)min(max(gl, 0), Nl - 1);
        l1 = ex[gc]; l2 = (ex + (size_t)Nl)[gc];
        r1 = (ex + (size_t)2 * Nl)[gc]; r2 = (ex + (size_t)3 * Nl)[gc];
    }
    __syncthreads(); // all sweeps done: the exchange area may be overwritten
    // the relations pass hands the records of waves 1.. to wave 0, which keeps its own
    const int xslot = SOLVE ? wave : wave - 1;
    if (len > 0 && xslot >= 0) {
        double *dst = xch + (size_t)xslot * NREL * 64 + lane;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 5; ++j) {
                dst[(i * 5 + j) * 64] = mine.T[i][j];
                if (!XU || wave < NSUB - 1) dst[(10 + i * 5 + j) * 64] = mine.B[i][j];
            }
    }
    __syncthreads();

    if (!SOLVE) {
        if (DIR == 0 && p.res != nullptr && tid == 0) {
            double m = 0.0;
            unsigned f = 0;
            for (int w = 0; w < NSUB; ++w) { m = fmax(m, sRed[w]); f |= sFlag[w]; }
            unsigned long long *rs = p.res + (size_t)(blockIdx.x % p.res_spread) * RES_WORDS;
            atomicMax(&rs[RES_RMAX], (unsigned long long)__double_as_longlong(m));
            if (f) atomicOr(&rs[RES_FLAGS], (unsigned long long)f);
        }
        if (wave == 0 && owned) {
            Rel seg;
            chain_symbolic(mine, xch, lane, nsub, seg);
            rel_store(p.rel + (size_t)qseg * NREL * Nl + 2 * (size_t)(unsigned)gl, Nl, seg);
        }
        return;
    }

    // ---- SOLVE: boundary values of this wave's sub-segment, then back-substitution
    double wl1 = 0.0, wl2 = 0.0, xr1 = 0.0, xr2 = 0.0;
    if (len > 0) chain_numeric<XU>(xch, lane, nsub, wave, l1, l2, r1, r2, wl1, wl2, xr1, xr2);

    if (DIR == 0) {
        // w goes straight from registers to memory: lanes cover consecutive x
        if (len > 0) {
#pragma unroll
            for (int k = SUB - 1; k >= 0; --k) {
                if (k < len) {
                    const double x = fz[k] + fph[k] * wl1 + sB[(ps + k) * WPITCH + lane] * wl2 - fa[k] * xr1 - fb[k] * xr2;
                    if (owned) (p.out + (size_t)(pbase + ps + k) * nx)[(unsigned)gl] = x;
                    xr2 = xr1;
                    xr1 = x;
                }
            }
        }
        return;
    } else {
        __syncthreads(); // relation records consumed: sB becomes the output staging tile
        // back-substitution stages v; u_{k+1} = u_k + v, the update ratio and the flags
        // are formed in the row-wise store loop (u_k from the LDS u tile)
        if (len > 0) {
#pragma unroll
            for (int k = SUB - 1; k >= 0; --k) {
                if (k < len) {
                    const double v = fz[k] + fph[k] * wl1 + fps[k] * wl2 - fa[k] * xr1 - fb[k] * xr2;
                    xr2 = xr1;
                    xr1 = v;
                    sB[lane * WPITCH + ps + k] = v;
                }
            }
        }
        __syncthreads();
        double emax = 0.0;
        // mass diagnostic of the iterate (wave-uniform switch): compensated sum and minimum
        const bool diag = p.mass != nullptr;
        double ms = 0.0, mc = 0.0, mmin = __builtin_inf();
#pragma unroll
        for (int r = 0; r < TILE / NSUB; ++r) {
            const int ly = wave + NSUB * r;
            if (ly < nlt && lane < npos) {
                const double v = sB[ly * WPITCH + lane];
                const double uk = uat<DIR>(sU, ly, lane);
                const double un = uk + v;
                emax = fmax(emax, fabs(v) * rcp(fabs(uk)));
                if (!(un > 0.0)) flags |= (un != un || v != v) ? FLAG_NAN : FLAG_NONPOS;
                (p.out + (size_t)(y0 + ly) * nx + x0)[(unsigned)lane] = un;
                if (diag) {
                    two_sum_acc(ms, mc, un);
                    mmin = fmin(mmin, un);
                }
            }
        }
        const double wm = wave_max(emax);
        const unsigned wf = wave_or(flags);
        if (lane == 0 && p.res != nullptr) {
            unsigned long long *rs = p.res + (size_t)((blockIdx.x * NSUB + wave) % p.res_spread) * RES_WORDS;
            atomicMax(&rs[RES_EMAX], (unsigned long long)__double_as_longlong(wm));
            if (wf) atomicOr(&rs[RES_FLAGS], (unsigned long long)wf);
        }
        if (diag) {
            // fixed-order butterfly over the lanes, then the four waves in order: the tile's
            // record does not depend on scheduling
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                comp_add(ms, mc, __shfl_xor(ms, o), __shfl_xor(mc, o));
                mmin = fmin(mmin, __shfl_xor(mmin, o));
            }
            __syncthreads(); // the output tile is no longer read
            if (lane == 0) {
                sB[3 * wave] = ms;
                sB[3 * wave + 1] = mc;
                sB[3 * wave + 2] = mmin;
            }
            __syncthreads();
            if (tid == 0) {
                double s = sB[0], c = sB[1], m = sB[2];
                for (int w = 1; w < NSUB; ++w) {
                    comp_add(s, c, sB[3 * w], sB[3 * w + 1]);
                    m = fmin(m, sB[3 * w + 2]);
                }
                double *o = p.mass + 4 * ((size_t)ty * p.tiles_x + tx);
                o[0] = s;
                o[1] = c;
                o[2] = m;
                o[3] = 0.0;
            }
        }
    }
}

#define TF_PASS_ATTR                                                                         \
    __launch_bounds__(BLOCK)                                                                 \
    __attribute__((amdgpu_waves_per_eu(TF_PASS_WPE, TF_PASS_WPE)))
// waves per SIMD each pass is compiled for (pass_waves_per_eu): the relations passes of the
// n = 3, m = 2 model fit in 128 VGPRs (their LDS footprint admits 4 workgroups per CU); the
// solve passes hold their factors in registers
#define TF_PASS_WPE pass_waves_per_eu(DIR, SOLVE, KM)
// (NLC and polymer chosen by timing at 8192^2: they need more registers per wave, the y
// relations pass of NLC the most; the linear model fits the n = 3, m = 2 budget, the
// general power law 168 VGPRs)
constexpr int pass_waves_per_eu(int dir, bool solve, int km)
{
    return solve ? K3_WAVES_PER_EU
                 : (km == KM_P32 || km == KM_LINEAR) ? (dir == 0 ? K1Y_WAVES_PER_EU : K1X_WAVES_PER_EU)
                 : km == KM_NLC ? (dir == 0 ? 2 : 3)
                 : 3;
}

template <int DIR, bool SOLVE, int KM>
__global__ void TF_PASS_ATTR k_pass(PassParams p)
{
    if (p.res_clear != nullptr && blockIdx.x == 0)
        for (int i = threadIdx.x; i < p.res_spread * RES_WORDS; i += BLOCK) p.res_clear[i] = 0ull;
    const int t = xcd_tile(blockIdx.x, p.tiles_x * p.tiles_y);
    tile_body<DIR, SOLVE, KM>(p, t % p.tiles_x, t / p.tiles_x);
}

// Ensemble version: block -> (film, tile) from the work list; the film's geometry,
// model, dt and buffer rotation come from the device tables, so one launch (and one
// captured graph) serves every film. Films that are not iterating exit at once.
template <int DIR, bool SOLVE, int KM>
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
    p.ids2 = 1.0 / (d.ds * d.ds);
    p.f0s = p.ids2 * d.M.cap;
    p.ka = 0.5 * e.theta * s->dt * p.ids2;
    p.K0 = 3.0 * p.ka * p.ids2 * d.M.cap;
    p.K1 = p.ka * d.M.Dn;
    p.M = d.M;
    p.u = B[s->it] + d.off;
    p.in2 = DIR == 0 ? (e.theta < 1.0 ? e.bn : B[s->cur]) + d.off : e.w + d.off;
    p.out = DIR == 0 ? e.w + d.off : B[s->nxt] + d.off;
    p.rel = e.rel + d.roff * NREL;
    p.ext = e.ext + d.roff * NEXT;
    p.res = s->red;
    p.res_spread = ENS_RES_SPREAD;
    tile_body<DIR, SOLVE, KM>(p, tx, ty);
}

// ------------------------------------------------------------------------------------
// Interface chain. Per line, the segment relations
//   T_q = t_q + Tl_q B_{q-1} + Tr_q T_{q+1},   B_q = b_q + Bl_q B_{q-1} + Br_q T_{q+1}
// (T_q, B_q: top and bottom pairs of segment q; B_{-1} = T_P = 0 at the line ends)
// form a block-tridiagonal system in 2x2 blocks. It is eliminated from both ends at
// once: one wave sweeps segments 0..m-1 forward,
//   B_q = bt_q + M_q T_{q+1},  T_q = tau_q + N_q T_{q+1},
// the other sweeps segments P-1..m backward,
//   T_q = tt_q + R_q B_{q-1},  B_q = bb_q + S_q B_{q-1},
// the two meet at the pair (B_{m-1}, T_m), and each substitutes back over its half,
// giving every segment its two left (B_{q-1}) and two right (T_{q+1}) neighbours.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void load_rec(const double *r, size_t NL, double (&T)[2][5], double (&B)[2][5])
{
    Rel S;
    rel_fetch(r, NL, S);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            T[i][j] = S.T[i][j];
            B[i][j] = S.B[i][j];
        }
}

// Six fields (a0, a1, X) of a chain record from field 0 of `w` (paired layout).
__device__ __forceinline__ void store6(double *w, size_t NL, double a0, double a1, const M2 &X)
{
    rec_put2(w, NL, 0, a0, a1);
    rec_put2(w, NL, 1, X.a, X.b);
    rec_put2(w, NL, 2, X.c, X.d);
}

// Meeting record of one line: the forward wave leaves (bt_{m-1}, M_{m-1}), the backward
// wave (tt_m, R_m).
struct ChainMeet {
    double v[12][64];
};

// Records are loaded CHAIN_DEPTH segments ahead of their use (register rings indexed
// statically through the unrolled inner loops): the chain is bound by memory latency. Four
// segments (a ring of 40 doubles per lane, 203 VGPRs) measured faster than eight at 2048
// lines and the same at 8192.
#ifndef CHAIN_DEPTH
#define CHAIN_DEPTH 4
#endif

__device__ __forceinline__ void chain_line(const ChainParams &c, int line, int wave, int lane, ChainMeet &mt)
{
    constexpr int D = CHAIN_DEPTH;
    const size_t NL = (size_t)c.nlines;
    const size_t RS = (size_t)NREL * NL, CS = (size_t)NCHAIN * NL, ES = (size_t)NEXT * NL;
    const int P = c.P, m = P / 2;
    const bool live = line < c.nlines;
    const double *rb = c.rel + 2 * (size_t)line;
    double *cb = c.chain + 2 * (size_t)line;
    double *eb = c.ext + line;
    double x0 = 0.0, x1 = 0.0;   // wave 0: bt_q; wave 1: tt_q
    M2 X = {0, 0, 0, 0};         // wave 0: M_q;  wave 1: R_q
    if (live) {
        double RT[D][2][5], RB[D][2][5];
        if (wave == 0) {
            // forward over q = 0..m-1: chain record (tau_q, N_q, bt_q, M_q)
#pragma unroll
            for (int j = 0; j < D; ++j)
                if (j < m) load_rec(rb + (size_t)j * RS, NL, RT[j], RB[j]);
            for (int q0 = 0; q0 < m; q0 += D) {
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const int q = q0 + j;
                    if (q < m) {
                        const double(&T)[2][5] = RT[j];
                        const double(&B)[2][5] = RB[j];
                        const M2 Tl = {T[0][1], T[0][2], T[1][1], T[1][2]}, Tr = {T[0][3], T[0][4], T[1][3], T[1][4]};
                        const M2 Bl = {B[0][1], B[0][2], B[1][1], B[1][2]}, Br = {B[0][3], B[0][4], B[1][3], B[1][4]};
                        double tau0, tau1;
                        M2 N;
                        if (q == 0) {
                            tau0 = T[0][0]; tau1 = T[1][0]; N = Tr;
                            x0 = B[0][0]; x1 = B[1][0]; X = Br;
                        } else {
                            const M2 K = inv_i_minus(mul(Tl, X));
                            const double s0 = T[0][0] + Tl.a * x0 + Tl.b * x1;
                            const double s1 = T[1][0] + Tl.c * x0 + Tl.d * x1;
                            tau0 = K.a * s0 + K.b * s1;
                            tau1 = K.c * s0 + K.d * s1;
                            N = mul(K, Tr);
                            const double v0 = x0 + X.a * tau0 + X.b * tau1;
                            const double v1 = x1 + X.c * tau0 + X.d * tau1;
                            const M2 BM = mul(mul(Bl, X), N);
                            x0 = B[0][0] + Bl.a * v0 + Bl.b * v1;
                            x1 = B[1][0] + Bl.c * v0 + Bl.d * v1;
                            X = {BM.a + Br.a, BM.b + Br.b, BM.c + Br.c, BM.d + Br.d};
                        }
                        double *w = cb + (size_t)q * CS;
                        store6(w, NL, tau0, tau1, N);
                        store6(w + 6 * NL, NL, x0, x1, X);
                        if (q + D < m) load_rec(rb + (size_t)(q + D) * RS, NL, RT[j], RB[j]);
                    }
                }
            }
        } else {
            // backward over q = P-1..m: chain record (tt_q, R_q, bb_q, S_q)
            const int nb = P - m;  // segments of this half; step i handles q = P-1-i
#pragma unroll
            for (int j = 0; j < D; ++j)
                if (j < nb) load_rec(rb + (size_t)(P - 1 - j) * RS, NL, RT[j], RB[j]);
            for (int i0 = 0; i0 < nb; i0 += D) {
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const int i = i0 + j, q = P - 1 - i;
                    if (i < nb) {
                        const double(&T)[2][5] = RT[j];
                        const double(&B)[2][5] = RB[j];
                        const M2 Tl = {T[0][1], T[0][2], T[1][1], T[1][2]}, Tr = {T[0][3], T[0][4], T[1][3], T[1][4]};
                        const M2 Bl = {B[0][1], B[0][2], B[1][1], B[1][2]}, Br = {B[0][3], B[0][4], B[1][3], B[1][4]};
                        double bb0, bb1;
                        M2 S;
                        if (i == 0) {
                            bb0 = B[0][0]; bb1 = B[1][0]; S = Bl;
                            x0 = T[0][0]; x1 = T[1][0]; X = Tl;
                        } else {
                            const M2 K = inv_i_minus(mul(Br, X));
                            const double s0 = B[0][0] + Br.a * x0 + Br.b * x1;
                            const double s1 = B[1][0] + Br.c * x0 + Br.d * x1;
                            bb0 = K.a * s0 + K.b * s1;
                            bb1 = K.c * s0 + K.d * s1;
                            S = mul(K, Bl);
                            const double v0 = x0 + X.a * bb0 + X.b * bb1;
                            const double v1 = x1 + X.c * bb0 + X.d * bb1;
                            const M2 TRS = mul(mul(Tr, X), S);
                            x0 = T[0][0] + Tr.a * v0 + Tr.b * v1;
                            x1 = T[1][0] + Tr.c * v0 + Tr.d * v1;
                            X = {TRS.a + Tl.a, TRS.b + Tl.b, TRS.c + Tl.c, TRS.d + Tl.d};
                        }
                        double *w = cb + (size_t)q * CS;
                        store6(w, NL, x0, x1, X);
                        store6(w + 6 * NL, NL, bb0, bb1, S);
                        if (i + D < nb) load_rec(rb + (size_t)(q - D) * RS, NL, RT[j], RB[j]);
                    }
                }
            }
        }
    }
    // meet: B_{m-1} = bt + M T_m and T_m = tt + R B_{m-1}
    mt.v[wave * 6 + 0][lane] = x0; mt.v[wave * 6 + 1][lane] = x1;
    mt.v[wave * 6 + 2][lane] = X.a; mt.v[wave * 6 + 3][lane] = X.b;
    mt.v[wave * 6 + 4][lane] = X.c; mt.v[wave * 6 + 5][lane] = X.d;
    __syncthreads();
    if (!live) return;
    const double bt0 = mt.v[0][lane], bt1 = mt.v[1][lane];
    const M2 Mm = {mt.v[2][lane], mt.v[3][lane], mt.v[4][lane], mt.v[5][lane]};
    const double tt0 = mt.v[6][lane], tt1 = mt.v[7][lane];
    const M2 Rm = {mt.v[8][lane], mt.v[9][lane], mt.v[10][lane], mt.v[11][lane]};
    double Bm0 = 0.0, Bm1 = 0.0; // B_{m-1}
    if (m > 0) {
        const M2 K = inv_i_minus(mul(Mm, Rm));
        const double s0 = bt0 + Mm.a * tt0 + Mm.b * tt1, s1 = bt1 + Mm.c * tt0 + Mm.d * tt1;
        Bm0 = K.a * s0 + K.b * s1;
        Bm1 = K.c * s0 + K.d * s1;
    }
    const double Tm0 = tt0 + Rm.a * Bm0 + Rm.b * Bm1, Tm1 = tt1 + Rm.c * Bm0 + Rm.d * Bm1; // T_m
    // substitution rings: (a, A) of segment q and its neighbour's (p, Pq)
    double RA[D][6], RN[D][6];
    auto ld6 = [&](const double *w, double (&o)[6]) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double2 v = rec_get2(w, NL, k);
            o[2 * k] = v.x;
            o[2 * k + 1] = v.y;
        }
    };
    if (wave == 0) {
        // q = m-1..0: T_q = tau_q + N_q T_{q+1}, B_{q-1} = bt_{q-1} + M_{q-1} T_q
        double tn0 = Tm0, tn1 = Tm1;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int q = m - 1 - j;
            if (q >= 0) ld6(cb + (size_t)q * CS, RA[j]);
            if (q >= 1) ld6(cb + (size_t)(q - 1) * CS + 6 * NL, RN[j]);
        }
        for (int i0 = 0; i0 < m; i0 += D) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int i = i0 + j, q = m - 1 - i;
                if (i < m) {
                    const double(&a)[6] = RA[j];
                    const double(&pn)[6] = RN[j];
                    const double t0 = a[0] + a[2] * tn0 + a[3] * tn1;
                    const double t1 = a[1] + a[4] * tn0 + a[5] * tn1;
                    double *e = eb + (size_t)q * ES;
                    e[2 * NL] = tn0;
                    e[3 * NL] = tn1;
                    e[0] = q > 0 ? pn[0] + pn[2] * t0 + pn[3] * t1 : 0.0;
                    e[NL] = q > 0 ? pn[1] + pn[4] * t0 + pn[5] * t1 : 0.0;
                    tn0 = t0; tn1 = t1;
                    const int qn = q - D;
                    if (qn >= 0) ld6(cb + (size_t)qn * CS, RA[j]);
                    if (qn >= 1) ld6(cb + (size_t)(qn - 1) * CS + 6 * NL, RN[j]);
                }
            }
        }
    } else {
        // q = m..P-1: B_q = bb_q + S_q B_{q-1}, T_{q+1} = tt_{q+1} + R_{q+1} B_q
        double bp0 = Bm0, bp1 = Bm1;
        const int nb = P - m;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int q = m + j;
            if (q < P) ld6(cb + (size_t)q * CS + 6 * NL, RA[j]);
            if (q + 1 < P) ld6(cb + (size_t)(q + 1) * CS, RN[j]);
        }
        for (int i0 = 0; i0 < nb; i0 += D) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const int i = i0 + j, q = m + i;
                if (i < nb) {
                    const double(&a)[6] = RA[j];
                    const double(&rn)[6] = RN[j];
                    const double b0 = a[0] + a[2] * bp0 + a[3] * bp1;
                    const double b1 = a[1] + a[4] * bp0 + a[5] * bp1;
                    double *e = eb + (size_t)q * ES;
                    e[0] = bp0;
                    e[NL] = bp1;
                    e[2 * NL] = q + 1 < P ? rn[0] + rn[2] * b0 + rn[3] * b1 : 0.0;
                    e[3 * NL] = q + 1 < P ? rn[1] + rn[4] * b0 + rn[5] * b1 : 0.0;
                    bp0 = b0; bp1 = b1;
                    const int qn = q + D;
                    if (qn < P) ld6(cb + (size_t)qn * CS + 6 * NL, RA[j]);
                    if (qn + 1 < P) ld6(cb + (size_t)(qn + 1) * CS, RN[j]);
                }
            }
        }
    }
}

__global__ void __launch_bounds__(128) k_chain(ChainParams c)
{
    __shared__ ChainMeet mt;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    chain_line(c, blockIdx.x * 64 + lane, wave, lane, mt);
}

// Ensemble version: block -> (film, block of 64 lines); dir 0 chains the y sweep.
__global__ void __launch_bounds__(128) k_chain_ens(EnsParams e, int dir)
{
    __shared__ ChainMeet mt;
    const int f = e.items[2 * blockIdx.x], lb = e.items[2 * blockIdx.x + 1];
    const FilmState *s = e.state + f;
    if (!s->active) return;
    const FilmDesc d = e.desc[f];
    ChainParams c{dir == 0 ? d.nx : d.ny, dir == 0 ? d.Py : d.Px, e.rel + d.roff * NREL, e.chain + d.roff * NCHAIN,
                  e.ext + d.roff * NEXT};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    chain_line(c, lb * 64 + lane, wave, lane, mt);
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

// D(u) at cell (i, j): the flux differences of eq. GovEqnCell2 with zero boundary fluxes
// (NOF0: the f1 part only).
template <bool P32, bool NOF0>
__device__ __forceinline__ double flux_div_at(const double *u, int nx, int ny, int i, int j, double ids, double ids2,
                                              const Model &M)
{
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
    return (F[1] - F[0] + F[3] - F[2]) * ids;
}

template <bool P32, bool NOF0>
__global__ void __launch_bounds__(256) k_flux_divergence(int nx, int ny, double ids, double ids2, Model M,
                                                         const double *u, double alpha, double beta,
                                                         const double *add, double *out)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= nx || j >= ny) return;
    const double D = flux_div_at<P32, NOF0>(u, nx, ny, i, j, ids, ids2, M);
    const size_t o = (size_t)j * nx + i;
    out[o] = (add != nullptr ? alpha * add[o] : 0.0) + beta * D;
}

// Ensemble b^n = u^n - (1 - theta) dt D(u^n), block -> one y-sweep tile (TILE columns x one
// segment of rows) of a film that is active and at the first iteration of its attempt (the
// same arithmetic as k_flux_divergence with alpha = 1, so the ensemble matches the single film).
__global__ void __launch_bounds__(256) k_bn_ens(EnsParams e)
{
    const int t = xcd_tile(blockIdx.x, e.nitems);
    const int f = e.items[3 * t], tx = e.items[3 * t + 1], ty = e.items[3 * t + 2];
    const FilmState *s = e.state + f;
    if (!s->active || s->k != 0) return;
    const FilmDesc d = e.desc[f];
    const double *B[3] = {e.buf0, e.buf1, e.buf2};
    const double *un = B[s->cur] + d.off;
    double *bn = e.bn + d.off;
    const double ids = 1.0 / d.ds, ids2 = ids * ids;
    const double beta = -(1.0 - e.theta) * s->dt;
    const int i0 = tx * TILE, i1 = min(i0 + TILE, d.nx);
    const int j0 = seg_start(ty, d.ny), j1 = seg_start(ty + 1, d.ny);
    const int w = i1 - i0;
    for (int c = threadIdx.x; c < w * (j1 - j0); c += 256) {
        const int i = i0 + c % w, j = j0 + c / w;
        const double D = d.M.p32 ? flux_div_at<true, false>(un, d.nx, d.ny, i, j, ids, ids2, d.M)
                                 : flux_div_at<false, false>(un, d.nx, d.ny, i, j, ids, ids2, d.M);
        const size_t o = (size_t)j * d.nx + i;
        bn[o] = un[o] + beta * D; // fma(beta, D, u), as in k_flux_divergence
    }
}

// ------------------------------------------------------------------------------------
// Mass diagnostic: per-block compensated (Neumaier) sum, minimum and NaN flag, reduced
// in a fixed tree order; the host adds the block records in index order.
// ------------------------------------------------------------------------------------
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


// Per-tile mass records of the x solve combined in a fixed order (strided per thread, then
// a tree): out = {sum, min}.
__global__ void __launch_bounds__(256) k_mass_tiles(const double *part, int ntiles, double *out)
{
    __shared__ double ss[256], sc[256], sm[256];
    double s = 0.0, c = 0.0, m = __builtin_inf();
    for (int i = threadIdx.x; i < ntiles; i += 256) {
        comp_add(s, c, part[4 * (size_t)i], part[4 * (size_t)i + 1]);
        m = fmin(m, part[4 * (size_t)i + 2]);
    }
    ss[threadIdx.x] = s; sc[threadIdx.x] = c; sm[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double a = ss[threadIdx.x], ca = sc[threadIdx.x];
            comp_add(a, ca, ss[threadIdx.x + w], sc[threadIdx.x + w]);
            ss[threadIdx.x] = a;
            sc[threadIdx.x] = ca;
            sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = ss[0] + sc[0];
        out[1] = sm[0];
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
        // combine the copies (maxima of non-negative doubles compare as bit patterns), clear them
        unsigned long long em = 0ull, rm = 0ull, flags = 0ull;
        for (int c = 0; c < ENS_RES_SPREAD; ++c) {
            unsigned long long *w = s.red + c * RES_WORDS;
            em = w[RES_EMAX] > em ? w[RES_EMAX] : em;
            rm = w[RES_RMAX] > rm ? w[RES_RMAX] : rm;
            flags |= w[RES_FLAGS];
            w[RES_EMAX] = 0ull;
            w[RES_RMAX] = 0ull;
            w[RES_FLAGS] = 0ull;
        }
        const double e = __longlong_as_double((long long)em);
        const double r = __longlong_as_double((long long)rm);
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
    for (int c = 0; c < ENS_RES_SPREAD; ++c) {
        s.red[c * RES_WORDS + RES_EMAX] = 0ull;
        s.red[c * RES_WORDS + RES_RMAX] = 0ull;
        s.red[c * RES_WORDS + RES_FLAGS] = 0ull;
    }
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
template <int KM>
static void launch_pass_km(int dir, bool solve, const PassParams &p, hipStream_t s)
{
    const dim3 grid(p.tiles_x * p.tiles_y), block(BLOCK);
    if (dir == 0 && !solve) k_pass<0, false, KM><<<grid, block, 0, s>>>(p);
    else if (dir == 0) k_pass<0, true, KM><<<grid, block, 0, s>>>(p);
    else if (!solve) k_pass<1, false, KM><<<grid, block, 0, s>>>(p);
    else k_pass<1, true, KM><<<grid, block, 0, s>>>(p);
}

hipError_t launch_pass(int dir, bool solve, const PassParams &p, hipStream_t s)
{
    switch (p.M.kind) {
    case MODEL_LINEAR: launch_pass_km<KM_LINEAR>(dir, solve, p, s); break;
    case MODEL_NLC: launch_pass_km<KM_NLC>(dir, solve, p, s); break;
    case MODEL_POLYMER: launch_pass_km<KM_POLYMER>(dir, solve, p, s); break;
    default:
        if (p.M.p32) launch_pass_km<KM_P32>(dir, solve, p, s);
        else launch_pass_km<KM_POWER>(dir, solve, p, s);
    }
    return hipGetLastError();
}

hipError_t launch_chain(const ChainParams &c, hipStream_t s)
{
    k_chain<<<dim3((c.nlines + 63) / 64), dim3(128), 0, s>>>(c);
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

// f0, f0', f1, f1' of the model at n thicknesses (out[4k + 0..3]).
__global__ void __launch_bounds__(256) k_model_coeffs(Model M, const double *__restrict__ h, int n,
                                                      double *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double f0, f1, f0p, f1p;
    model_coefs<false>(M, h[k], f0, f1, f0p, f1p);
    out[4 * k + 0] = f0;
    out[4 * k + 1] = f0p;
    out[4 * k + 2] = f1;
    out[4 * k + 3] = f1p;
}

hipError_t launch_model_coeffs(const Model &M, const double *h, int n, double *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_model_coeffs<<<(n + 255) / 256, 256, 0, s>>>(M, h, n, out);
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

hipError_t launch_mass_tiles(const double *part, int ntiles, double *out, hipStream_t s)
{
    k_mass_tiles<<<dim3(1), dim3(256), 0, s>>>(part, ntiles, out);
    return hipGetLastError();
}

} // namespace tf

namespace tf {

template <int KM>
static void launch_pass_ens_km(int dir, bool solve, const EnsParams &e, hipStream_t s)
{
    const dim3 grid(e.nitems), block(BLOCK);
    if (dir == 0 && !solve) k_pass_ens<0, false, KM><<<grid, block, 0, s>>>(e);
    else if (dir == 0) k_pass_ens<0, true, KM><<<grid, block, 0, s>>>(e);
    else if (!solve) k_pass_ens<1, false, KM><<<grid, block, 0, s>>>(e);
    else k_pass_ens<1, true, KM><<<grid, block, 0, s>>>(e);
}

// km: the KernelModel every film of the ensemble shares
hipError_t launch_pass_ens(int dir, bool solve, int km, const EnsParams &e, hipStream_t s)
{
    switch (km) {
    case KM_P32: launch_pass_ens_km<KM_P32>(dir, solve, e, s); break;
    case KM_POWER: launch_pass_ens_km<KM_POWER>(dir, solve, e, s); break;
    case KM_LINEAR: launch_pass_ens_km<KM_LINEAR>(dir, solve, e, s); break;
    case KM_NLC: launch_pass_ens_km<KM_NLC>(dir, solve, e, s); break;
    default: launch_pass_ens_km<KM_POLYMER>(dir, solve, e, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_bn_ens(const EnsParams &e, hipStream_t s)
{
    k_bn_ens<<<dim3(e.nitems), dim3(256), 0, s>>>(e);
    return hipGetLastError();
}

hipError_t launch_chain_ens(const EnsParams &e, int dir, hipStream_t s)
{
    k_chain_ens<<<dim3(e.nitems), dim3(128), 0, s>>>(e, dir);
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
