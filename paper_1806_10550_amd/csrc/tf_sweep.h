// Per-cell and per-face arithmetic of the forward line sweeps, shared by the tile
// kernels (tf_kernels.hip) and the whole-row kernel (tf_xrow.hip).
#pragma once

#include "tf_device.h"

namespace tf {

// Per-cell quantities of the sweeps, scaled so that each face record takes few
// operations (ka = c / (2 ds^2), c = theta dt):
//   lap = u_E + u_W + u_N + u_S - 4u      (ds^2 times the 5-point Laplacian)
//   f0  = cap h^3 / ds^2,   f1 = h^3 Pi'(h)
//   g0  = ka f0'(h) / ds^2,   g1 = ka f1'(h)
struct CellS {
    double u, lap, f0, f1, g0, g1;
};

// Cell quantities from the cell value u and lap (ds^2 times its 5-point Laplacian).
template <int KM>
__device__ __forceinline__ CellS cell_core(const PassParams &p, double u, double lap)
{
    CellS c;
    c.u = u;
    c.lap = lap;
    if constexpr (KM == KM_LINEAR) {
        c.f0 = p.f0s;
        c.g0 = 0.0;
        c.f1 = p.M.Cm;
        c.g1 = 0.0;
        return c;
    }
    const double r = rcp(c.u);
    const double u2 = c.u * c.u;
    c.f0 = (u2 * c.u) * p.f0s;
    c.g0 = p.K0 * u2;
    if constexpr (KM == KM_P32) {
        c.f1 = __builtin_fma(-p.M.Cn, r, p.M.Cm);
        c.g1 = p.K1 * (r * r);
    } else if constexpr (KM == KM_POWER) {
        // r^(m-1), r^(n-1) by fixed-step powering (0 <= m-1 < n-1 <= 15), then one
        // multiplication by h = 1/r for r^(m-2), r^(n-2)
        const Model &M = p.M;
        const double pm1 = pow16(r, M.m - 1), pn1 = pm1 * pow16(r, M.n - M.m);
        c.f1 = M.Cm * (pm1 * c.u) - M.Cn * (pn1 * c.u);
        c.g1 = p.ka * (M.Dn * pn1 - M.Dm * pm1);
    } else {
        double pip, pipp;
        if constexpr (KM == KM_NLC) nlc_derivs(p.M, c.u, r, pip, pipp);
        else polymer_derivs(p.M, c.u, r, pip, pipp);
        c.f1 = (u2 * c.u) * pip;
        c.g1 = p.ka * (3.0 * u2 * pip + (u2 * c.u) * pipp);
    }
    return c;
}

// Face record between the cells L and R of a line (raw differences Lam = lap_R - lap_L,
// Gam = u_R - u_L; A and B are the face means of f0 and f1):
//   kA = c A / ds^4,
//   P  = c/ds d(flux)/du_L without the fourth-difference part = ka (f0'_L Lam/ds^2 + f1'_L Gam - 2B),
//   Q  = the same for u_R with +2B,
//   F  = 2 ds times the face flux A (lap_R - lap_L)/ds^3 + B Gam/ds  (y sweep only).
// Boundary faces carry no flux: every entry is zero there.
struct FaceS {
    double kA, P, Q, F;
};

template <bool FLUX>
__device__ __forceinline__ FaceS face_s(const CellS &L, const CellS &R, bool interior, double ka)
{
    const double S0 = L.f0 + R.f0, S1 = L.f1 + R.f1;
    const double Lam = R.lap - L.lap, Gam = R.u - L.u;
    const double kS1 = ka * S1;
    FaceS f;
    f.kA = interior ? ka * S0 : 0.0;
    f.P = interior ? __builtin_fma(L.g0, Lam, __builtin_fma(L.g1, Gam, -kS1)) : 0.0;
    f.Q = interior ? __builtin_fma(R.g0, Lam, __builtin_fma(R.g1, Gam, kS1)) : 0.0;
    f.F = (FLUX && interior) ? __builtin_fma(S0, Lam, S1 * Gam) : 0.0;
    return f;
}

} // namespace tf
