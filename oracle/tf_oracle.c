/*
 * tf_oracle.c -- plain, slow CPU reference ("oracle") for the ADI-Newton time
 * step of the thin-film equation of Lam, Cummings & Kondic, "Computing dynamics
 * of thin films via large scale GPU-based simulations" (arXiv:1806.10550).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library. It shares no code, header or
 * constant with the GPU library; it is written from the paper's definitions in
 * the most direct form, in FP64, with no blocking, fusion or reordering:
 *
 *   cells, cell centres, flux form          Sec. "Conservation Law", eq. GovEqnCell2
 *   time discretisation (theta scheme)      Sec. "Temporal Discretization", eq. TrapRule
 *                                           (theta = 1/2 is the paper's rule, theta = 1 is
 *                                            backward Euler)
 *   Newton + ADI factorisation              eqs. NewtonIterativeForm, DirectionSplit,
 *                                           JacobianSystem1-3 (y solve, then x solve)
 *   acceptance test / adaptive dt           eq. NewtonError, Fig. FlowChartTime
 *   flux-difference operator D, J_x, J_y    Sec. "Flux Discretization"
 *   no-flux boundaries, ghost points        Sec. "Boundary Conditions"
 *   pentadiagonal line solves               Appendix A.3.1 (here: textbook band Gaussian
 *                                           elimination with partial pivoting)
 *   model f0 = h^3, f1 = kappa h^3 f'(h),   eq. GeneralDisPreForm with the power-law part
 *   f = (b/h)^n - (b/h)^m                   of eq. DisjPressNLC
 *   NLC model f0 = C h^3, f1 = h^3 Pi'(h)   eqs. GeneralDisPreForm, DisjPressNLC, mh_model
 *   polymer model, same f0, f1              eqs. GeneralDisPreForm, DisjPressPolymer
 *   linear test model f0 = c0, f1 = c1      Sec. "Thin Film Models"
 *
 * Readings of points the paper leaves open are listed where they are used.
 * Storage: u[j*nx + i], i along x (0..nx-1), j along y (0..ny-1), row-major.
 * Independent lines/cells are distributed over OpenMP threads; every result is
 * independent of the thread count (no floating-point reductions across threads
 * except exact maxima).
 */
#include <math.h>
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* status codes (same numeric meaning as the GPU library's, defined here on purpose) */
enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOMEM = 2, OR_ENOCONV = 4, OR_ENONPOS = 5, OR_ESINGULAR = 7 };
enum { OR_POWERLAW = 0, OR_LINEAR = 1, OR_NLC = 2, OR_POLYMER = 3 };

typedef struct {
    int kind;        /* OR_POWERLAW, OR_LINEAR, OR_NLC or OR_POLYMER */
    double kappa, b, n, m; /* power law: f(h) = (b/h)^n - (b/h)^m, f1 = kappa h^3 f'(h) */
    double c0, c1;   /* linear test model */
    double cap;      /* NLC / polymer: inverse capillary number C in f0 = C h^3 */
    double K, N, beta, w; /* NLC: Pi = K[(b/h)^3 - (b/h)^2] + N/2 (m(h)/h)^2 (b as above) */
    double Cst, Aox, Asi, d; /* polymer: psi = Cst/h^8 - Aox/(12 pi h^2) + (Aox - Asi)/(12 pi (h+d)^2) */
} or_model;

typedef struct {
    double theta, tol, dt_min, dt_max, dt_shrink, dt_grow;
    int max_newton, grow_after, adaptive;
} or_scheme;

typedef struct {
    double t, dt_used, e_final, r_final;
    int newton_iters, rejections, status, total_iters;
} or_step_info;

#define IDX(i, j) ((size_t)(j) * (size_t)nx + (size_t)(i))

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------------------
 * Model functions (eq. GeneralDisPreForm with the power-law disjoining pressure).
 * f0 = h^3, f1 = kappa h^3 f'(h), with f(h) = (b/h)^n - (b/h)^m, written out from
 * the definitions; f0', f1' are their h-derivatives.
 * ------------------------------------------------------------------------- */
/* Disjoining pressure Pi(h) and its first two derivatives for the NLC model (eqs.
 * DisjPressNLC, mh_model) and the polymer model (eq. DisjPressPolymer, Pi = -psi').
 * Written out from the definitions:
 *   NLC:  Pi = K (b^3 h^-3 - b^2 h^-2) + N/2 q^2,  q = m(h)/h = g(h) r(h),
 *         g = (1 + tanh z)/2, z = (h - 2b)/w,  r = h / (h^2 + beta^2);
 *   polymer: Pi = 8 Cst h^-9 - 2a h^-3 + 2c (h+d)^-3,  a = Aox/(12 pi), c = (Aox-Asi)/(12 pi). */
void or_disjoining(const or_model *M, double h, double *Pi, double *Pip, double *Pipp)
{
    if (M->kind == OR_NLC) {
        const double b = M->b, K = M->K, N = M->N, be2 = M->beta * M->beta, w = M->w;
        const double z = (h - 2.0 * b) / w, th = tanh(z), sech2 = 1.0 - th * th;
        const double g = 0.5 * (1.0 + th);
        const double gp = 0.5 * sech2 / w;
        const double gpp = -sech2 * th / (w * w);
        const double den = h * h + be2;
        const double r = h / den;
        const double rp = (be2 - h * h) / (den * den);
        const double rpp = 2.0 * h * (h * h - 3.0 * be2) / (den * den * den);
        const double q = g * r, qp = gp * r + g * rp, qpp = gpp * r + 2.0 * gp * rp + g * rpp;
        const double b2 = b * b, b3 = b2 * b;
        *Pi = K * (b3 / (h * h * h) - b2 / (h * h)) + 0.5 * N * q * q;
        *Pip = K * (-3.0 * b3 / pow(h, 4.0) + 2.0 * b2 / (h * h * h)) + N * q * qp;
        *Pipp = K * (12.0 * b3 / pow(h, 5.0) - 6.0 * b2 / pow(h, 4.0)) + N * (qp * qp + q * qpp);
    } else {
        const double a = M->Aox / (12.0 * M_PI), c = (M->Aox - M->Asi) / (12.0 * M_PI), hd = h + M->d;
        *Pi = 8.0 * M->Cst / pow(h, 9.0) - 2.0 * a / pow(h, 3.0) + 2.0 * c / pow(hd, 3.0);
        *Pip = -72.0 * M->Cst / pow(h, 10.0) + 6.0 * a / pow(h, 4.0) - 6.0 * c / pow(hd, 4.0);
        *Pipp = 720.0 * M->Cst / pow(h, 11.0) - 24.0 * a / pow(h, 5.0) + 24.0 * c / pow(hd, 5.0);
    }
}

void or_coeffs(const or_model *M, double h, double *f0, double *f0p, double *f1, double *f1p)
{
    if (M->kind == OR_LINEAR) {
        *f0 = M->c0; *f0p = 0.0; *f1 = M->c1; *f1p = 0.0;
        return;
    }
    if (M->kind == OR_NLC || M->kind == OR_POLYMER) {
        /* eq. GeneralDisPreForm read as f0 = C h^3, f1 = h^3 Pi'(h) (the form that gives the
         * growth rates printed with Fig. dispersion_curves) */
        double Pi, Pip, Pipp;
        or_disjoining(M, h, &Pi, &Pip, &Pipp);
        *f0 = M->cap * h * h * h;
        *f0p = 3.0 * M->cap * h * h;
        *f1 = h * h * h * Pip;
        *f1p = 3.0 * h * h * Pip + h * h * h * Pipp;
        return;
    }
    const double n = M->n, m = M->m, b = M->b;
    /* f'(h)  = -n b^n h^(-n-1) + m b^m h^(-m-1)
     * f''(h) =  n(n+1) b^n h^(-n-2) - m(m+1) b^m h^(-m-2) */
    const double fp  = -n * pow(b, n) * pow(h, -n - 1.0) + m * pow(b, m) * pow(h, -m - 1.0);
    const double fpp =  n * (n + 1.0) * pow(b, n) * pow(h, -n - 2.0)
                      - m * (m + 1.0) * pow(b, m) * pow(h, -m - 2.0);
    *f0  = h * h * h;
    *f0p = 3.0 * h * h;
    *f1  = M->kappa * h * h * h * fp;
    *f1p = M->kappa * (3.0 * h * h * fp + h * h * h * fpp);
}

/* Ghost values by even reflection across the boundary faces (Sec. "Boundary
 * Conditions": u_x = u_xxx = 0 read as a symmetry condition): u_{-1}=u_0,
 * u_{-2}=u_1, u_{I}=u_{I-1}, u_{I+1}=u_{I-2}; the same in y. */
static inline int refl(int k, int n)
{
    if (k < 0) k = -1 - k;
    if (k >= n) k = 2 * n - 1 - k;
    return k;
}

static inline double U(const double *u, int nx, int ny, int i, int j)
{
    return u[IDX(refl(i, nx), refl(j, ny))];
}

/* Five-point cell-centred Laplacian L[u] (the linear operator of Sec. "Flux
 * Discretization", item 2: computed from cell-centre values). */
static inline double lap_at(const double *u, int nx, int ny, double ds, int i, int j)
{
    return (U(u, nx, ny, i + 1, j) + U(u, nx, ny, i - 1, j) + U(u, nx, ny, i, j + 1)
            + U(u, nx, ny, i, j - 1) - 4.0 * U(u, nx, ny, i, j)) / (ds * ds);
}

/* ---------------------------------------------------------------------------
 * Flux-difference operator D (eq. FluxDiffOper and the expression for D that
 * follows it):  D_ij = (F_{x,+} - F_{x,-} + F_{y,+} - F_{y,-}) / ds.
 * A face flux is F = f0_face * (L_R - L_L)/ds + f1_face * (u_R - u_L)/ds, where the
 * face values of f0, f1 are the mean of the two adjacent cell-centre values
 * (Sec. "Flux Discretization", item 3), and the flux through the domain boundary
 * is zero (no-flux boundary conditions).
 * part = 0: full model; part = 1: d/dkappa of D for the power-law model (f0 term
 * dropped, f1 replaced by h^3 f'(h)).
 * ------------------------------------------------------------------------- */
static int flux_divergence_part(const or_model *M, int part, int nx, int ny, double ds,
                                const double *u, double *D)
{
    const size_t N = (size_t)nx * ny;
    double *lap = malloc(N * sizeof(double));
    double *f0 = malloc(N * sizeof(double));
    double *f1 = malloc(N * sizeof(double));
    double *fx = malloc((size_t)(nx + 1) * ny * sizeof(double)); /* face k: between cells k-1 and k */
    double *fy = malloc((size_t)nx * (ny + 1) * sizeof(double));
    if (!lap || !f0 || !f1 || !fx || !fy) {
        free(lap); free(f0); free(f1); free(fx); free(fy);
        return OR_ENOMEM;
    }
    /* part 1 evaluates the same operator with f0 = 0 and f1 = h^3 f'(h) (kappa = 1) */
    or_model Mp = *M;
    if (part == 1) Mp.kappa = 1.0;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double a0, a0p, a1, a1p;
            or_coeffs(&Mp, u[IDX(i, j)], &a0, &a0p, &a1, &a1p);
            f0[IDX(i, j)] = part == 1 ? 0.0 : a0;
            f1[IDX(i, j)] = a1;
            lap[IDX(i, j)] = lap_at(u, nx, ny, ds, i, j);
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int k = 0; k <= nx; ++k) {
            double F = 0.0;
            if (k > 0 && k < nx) {
                const size_t L = IDX(k - 1, j), R = IDX(k, j);
                const double A = 0.5 * (f0[L] + f0[R]);
                const double B = 0.5 * (f1[L] + f1[R]);
                F = A * (lap[R] - lap[L]) / ds + B * (u[R] - u[L]) / ds;
            }
            fx[(size_t)j * (nx + 1) + k] = F;
        }
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= ny; ++k)
        for (int i = 0; i < nx; ++i) {
            double F = 0.0;
            if (k > 0 && k < ny) {
                const size_t L = IDX(i, k - 1), R = IDX(i, k);
                const double A = 0.5 * (f0[L] + f0[R]);
                const double B = 0.5 * (f1[L] + f1[R]);
                F = A * (lap[R] - lap[L]) / ds + B * (u[R] - u[L]) / ds;
            }
            fy[(size_t)k * nx + i] = F;
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            D[IDX(i, j)] = (fx[(size_t)j * (nx + 1) + i + 1] - fx[(size_t)j * (nx + 1) + i]
                            + fy[(size_t)(j + 1) * nx + i] - fy[(size_t)j * nx + i]) / ds;
    free(lap); free(f0); free(f1); free(fx); free(fy);
    return OR_OK;
}

int or_flux_divergence(const or_model *M, int nx, int ny, double ds, const double *u, double *D)
{
    if (!M || nx < 2 || ny < 2 || ds <= 0.0 || !u || !D) return OR_EINVAL;
    return flux_divergence_part(M, 0, nx, ny, ds, u, D);
}

int or_flux_divergence_dkappa(const or_model *M, int nx, int ny, double ds, const double *u, double *D)
{
    if (!M || M->kind != OR_POWERLAW || nx < 2 || ny < 2 || ds <= 0.0 || !u || !D) return OR_EINVAL;
    return flux_divergence_part(M, 1, nx, ny, ds, u, D);
}

/* Residual G(u) = u - u^n + dt [theta D(u) + (1-theta) D(u^n)]  (eq. TrapRule with a
 * general theta; theta = 1/2 reproduces the paper's trapezoidal rule exactly). */
int or_residual(const or_model *M, int nx, int ny, double ds, double dt, double theta,
                const double *un, const double *u, double *G)
{
    const size_t N = (size_t)nx * ny;
    double *Du = malloc(N * sizeof(double)), *Dn = malloc(N * sizeof(double));
    if (!Du || !Dn) { free(Du); free(Dn); return OR_ENOMEM; }
    int st = or_flux_divergence(M, nx, ny, ds, u, Du);
    if (st == OR_OK) st = or_flux_divergence(M, nx, ny, ds, un, Dn);
    if (st == OR_OK)
        for (size_t p = 0; p < N; ++p)
            G[p] = u[p] - un[p] + dt * (theta * Du[p] + (1.0 - theta) * Dn[p]);
    free(Du); free(Dn);
    return st;
}

/* ---------------------------------------------------------------------------
 * Band matrices of I + c J_x (one grid row) and I + c J_y (one grid column).
 * J_x is the Jacobian of (F_{x,+} - F_{x,-})/ds restricted to its pure x-derivative
 * terms (Sec. "Flux Discretization"; eqs. DirectionSplit, JacobianSystem1-2).
 * Reading used: linearising a face flux F = A (L_R - L_L)/ds + B (u_R - u_L)/ds gives
 *   dF = A T[d] + (f0'_L d_L + f0'_R d_R) Lam/2 + B (d_R - d_L)/ds + (f1'_L d_L + f1'_R d_R) Gam/2
 * with Lam = (L_R - L_L)/ds (full Laplacian), Gam = (u_R - u_L)/ds and
 * T[d] = (d_{R+1} - 3 d_R + 3 d_L - d_{L-1})/ds^3, the x-part of the Laplacian
 * difference; the cross-direction part A (Lyy_R - Lyy_L)[d]/ds belongs to J_xy and is
 * left in the residual. The perturbation d is even-reflected at the boundary like u,
 * and the boundary-face fluxes stay zero (Sec. "Boundary Conditions").
 * band[o*len + p], o = 0..4 is the entry (p, p + o - 2).
 * ------------------------------------------------------------------------- */
static void face_weights(const or_model *M, double ds, double uL, double uR, double lapL, double lapR,
                         int L, int len, int *cell, double *w)
{
    double f0L, f0pL, f1L, f1pL, f0R, f0pR, f1R, f1pR;
    or_coeffs(M, uL, &f0L, &f0pL, &f1L, &f1pL);
    or_coeffs(M, uR, &f0R, &f0pR, &f1R, &f1pR);
    const double A = 0.5 * (f0L + f0R), B = 0.5 * (f1L + f1R);
    const double Lam = (lapR - lapL) / ds, Gam = (uR - uL) / ds;
    const double ds3 = ds * ds * ds;
    const int R = L + 1;
    /* cells L-1, L, R, R+1, folded by reflection d_{-1} = d_0, d_len = d_{len-1} */
    cell[0] = refl(L - 1, len); cell[1] = L; cell[2] = R; cell[3] = refl(R + 1, len);
    w[0] = -A / ds3;
    w[1] = 3.0 * A / ds3 + 0.5 * f0pL * Lam + 0.5 * f1pL * Gam - B / ds;
    w[2] = -3.0 * A / ds3 + 0.5 * f0pR * Lam + 0.5 * f1pR * Gam + B / ds;
    w[3] = A / ds3;
}

static void bands_line(const or_model *M, int nx, int ny, double ds, const double *u, double c,
                       int dir /*0: row j along x, 1: column i along y*/, int line, double *band)
{
    const int len = dir == 0 ? nx : ny;
    memset(band, 0, 5 * (size_t)len * sizeof(double));
    for (int p = 0; p < len; ++p) band[2 * len + p] = 1.0;
    for (int L = 0; L + 1 < len; ++L) {
        const int R = L + 1;
        double uL, uR, lapL, lapR;
        if (dir == 0) {
            uL = u[IDX(L, line)]; uR = u[IDX(R, line)];
            lapL = lap_at(u, nx, ny, ds, L, line); lapR = lap_at(u, nx, ny, ds, R, line);
        } else {
            uL = u[IDX(line, L)]; uR = u[IDX(line, R)];
            lapL = lap_at(u, nx, ny, ds, line, L); lapR = lap_at(u, nx, ny, ds, line, R);
        }
        int cell[4]; double w[4];
        face_weights(M, ds, uL, uR, lapL, lapR, L, len, cell, w);
        /* row L gains +dF/ds (face L+1/2 is its "+" face), row R gains -dF/ds */
        for (int q = 0; q < 4; ++q) {
            band[(size_t)(cell[q] - L + 2) * len + L] += c * w[q] / ds;
            band[(size_t)(cell[q] - R + 2) * len + R] -= c * w[q] / ds;
        }
    }
}

void or_bands_x(const or_model *M, int nx, int ny, double ds, const double *u, double c, int j, double *band)
{
    bands_line(M, nx, ny, ds, u, c, 0, j, band);
}

void or_bands_y(const or_model *M, int nx, int ny, double ds, const double *u, double c, int i, double *band)
{
    bands_line(M, nx, ny, ds, u, c, 1, i, band);
}

/* ---------------------------------------------------------------------------
 * Band Gaussian elimination with partial pivoting (textbook algorithm for a
 * matrix with lower bandwidth 2 and upper bandwidth 2; after row interchanges the
 * upper factor has bandwidth 4). The paper solves each line with an LU
 * factorisation (Appendix A.3.1); pivoting is added here so the reference does not
 * rely on diagonal dominance.
 * band: 5 x n as above (not modified). rhs: n (not modified). x: n.
 * Work storage: row r holds columns r-2 .. r+4 at w[r*7 + (col - r + 2)].
 * ------------------------------------------------------------------------- */
static double *wget(double *w, int r, int col) { return &w[(size_t)r * 7 + (size_t)(col - r + 2)]; }

int or_band_solve(int n, const double *band, const double *rhs, double *x)
{
    if (n < 1) return OR_EINVAL;
    double *w = calloc((size_t)n * 7, sizeof(double));
    double *b = malloc((size_t)n * sizeof(double));
    if (!w || !b) { free(w); free(b); return OR_ENOMEM; }
    for (int r = 0; r < n; ++r) {
        for (int o = 0; o < 5; ++o) {
            const int col = r + o - 2;
            if (col >= 0 && col < n) *wget(w, r, col) = band[(size_t)o * n + r];
        }
        b[r] = rhs[r];
    }
    int status = OR_OK;
    for (int k = 0; k < n; ++k) {
        const int last = k + 2 < n - 1 ? k + 2 : n - 1;
        int piv = k;
        double best = fabs(*wget(w, k, k));
        for (int r = k + 1; r <= last; ++r)
            if (fabs(*wget(w, r, k)) > best) { best = fabs(*wget(w, r, k)); piv = r; }
        if (best == 0.0) { status = OR_ESINGULAR; break; }
        const int cmax = k + 4 < n - 1 ? k + 4 : n - 1;
        if (piv != k) {
            for (int col = k; col <= cmax; ++col) {
                double t = *wget(w, k, col);
                /* row piv stores columns piv-2..piv+4, which covers k..k+4 */
                *wget(w, k, col) = *wget(w, piv, col);
                *wget(w, piv, col) = t;
            }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        const double pivot = *wget(w, k, k);
        for (int r = k + 1; r <= last; ++r) {
            const double l = *wget(w, r, k) / pivot;
            if (l == 0.0) continue;
            for (int col = k; col <= cmax; ++col) *wget(w, r, col) -= l * *wget(w, k, col);
            b[r] -= l * b[k];
        }
    }
    if (status == OR_OK)
        for (int k = n - 1; k >= 0; --k) {
            const int cmax = k + 4 < n - 1 ? k + 4 : n - 1;
            double s = b[k];
            for (int col = k + 1; col <= cmax; ++col) s -= *wget(w, k, col) * x[col];
            x[k] = s / *wget(w, k, k);
        }
    free(w); free(b);
    return status;
}

/* Transpose of a 5-band matrix: entry (p, p+o-2) moves to (p+o-2, p). */
void or_band_transpose(int n, const double *band, double *bt)
{
    memset(bt, 0, 5 * (size_t)n * sizeof(double));
    for (int p = 0; p < n; ++p)
        for (int o = 0; o < 5; ++o) {
            const int col = p + o - 2;
            if (col < 0 || col >= n) continue;
            /* in the transpose, row col has the entry at column p: offset p - col */
            bt[(size_t)(p - col + 2) * n + col] = band[(size_t)o * n + p];
        }
}

/* ---------------------------------------------------------------------------
 * One ADI-Newton iteration (eqs. JacobianSystem1-3): with c = theta dt,
 *   (I + c J_y(u_k)) w = -G(u_k)      one banded solve per grid column
 *   (I + c J_x(u_k)) v = w            one banded solve per grid row
 *   u_{k+1} = u_k + v,  e = max |v / u_k|  (eq. NewtonError),  r = max |G(u_k)|.
 * Dn = D(u^n) (needed only when theta < 1; may be NULL when theta == 1).
 * ------------------------------------------------------------------------- */
int or_adi_iteration(const or_model *M, int nx, int ny, double ds, double dt, double theta,
                     const double *un, const double *Dn, const double *uk, double *ukp1,
                     double *e_out, double *r_out)
{
    const size_t N = (size_t)nx * ny;
    const double c = theta * dt;
    double *rhs = malloc(N * sizeof(double)), *w = malloc(N * sizeof(double));
    if (!rhs || !w) { free(rhs); free(w); return OR_ENOMEM; }
    int st = or_flux_divergence(M, nx, ny, ds, uk, rhs); /* rhs <- D(u_k) */
    if (st != OR_OK) { free(rhs); free(w); return st; }
    double rmax = 0.0;
    int rnan = 0;
    for (size_t p = 0; p < N; ++p) {
        const double Dn_p = (theta < 1.0 && Dn) ? Dn[p] : 0.0;
        const double G = uk[p] - un[p] + dt * (theta * rhs[p] + (1.0 - theta) * Dn_p);
        if (isnan(G)) rnan = 1;
        else if (fabs(G) > rmax) rmax = fabs(G);
        rhs[p] = -G;
    }
    if (rnan) rmax = NAN;
    int bad = 0;
#pragma omp parallel
    {
        double *band = malloc(5 * (size_t)(nx > ny ? nx : ny) * sizeof(double));
        double *line = malloc((size_t)(nx > ny ? nx : ny) * sizeof(double));
        double *sol = malloc((size_t)(nx > ny ? nx : ny) * sizeof(double));
        if (!band || !line || !sol) {
#pragma omp atomic write
            bad = OR_ENOMEM;
        }
#pragma omp for schedule(static)
        for (int i = 0; i < nx; ++i) {
            if (!band || !line || !sol) continue;
            or_bands_y(M, nx, ny, ds, uk, c, i, band);
            for (int j = 0; j < ny; ++j) line[j] = rhs[IDX(i, j)];
            if (or_band_solve(ny, band, line, sol) != OR_OK) {
#pragma omp atomic write
                bad = OR_ESINGULAR;
                continue;
            }
            for (int j = 0; j < ny; ++j) w[IDX(i, j)] = sol[j];
        }
#pragma omp for schedule(static)
        for (int j = 0; j < ny; ++j) {
            if (!band || !line || !sol) continue;
            or_bands_x(M, nx, ny, ds, uk, c, j, band);
            for (int i = 0; i < nx; ++i) line[i] = w[IDX(i, j)];
            if (or_band_solve(nx, band, line, sol) != OR_OK) {
#pragma omp atomic write
                bad = OR_ESINGULAR;
                continue;
            }
            for (int i = 0; i < nx; ++i) rhs[IDX(i, j)] = sol[i]; /* rhs <- v */
        }
        free(band); free(line); free(sol);
    }
    if (bad) { free(rhs); free(w); return bad; }
    double e = 0.0;
    int enan = 0;
    for (size_t p = 0; p < N; ++p) {
        const double v = rhs[p];
        ukp1[p] = uk[p] + v;
        const double q = fabs(v / uk[p]);
        if (isnan(q)) enan = 1;
        else if (q > e) e = q;
    }
    *e_out = enan ? NAN : e;
    if (r_out) *r_out = rmax;
    free(rhs); free(w);
    return OR_OK;
}

static int state_ok(const double *u, size_t N)
{
    for (size_t p = 0; p < N; ++p)
        if (!(u[p] > 0.0)) return 0; /* catches h <= 0 and NaN */
    return 1;
}

/* ---------------------------------------------------------------------------
 * One accepted time step with the control of Fig. FlowChartTime:
 *   start from u_(0) = u^n; iterate until max|v/u_k| < tol (eq. NewtonError);
 *   an iterate with h <= 0 or NaN fails the solution criteria at once (f is
 *   singular at h = 0); after max_newton iterations without acceptance the
 *   attempt is rejected, dt <- dt * dt_shrink, and the step fails with ENOCONV
 *   if dt < dt_min (or at once when adaptive == 0);
 *   after grow_after consecutive accepted steps dt <- min(dt * dt_grow, dt_max).
 * u: in/out (left at u^n on failure). *dt_inout: dt to try / dt for the next step.
 * *successes_inout: consecutive accepted steps carried between calls.
 * ------------------------------------------------------------------------- */
int or_step(const or_model *M, const or_scheme *S, int nx, int ny, double ds, double *u,
            double *dt_inout, int *successes_inout, or_step_info *info)
{
    if (!M || !S || !u || !dt_inout || nx < 2 || ny < 2 || ds <= 0.0) return OR_EINVAL;
    const size_t N = (size_t)nx * ny;
    if (!state_ok(u, N)) return OR_ENONPOS;
    double *un = malloc(N * sizeof(double)), *a = malloc(N * sizeof(double));
    double *bb = malloc(N * sizeof(double)), *Dn = NULL;
    if (!un || !a || !bb) { free(un); free(a); free(bb); return OR_ENOMEM; }
    memcpy(un, u, N * sizeof(double));
    if (S->theta < 1.0) {
        Dn = malloc(N * sizeof(double));
        if (!Dn || or_flux_divergence(M, nx, ny, ds, un, Dn) != OR_OK) {
            free(un); free(a); free(bb); free(Dn); return OR_ENOMEM;
        }
    }
    double dt = *dt_inout;
    int rejections = 0, total = 0, status = OR_ENOCONV;
    double e = 0.0, r = 0.0;
    int iters = 0;
    for (;;) {
        const double *cur = un;
        double *nxt = a;
        int accepted = 0;
        for (iters = 1; iters <= S->max_newton; ++iters) {
            int st = or_adi_iteration(M, nx, ny, ds, dt, S->theta, un, Dn, cur, nxt, &e, &r);
            ++total;
            if (st != OR_OK) break;
            if (!state_ok(nxt, N)) break;
            if (e < S->tol) { accepted = 1; cur = nxt; break; }
            cur = nxt;
            nxt = (nxt == a) ? bb : a;
        }
        if (accepted) {
            memcpy(u, cur, N * sizeof(double));
            status = OR_OK;
            break;
        }
        ++rejections;
        *successes_inout = 0;
        if (!S->adaptive) { status = OR_ENOCONV; break; }
        dt *= S->dt_shrink;
        if (dt < S->dt_min) { status = OR_ENOCONV; break; }
    }
    if (info) {
        info->dt_used = dt; info->e_final = e; info->r_final = r;
        info->newton_iters = iters; info->rejections = rejections;
        info->status = status; info->total_iters = total;
    }
    if (status == OR_OK) {
        *successes_inout += 1;
        if (S->adaptive && *successes_inout >= S->grow_after) {
            dt = dt * S->dt_grow;
            if (dt > S->dt_max) dt = S->dt_max;
            *successes_inout = 0;
        }
        *dt_inout = dt;
    } else {
        *dt_inout = dt;
    }
    free(un); free(a); free(bb); free(Dn);
    return status;
}

/* ---------------------------------------------------------------------------
 * Full Jacobian J_D of D, applied to a vector (J v) or transposed (J^T mu), from
 * the analytic derivative of each face flux:
 *   dF/du_L = f0'_L Lam/2 + A dLam/du_L + f1'_L Gam/2 - B/ds
 *   dF/du_R = f0'_R Lam/2 + A dLam/du_R + f1'_R Gam/2 + B/ds
 *   dF/du_q = A dLam/du_q for the other cells q of the two Laplacian stencils,
 * where dLap_c/du_q = 1/ds^2 for an in-domain neighbour q of c and
 * dLap_c/du_c = -(number of in-domain neighbours)/ds^2 (reflected ghosts cancel).
 * D_c = sum over faces of +-F/ds, so J = sum_f (e_L - e_R) dF_f/du / ds.
 * Used by the adjoint (not part of the paper) and by the tests.
 * ------------------------------------------------------------------------- */
typedef struct { int n; size_t idx[10]; double w[10]; } sparse_row;

static void sr_add(sparse_row *s, size_t idx, double w)
{
    for (int q = 0; q < s->n; ++q)
        if (s->idx[q] == idx) { s->w[q] += w; return; }
    s->idx[s->n] = idx; s->w[s->n] = w; s->n++;
}

static void add_lap_grad(sparse_row *s, int nx, int ny, double ds, int i, int j, double scale)
{
    const double inv = scale / (ds * ds);
    int cnt = 0;
    if (i + 1 < nx) { sr_add(s, IDX(i + 1, j), inv); ++cnt; }
    if (i - 1 >= 0) { sr_add(s, IDX(i - 1, j), inv); ++cnt; }
    if (j + 1 < ny) { sr_add(s, IDX(i, j + 1), inv); ++cnt; }
    if (j - 1 >= 0) { sr_add(s, IDX(i, j - 1), inv); ++cnt; }
    sr_add(s, IDX(i, j), -cnt * inv);
}

/* gradient of the flux through the interior face between cells (iL,jL) and (iR,jR) */
static void face_flux_grad(const or_model *M, int nx, int ny, double ds, const double *u,
                           int iL, int jL, int iR, int jR, sparse_row *s)
{
    s->n = 0;
    const size_t L = IDX(iL, jL), R = IDX(iR, jR);
    double f0L, f0pL, f1L, f1pL, f0R, f0pR, f1R, f1pR;
    or_coeffs(M, u[L], &f0L, &f0pL, &f1L, &f1pL);
    or_coeffs(M, u[R], &f0R, &f0pR, &f1R, &f1pR);
    const double A = 0.5 * (f0L + f0R), B = 0.5 * (f1L + f1R);
    const double lapL = lap_at(u, nx, ny, ds, iL, jL), lapR = lap_at(u, nx, ny, ds, iR, jR);
    const double Lam = (lapR - lapL) / ds, Gam = (u[R] - u[L]) / ds;
    sr_add(s, L, 0.5 * f0pL * Lam + 0.5 * f1pL * Gam - B / ds);
    sr_add(s, R, 0.5 * f0pR * Lam + 0.5 * f1pR * Gam + B / ds);
    add_lap_grad(s, nx, ny, ds, iR, jR, A / ds);
    add_lap_grad(s, nx, ny, ds, iL, jL, -A / ds);
}

static int jacobian_apply(const or_model *M, int nx, int ny, double ds, const double *u,
                          const double *in, double *out, int transpose)
{
    const size_t N = (size_t)nx * ny;
    memset(out, 0, N * sizeof(double));
    /* serial over faces: the transposed product scatters into shared entries */
    sparse_row s;
    for (int dir = 0; dir < 2; ++dir)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int iR = dir == 0 ? i + 1 : i, jR = dir == 0 ? j : j + 1;
                if (iR >= nx || jR >= ny) continue;
                face_flux_grad(M, nx, ny, ds, u, i, j, iR, jR, &s);
                const size_t L = IDX(i, j), R = IDX(iR, jR);
                if (!transpose) {
                    double dF = 0.0;
                    for (int q = 0; q < s.n; ++q) dF += s.w[q] * in[s.idx[q]];
                    out[L] += dF / ds;
                    out[R] -= dF / ds;
                } else {
                    const double om = (in[L] - in[R]) / ds;
                    for (int q = 0; q < s.n; ++q) out[s.idx[q]] += om * s.w[q];
                }
            }
    return OR_OK;
}

int or_jacobian_apply(const or_model *M, int nx, int ny, double ds, const double *u,
                      const double *v, double *out)
{
    return jacobian_apply(M, nx, ny, ds, u, v, out, 0);
}

int or_jacobian_apply_t(const or_model *M, int nx, int ny, double ds, const double *u,
                        const double *mu, double *out)
{
    return jacobian_apply(M, nx, ny, ds, u, mu, out, 1);
}

/* ---------------------------------------------------------------------------
 * Discrete adjoint of one converged time step (not in the paper; it differentiates
 * the implicit step map G(u^{n+1}; u^n, kappa) = 0 by the implicit-function theorem):
 *   (I + theta dt J_D(u^{n+1}))^T mu = lambda^{n+1}
 *   lambda^n = mu - (1 - theta) dt J_D(u^n)^T mu
 *   dL/dkappa -= dt mu . [theta dD/dkappa(u^{n+1}) + (1 - theta) dD/dkappa(u^n)]
 * The linear system is solved by Richardson iteration preconditioned with the
 * transposed ADI factors, P^{-T} = (I + c J_y)^{-T} (I + c J_x)^{-T}: a transposed row
 * solve, then a transposed column solve, until max|dmu| <= tol * max|mu|.
 * ------------------------------------------------------------------------- */
int or_adjoint_step(const or_model *M, int nx, int ny, double ds, double dt, double theta,
                    const double *u_n, const double *u_np1, const double *lam_np1,
                    double *lam_n, double *dL_dkappa, double tol, int max_iter, int *iters_out)
{
    const size_t N = (size_t)nx * ny;
    const double c = theta * dt;
    double *mu = calloc(N, sizeof(double)), *res = malloc(N * sizeof(double));
    double *tmp = malloc(N * sizeof(double)), *y = malloc(N * sizeof(double));
    if (!mu || !res || !tmp || !y) { free(mu); free(res); free(tmp); free(y); return OR_ENOMEM; }
    int it, status = OR_ENOCONV;
    for (it = 1; it <= max_iter; ++it) {
        /* res = lambda - (I + c J^T) mu */
        jacobian_apply(M, nx, ny, ds, u_np1, mu, tmp, 1);
        for (size_t p = 0; p < N; ++p) res[p] = lam_np1[p] - mu[p] - c * tmp[p];
        int bad = 0;
#pragma omp parallel
        {
            const int lmax = nx > ny ? nx : ny;
            double *band = malloc(5 * (size_t)lmax * sizeof(double));
            double *bt = malloc(5 * (size_t)lmax * sizeof(double));
            double *line = malloc((size_t)lmax * sizeof(double));
            double *sol = malloc((size_t)lmax * sizeof(double));
#pragma omp for schedule(static)
            for (int j = 0; j < ny; ++j) {
                or_bands_x(M, nx, ny, ds, u_np1, c, j, band);
                or_band_transpose(nx, band, bt);
                for (int i = 0; i < nx; ++i) line[i] = res[IDX(i, j)];
                if (or_band_solve(nx, bt, line, sol) != OR_OK) {
#pragma omp atomic write
                    bad = 1;
                    continue;
                }
                for (int i = 0; i < nx; ++i) y[IDX(i, j)] = sol[i];
            }
#pragma omp for schedule(static)
            for (int i = 0; i < nx; ++i) {
                or_bands_y(M, nx, ny, ds, u_np1, c, i, band);
                or_band_transpose(ny, band, bt);
                for (int j = 0; j < ny; ++j) line[j] = y[IDX(i, j)];
                if (or_band_solve(ny, bt, line, sol) != OR_OK) {
#pragma omp atomic write
                    bad = 1;
                    continue;
                }
                for (int j = 0; j < ny; ++j) tmp[IDX(i, j)] = sol[j];
            }
            free(band); free(bt); free(line); free(sol);
        }
        if (bad) { status = OR_ESINGULAR; break; }
        double dmax = 0.0, mmax = 0.0;
        for (size_t p = 0; p < N; ++p) {
            mu[p] += tmp[p];
            if (fabs(tmp[p]) > dmax) dmax = fabs(tmp[p]);
            if (fabs(mu[p]) > mmax) mmax = fabs(mu[p]);
        }
        if (dmax <= tol * mmax) { status = OR_OK; break; }
    }
    if (iters_out) *iters_out = it;
    if (status == OR_OK) {
        jacobian_apply(M, nx, ny, ds, u_n, mu, tmp, 1);
        for (size_t p = 0; p < N; ++p) lam_n[p] = mu[p] - (1.0 - theta) * dt * tmp[p];
        if (dL_dkappa && M->kind == OR_POWERLAW) {
            or_flux_divergence_dkappa(M, nx, ny, ds, u_np1, res);
            if (theta < 1.0) or_flux_divergence_dkappa(M, nx, ny, ds, u_n, y);
            double acc = 0.0;
            for (size_t p = 0; p < N; ++p)
                acc += mu[p] * (theta * res[p] + (theta < 1.0 ? (1.0 - theta) * y[p] : 0.0));
            *dL_dkappa -= dt * acc;
        }
    }
    free(mu); free(res); free(tmp); free(y);
    return status;
}

/* Compensated (Neumaier) sum and minimum, for the mass diagnostic (Sec. "Conservation
 * of Mass": the mean of the cell-centre values). */
void or_mass(int nx, int ny, const double *u, double *sum, double *hmin)
{
    const size_t N = (size_t)nx * ny;
    double s = 0.0, comp = 0.0, mn = INFINITY;
    for (size_t p = 0; p < N; ++p) {
        const double x = u[p], t = s + x;
        comp += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
        s = t;
        if (x < mn) mn = x;
    }
    *sum = s + comp;
    *hmin = mn;
}
