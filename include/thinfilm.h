/*
 * thinfilm.h -- C ABI of libthinfilm, an MI355X (gfx950) FP64 implementation of the
 * ADI-Newton time step for the thin-film equation
 *
 *     h_t + div[ f0(h) grad lap h + f1(h) grad h ] = 0,
 *     f0 = h^3,  f1 = kappa h^3 f'(h),  f(h) = (b/h)^n - (b/h)^m   (power law),
 *
 * or f0 = C h^3, f1 = h^3 Pi'(h) with the disjoining pressure Pi of the nematic liquid
 * crystal or the polymer film model (tf_set_model_nlc, tf_set_model_polymer), or the linear
 * test model f0 = c0, f1 = c1 (tf_set_model_linear),
 * on a cell-centred grid with no-flux boundaries (u_n = u_nnn = 0), following
 * M.-A. Y.-H. Lam, L. J. Cummings, L. Kondic, "Computing dynamics of thin films via
 * large scale GPU-based simulations", arXiv:1806.10550:
 *   - flux-form discretisation: Sec. "Conservation Law" (eq. GovEqnCell2) and
 *     Sec. "Flux Discretization" (face values of f0, f1 are means of the two cells);
 *   - boundary conditions: Sec. "Boundary Conditions" (even-reflection ghost cells);
 *   - time stepping: the theta scheme G(u) = u - u^n + dt[theta D(u) + (1-theta) D(u^n)]
 *     (theta = 1/2 is eq. TrapRule; theta = 1 is backward Euler);
 *   - Newton iteration with the ADI factorisation (I + c J_y)(I + c J_x), c = theta dt,
 *     y solve first, mixed terms left in the residual: eqs. DirectionSplit and
 *     JacobianSystem1-3;
 *   - acceptance test max|v/u_k| < tol (eq. NewtonError) and the adaptive time-step
 *     control of Fig. FlowChartTime.
 *
 * Memory: every array argument marked "device" is a pointer into HIP device memory
 * on the device that was current when the grid was created; "host" pointers are
 * ordinary host memory. Grids are row-major: h[j*nx + i], i along x, j along y,
 * contiguous, FP64. The caller owns all arrays it passes; the library owns its
 * scratch buffers and frees them in tf_destroy. All work is enqueued on the stream
 * given to tf_create; calls that make a host-side decision synchronise that stream.
 *
 * Errors: every call returns a tf_status; TF_OK is 0. On any error the bound state
 * is left at the last accepted time level. tf_last_error() describes the most recent
 * failure of the calling thread. No C++ exception crosses this interface.
 * A grid must not be used from two threads at once.
 */
#ifndef THINFILM_H
#define THINFILM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef int tf_status;
enum {
    TF_OK = 0,
    TF_EINVAL = 1,   /* bad argument */
    TF_ENOMEM = 2,   /* device or pinned-host allocation failed */
    TF_EDEVICE = 3,  /* a HIP call failed; see tf_last_error() */
    TF_ENOCONV = 4,  /* Newton did not converge and dt fell below dt_min (or adaptive == 0) */
    TF_ENONPOS = 5,  /* the state holds h <= 0 or NaN */
    TF_ESTATE = 6    /* no state bound, or model not set */
};

typedef struct tf_grid tf_grid;

/* Time-stepping scheme and the control of Fig. FlowChartTime.
 *   theta      1 = backward Euler, 0.5 = trapezoidal rule (eq. TrapRule); 0.5 <= theta <= 1
 *   tol        accept when max|v/u_k| < tol (eq. NewtonError)
 *   max_newton iterations per attempt (the paper's K)
 *   adaptive   0: a non-converged attempt fails the step with TF_ENOCONV;
 *              1: it is retried with dt *= dt_shrink until dt < dt_min (TF_ENOCONV);
 *                 after grow_after consecutive accepted steps dt = min(dt*dt_grow, dt_max). */
typedef struct {
    double theta, tol, dt_min, dt_max, dt_shrink, dt_grow;
    int max_newton, grow_after, adaptive;
} tf_scheme;

/* Per accepted step: time after the step, the dt it used, the final update ratio
 * max|v/u_k| and residual max|G|, Newton iterations of the accepted attempt, the
 * number of rejected attempts, the status, and (only when mass diagnostics are on,
 * see tf_set_diagnostics) the compensated sum of h and its minimum. */
typedef struct {
    double t, dt_used, e_final, r_final, mass, hmin;
    int newton_iters, rejections, status, total_iters;
} tf_step_info;

/* Create a grid of nx x ny cells of side ds (nx, ny >= 4, ds > 0) whose work is
 * enqueued on `stream` (a hipStream_t; NULL = the default stream). Allocates the
 * device scratch (about 5 fields of nx*ny doubles). Default scheme: theta = 1,
 * tol = 1e-10, max_newton = 5000, adaptive = 0, dt_min = 1e-6, dt_max = 1,
 * dt_shrink = 0.5, dt_grow = 1.1, grow_after = 5. */
tf_status tf_create(int nx, int ny, double ds, void *stream, tf_grid **out);
tf_status tf_destroy(tf_grid *g);

/* Power-law model: f = (b/h)^n - (b/h)^m, f1 = kappa h^3 f'(h) (eq. GeneralDisPreForm
 * with the power-law term of eq. DisjPressNLC). b > 0; n and m integral with
 * 16 >= n > m >= 1 (TF_EINVAL otherwise). kappa may have any sign. */
tf_status tf_set_model(tf_grid *g, double kappa, double b, double n, double m);
/* Linear test model (Sec. "Thin Film Models"): f0 = c0, f1 = c1, constants, so that the
 * step is linear in h (the paper's validation runs use c0 = 1, c1 = 1: q_m = 1/sqrt(2),
 * omega_m = 1/4). Needs finite c0 > 0 and c1 (TF_EINVAL otherwise). The positivity
 * check on h (TF_ENONPOS) still applies. */
tf_status tf_set_model_linear(tf_grid *g, double c0, double c1);
/* Nematic liquid crystal model (Sec. "Thin Film Models", eqs. GeneralDisPreForm,
 * DisjPressNLC, mh_model): f0 = C h^3, f1 = h^3 Pi'(h) (without the division by C that
 * eq. GeneralDisPreForm prints: this is the reading under which the growth rates printed
 * with Fig. dispersion_curves follow),
 *     Pi = K[(b/h)^3 - (b/h)^2] + (N/2) (m(h)/h)^2,  m = g(h) h^2 / (h^2 + beta^2),
 *     g = (1 + tanh((h - 2b)/w)) / 2.
 * The paper's parameters (eq. NLC_paras): C = 0.0857, K = 36, N = 1.67, beta = 1,
 * w = 0.05, b = 0.01. Needs finite values with C, w, b > 0 and K, N >= 0 (TF_EINVAL
 * otherwise). Replaces any model set before; invalidates the bound state's check. */
tf_status tf_set_model_nlc(tf_grid *g, double C, double K, double N, double beta, double w, double b);
/* Polymer film model (Sec. "Thin Film Models", eqs. GeneralDisPreForm, DisjPressPolymer):
 * f0 = C h^3, f1 = h^3 Pi'(h) (same reading as above), Pi = -psi'(h),
 *     psi = Cst h^-8 - Aox / (12 pi h^2) + (Aox - Asi) / (12 pi (h + d)^2).
 * The paper's parameters (eq. Polymer_scales): C = 0.00581, Cst = 1.181, Aox = 41.25,
 * Asi = -243.75, d = 191. Needs finite values with C > 0, d >= 0 (TF_EINVAL otherwise). */
tf_status tf_set_model_polymer(tf_grid *g, double C, double Cst, double Aox, double Asi, double d);
/* The grid's model coefficients at n thicknesses: out[4k + 0..3] = f0, f0', f1, f1' at h[k]
 * (eq. GeneralDisPreForm; these give the linear growth rate sigma(q) = q^2 (f1 - f0 q^2) of
 * a flat film, Sec. "Linear Stability Analysis"). h: device, n doubles (> 0); out: device,
 * 4n doubles. Evaluated by the same device code as the sweeps. TF_ESTATE without a model. */
tf_status tf_model_coeffs(tf_grid *g, const double *h, int n, double *out);
tf_status tf_set_scheme(tf_grid *g, const tf_scheme *s);
tf_status tf_get_scheme(const tf_grid *g, tf_scheme *s);
/* 1: fill tf_step_info.mass / hmin after every accepted step (Sec. "Conservation of
 * Mass"): the x sweep forms a compensated partial sum and minimum of each iterate as it
 * stores it, and the accepted iterate's records are combined in a fixed order (no extra
 * read of h). */
tf_status tf_set_diagnostics(tf_grid *g, int mass_every_step);

/* Line-solver variant of the x sweep (eqs. JacobianSystem2-3: one pentadiagonal system
 * per grid row, then u_{k+1} = u_k + v and the update ratio of eq. NewtonError). Both give
 * the same Newton root; they differ in rounding, so iterates agree to ~1e-13 relative.
 *   TF_XSWEEP_PARTITIONED  three kernels per sweep: segment relations of 64-cell tiles,
 *                          the interface chain of each row, then the segment solves
 *                          (any nx);
 *   TF_XSWEEP_ROW          one kernel: a workgroup holds whole rows, eliminates 16-cell
 *                          sub-segments per lane and couples them by a tree of merges in
 *                          LDS (4 <= nx <= 8192);
 *   TF_XSWEEP_AUTO         the row kernel when nx allows it (the default at tf_create).
 * TF_EINVAL for an unknown variant or TF_XSWEEP_ROW with nx > 8192. tf_get_xsweep returns
 * the variant in use (-1 for a NULL grid). The transposed row solves of tf_adjoint_step
 * follow the setting: TF_XSWEEP_ROW (with nx <= 4096) solves whole rows in one kernel,
 * otherwise the tuned stored-band solver (tf_autotune) other than that kernel is used. */
#define TF_XSWEEP_AUTO (-1)
#define TF_XSWEEP_PARTITIONED 0
#define TF_XSWEEP_ROW 1
tf_status tf_set_xsweep(tf_grid *g, int variant);
int tf_get_xsweep(const tf_grid *g);

/* Borrow the caller's state h (device, nx*ny FP64). The library reads and writes it
 * in place; during a call it may also hold iterates there. It must stay allocated
 * until unbound (tf_bind_state(g, NULL)) or tf_destroy. Resets the time to 0. */
tf_status tf_bind_state(tf_grid *g, double *h_dev);
/* The clock of the bound state (host scalars): time t and the number of consecutive accepted
 * steps that count towards the next dt growth of the adaptive control (Fig. FlowChartTime).
 * With the state itself and the dt proposed for the next step, it is all a later run needs to
 * continue exactly where this one stopped (checkpoint / resume): bind the saved state, set
 * the clock, step with the saved dt. tf_set_clock: TF_EINVAL for non-finite t or
 * successes < 0; call it after tf_bind_state, which resets the clock. */
tf_status tf_get_clock(const tf_grid *g, double *t, int *successes);
tf_status tf_set_clock(tf_grid *g, double t, int successes);

/* Advance the bound state by exactly one accepted step. *dt_inout: dt to try in,
 * dt for the next step out. info may be NULL. TF_ENONPOS if the state holds h <= 0
 * or NaN; TF_ENOCONV as in tf_scheme. */
tf_status tf_step(tf_grid *g, double *dt_inout, tf_step_info *info);
/* nsteps accepted steps; log (host, nsteps entries) may be NULL. Stops at the first
 * failure, leaving h at the last accepted state. */
tf_status tf_advance(tf_grid *g, int nsteps, double *dt_inout, tf_step_info *log);
/* tf_advance that also keeps every accepted state: after step s (0-based) the state is
 * copied into states[s] (host array of nsteps device pointers, each to nx*ny doubles on the
 * grid's device, disjoint from the bound state and from each other) on the grid's stream;
 * for the recomputation of a stretch of steps before its adjoint (tf_adjoint_steps). */
tf_status tf_advance_keep(tf_grid *g, int nsteps, double *dt_inout, double *const *states, tf_step_info *log);

/* Compensated sum of h and its minimum (Sec. "Conservation of Mass"); host outputs. */
tf_status tf_mass(tf_grid *g, double *mass, double *hmin);

/* One raw ADI-Newton iteration (eqs. JacobianSystem1-3) on caller buffers (device,
 * nx*ny each): u_kp1 = u_k + v with the grid's model and theta, for time step dt and
 * previous level u_n. Host outputs: e = max|v/u_k|, r = max|G(u_k)|, flags bit 0 =
 * an iterate value <= 0, bit 1 = NaN. u_kp1 must not alias u_k or u_n. */
tf_status tf_newton_iteration(tf_grid *g, const double *u_n, const double *u_k, double *u_kp1, double dt,
                              double *e, double *r, int *flags);
/* out = D(u), the flux-difference operator (eq. FluxDiffOper); device arrays. */
tf_status tf_flux_divergence(tf_grid *g, const double *u, double *out);

/* Per-kernel timing with HIP events recorded on the grid's stream around every
 * launch. tf_profile(g, 1) starts (and clears) recording; tf_profile_read fills
 * total milliseconds and launch counts for each kernel class in the order of
 * tf_profile_names() (comma-separated), up to n classes, and returns the number of
 * classes. */
tf_status tf_profile(tf_grid *g, int on);
int tf_profile_read(tf_grid *g, double *ms, long *count, int n);
const char *tf_profile_names(void);

/* ---- Ensembles ---------------------------------------------------------------------
 * Many independent films (different sizes, kappa and ds; common b, n, m) advanced in
 * lockstep: one Newton iteration of every film that is still iterating is one replay of
 * a captured HIP graph; each film's Newton / dt control (Fig. FlowChartTime) runs on the
 * device, so converged films drop out while the others continue. With theta < 1 each film's
 * b^n = u^n - (1 - theta) dt D(u^n) is formed on the device at the first iteration of every
 * attempt (eq. TrapRule in theta form), as the single-film path does. The films' states live in ONE packed device buffer: film f occupies nx[f]*ny[f]
 * row-major doubles starting at offsets[f] (tf_ensemble_offsets), films back to back in
 * the order given. Work is done on an internal stream ordered after `stream`. */
typedef struct tf_ensemble tf_ensemble;
tf_status tf_ensemble_create(int nfilms, const int *nx, const int *ny, const double *ds, const double *kappa,
                             double b, double n, double m, void *stream, tf_ensemble **out);
/* Give every film of the ensemble the linear, NLC or polymer model instead of the power law
 * of tf_ensemble_create (same parameters and checks as tf_set_model_linear, tf_set_model_nlc
 * and tf_set_model_polymer; the per-film kappa is then unused). Films may still differ in
 * size, ds and initial thickness. Waits for the ensemble's stream; TF_EINVAL for rejected
 * parameters. */
tf_status tf_ensemble_set_model_linear(tf_ensemble *e, double c0, double c1);
tf_status tf_ensemble_set_model_nlc(tf_ensemble *e, double C, double K, double N, double beta, double w, double b);
tf_status tf_ensemble_set_model_polymer(tf_ensemble *e, double C, double Cst, double Aox, double Asi, double d);
tf_status tf_ensemble_destroy(tf_ensemble *e);
/* scheme as for tf_set_scheme (theta in [0.5, 1]; theta < 1 allocates one packed field) */
tf_status tf_ensemble_set_scheme(tf_ensemble *e, const tf_scheme *s);
/* x-sweep line solver of every film (see tf_set_xsweep): TF_XSWEEP_AUTO gives film f the
 * variant tf_xsweep_choice(nx_f, rows of all films) (the default at creation); TF_XSWEEP_ROW the
 * whole-row kernel for every film whose rows fit a 4-wave workgroup (nx <= 4096; the others
 * stay partitioned); TF_XSWEEP_PARTITIONED the partitioned solver for all. The whole-row
 * films of an ensemble share one launch per iteration. tf_ensemble_xsweep returns a film's
 * variant (0 partitioned, 1 whole-row; -1 for a bad film index). */
tf_status tf_ensemble_set_xsweep(tf_ensemble *e, int variant);
int tf_ensemble_xsweep(const tf_ensemble *e, int film);
/* total number of cells (length of the packed buffer) */
long long tf_ensemble_size(const tf_ensemble *e);
/* host array of nfilms offsets (in doubles) of each film in the packed buffer */
tf_status tf_ensemble_offsets(const tf_ensemble *e, long long *offsets);
/* Borrow the packed state (device, tf_ensemble_size doubles); films holding h <= 0 or
 * NaN are marked TF_ENONPOS and never stepped. Resets every film's time and status. */
tf_status tf_ensemble_bind(tf_ensemble *e, double *packed_dev);
/* Advance every film by nsteps accepted steps. dt_per_film (host, nfilms): dt to try in,
 * next dt out. status_per_film (host, nullable): TF_OK, TF_ENOCONV or TF_ENONPOS per film
 * (a failed film keeps its last accepted state and stops). iters_per_film (host,
 * nullable): Newton iterations of each film in this call. Returns TF_OK when every film
 * succeeded, else the first failing film's status. */
tf_status tf_ensemble_step(tf_ensemble *e, int nsteps, double *dt_per_film, int *status_per_film,
                           int *iters_per_film);
/* Record of film `film` after the last tf_ensemble_step (time, last dt, iterations). */
tf_status tf_ensemble_film_info(const tf_ensemble *e, int film, tf_step_info *info);

/* ---- Discrete adjoint ----------------------------------------------------------------
 * Adjoint of one converged step u^{n+1} = S(u^n, kappa), S defined implicitly by
 * G(u^{n+1}; u^n, kappa) = u^{n+1} - u^n + dt[theta D(u^{n+1}) + (1-theta) D(u^n)] = 0
 * (eq. TrapRule in theta form; the grid's model and theta are used). Given
 * lambda^{n+1} = dL/du^{n+1} (device, in lambda_inout) it solves
 *     (I + theta dt J_D(u^{n+1}))^T mu = lambda^{n+1}
 * by Richardson iteration preconditioned with the transposed ADI factors
 * (I + c J_y)^-T (I + c J_x)^-T (eqs. DirectionSplit, JacobianSystem1-2) until
 * max|dmu| <= tol max|mu| (at most max_iter iterations; TF_ENOCONV otherwise, TF_ENONPOS if
 * an iterate turns NaN), then
 * writes lambda^n = mu - (1-theta) dt J_D(u^n)^T mu into lambda_inout and adds
 * -dt mu . [theta dD/dkappa(u^{n+1}) + (1-theta) dD/dkappa(u^n)] to *dL_dkappa_accum
 * (host, nullable; power-law model only, TF_EINVAL for the linear, NLC and polymer models). h_n, h_np1: the two time levels (device, nx*ny each, unchanged).
 * iters_out (host, nullable): Richardson iterations used. */
tf_status tf_adjoint_step(tf_grid *g, const double *h_n, const double *h_np1, double dt, double *lambda_inout,
                          double *dL_dkappa_accum, double tol, int max_iter, int *iters_out);
/* The adjoint steps of one stretch of nsteps fixed-dt steps in one call: states (host array
 * of nsteps + 1 device pointers) holds u at the stretch's time levels, states[0] the oldest;
 * tf_adjoint_step runs for n = nsteps-1 down to 0 with h_n = states[n], h_np1 = states[n+1],
 * taking lambda_inout from lambda^{nsteps} to lambda^0 and adding every step's dL/dkappa
 * contribution to *dL_dkappa_accum. iters_out: Richardson iterations of all steps. Stops at the
 * first failing step and returns its status. */
tf_status tf_adjoint_steps(tf_grid *g, int nsteps, const double *const *states, double dt, double *lambda_inout,
                           double *dL_dkappa_accum, double tol, int max_iter, int *iters_out);
/* out = J_D(u)^T mu with the full analytic Jacobian of the flux-difference operator D
 * (device arrays, nx*ny each). */
tf_status tf_jacobian_apply_t(tf_grid *g, const double *u, const double *mu, double *out);

/* ---- Radial Fourier transform of a film (App. "Radial Fourier Transform") ------------
 * tf_radial_spectrum: steps 1-4 of the appendix on the GPU. h: device, n x n FP64 film
 * (row-major, square grid of side L = n ds; 4 <= n <= 16384), read only. The magnitude of
 * the 2D DFT of h - h0, divided by n^2, is smoothed by a periodic convolution over the
 * integer wavenumbers (kx, ky) with the separable Gaussian weights exp(-d^2/(2 sigma^2))/Z,
 * |d| <= ceil(4 sigma) (sigma in wavenumber units, 0 <= sigma <= 64; 0 = no smoothing),
 * and averaged over each group of equal q_r, i.e. equal m = kx^2 + ky^2 (eq.
 * FFT_radial_averaging), q_r = 2 pi sqrt(m) / L. Output (host arrays of `capacity`
 * entries, in increasing q): q_out[p], s_out[p] (group mean) and count_out[p] (group size;
 * nullable) for every nonempty group with 0 < q_r <= qmax; *npoints (host) receives the
 * number of groups. TF_EINVAL when capacity is too small (npoints then holds the number
 * needed) or qmax spans more than 2^26 groups. Each group's sum is formed in a fixed order, so
 * the output is bit-reproducible. Work is enqueued on `stream` (hipStream_t, NULL = default)
 * and the call returns after it has finished. The FFT plan and device scratch (8 n (n + 2)
 * bytes plus the smoothing window, the group sums and an index of the window by group, about
 * 4 pi M bytes) are kept per (device, n) for later calls until tf_spectrum_release; calls are
 * serialised by a lock. */
tf_status tf_radial_spectrum(const double *h, int n, double ds, double h0, double sigma, double qmax, void *stream,
                             double *q_out, double *s_out, int *count_out, int capacity, int *npoints);
/* Frees the plans and scratch kept by tf_radial_spectrum on every device (waits for each
 * device first). Always TF_OK. */
tf_status tf_spectrum_release(void);
/* tf_spectrum_maxima: steps 5-7 of the appendix (host only; all pointers host). Fits the
 * radial data (q strictly increasing in (0, qmax], npoints >= 1) by least squares with a
 * continuous piecewise-linear function that is 0 at q = 0, with knots at 0, at every 10th
 * data point and at qmax (eq. PiecewiseFunction: 10 points per interval, the last interval
 * takes the remainder); evaluates it at nfine >= 8 equispaced points of [0, qmax] (the paper
 * uses 400) and smooths them by moving averages of half widths 3, 2, 1 (windows truncated at
 * the ends; result in curve_out[nfine], nullable); reports the local maxima (derivative by
 * second-order differences, a +/- sign change located by linear interpolation, negative
 * second difference) in peak_q / peak_s (capacity entries) and their number in *npeaks.
 * TF_EINVAL for unsorted or non-finite data, an interval without data, or too small a
 * capacity (npeaks then holds the number found). */
tf_status tf_spectrum_maxima(const double *q, const double *s, int npoints, double qmax, int nfine, double *curve_out,
                             double *peak_q, double *peak_s, int capacity, int *npeaks);

/* ---- Batched pentadiagonal solves on stored bands -----------------------------------
 * nlines independent systems of n unknowns (n >= 2). Layout position-major: element
 * (position p, line l) at p*nlines + l. bands: 5 device arrays of n*nlines doubles back
 * to back (a, b, c, d, e = offsets -2..+2: row p of line l reads x at p-2..p+2 with
 * coefficients a..e at (p, l); entries reaching outside the line must be zero).
 * transposed != 0 solves with the transposed matrices. variant: 0 = partitioned
 * (64-cell segments, interface chain), 1 = one lane per line (Thomas), 2 = block cyclic
 * reduction in LDS (one workgroup per line, n <= 2048), 3 = whole lines in one kernel
 * (16-cell sub-segments per lane coupled by a tree of merges in LDS, 4 <= n <= 4096),
 * -1 = the autotuned choice. No pivoting: the matrices must be factorable without it.
 * Allocates and frees its own scratch; synchronises `stream`. TF_EINVAL for bad sizes,
 * variant 2 with n > 2048 or variant 3 with n outside 4..4096. */
tf_status tf_penta_solve(int nlines, int n, const double *bands, const double *rhs, double *x, int transposed,
                         int variant, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tf_penta_solve with the same arguments
 * and results, except that it calls no hipMalloc, hipFree or other allocating routine and
 * does not synchronise: the work is enqueued on `stream` and the call returns. Its scratch
 * (interface records of the partitioned variant, the factor array of the Thomas variant;
 * cyclic reduction and the whole-line variant need none) is one static device array of TF_NOALLOC_SCRATCH_DOUBLES
 * doubles (16 MiB) per GPU, held until the process ends. The partitioned variant needs
 * 36 * ceil(n / 64) * nlines doubles of it, Thomas 3 * n * nlines; a solve that needs more
 * returns TF_EINVAL (variant -1 first falls back to cyclic reduction for n <= 2048, else to
 * the partitioned variant). Every call on one GPU shares that GPU's array: calls whose
 * solves overlap in time on one GPU (other streams or threads) race and give wrong
 * results; calls on one stream are ordered and safe. The array needs no clearing (each
 * solve writes the scratch it reads). TF_EDEVICE if the array's device address cannot be
 * obtained. */
#define TF_NOALLOC_SCRATCH_DOUBLES (1 << 21)
tf_status tf_penta_solve_noalloc(int nlines, int n, const double *bands, const double *rhs, double *x,
                                 int transposed, int variant, void *stream);
/* Time the candidates -- partitioned; Thomas with 64, 128 and 256 lines per workgroup;
 * block cyclic reduction (length <= 2048); whole lines in one kernel (4 <= length <= 4096)
 * -- on random diagonally dominant systems of
 * the given length and batch, plain (transposed = 0) or transposed solves (median of 5
 * timed runs after a warm-up), remember the fastest for solves of the same kind and
 * similar shape (used by tf_adjoint_step, whose solves are transposed, and by
 * tf_penta_solve with variant -1), and append a JSON line {arch, length, batch,
 * transposed, variant, block, ms: {...}} to cache_path (nullable). tf_autotune_load
 * reads such a file (entries of the current GPU architecture only; TF_EINVAL if there
 * are none). tf_autotune_choice returns the variant that would be used (0 ..= 3). */
tf_status tf_autotune(int length, int batch, int transposed, const char *cache_path);
tf_status tf_autotune_load(const char *cache_path);
int tf_autotune_choice(int length, int batch, int transposed);
/* Forward x sweep (eqs. JacobianSystem2-3 per grid row; see tf_set_xsweep): time both
 * variants -- partitioned (3 kernels) and whole-row (1 kernel, rows of at most 8192 cells)
 * -- on a film of `batch` rows of `length` cells (1 + 0.01 noise, the n = 3, m = 2 power law
 * with kappa = 10, b = 0.1, ds = 0.67347, dt = 0.2; median of 5 timed runs after a warm-up),
 * remember the faster for films of similar shape and append {arch, kind: "xsweep", length,
 * batch, variant, ms: {...}} to cache_path (nullable; tf_autotune_load reads these lines
 * too). TF_EINVAL for length or batch below 4. Grids (tf_create) and ensembles
 * (tf_ensemble_create, per film, with ny = the rows of all its films, since its x sweep is one
 * launch over all of them) take the variant tf_xsweep_choice(nx, ny) returns at creation: the
 * tuned entry of the nearest shape (log distance below 0.7), else the whole-row kernel when
 * the launch has at most 2048 rows; never the whole-row kernel for rows above 4096 cells.
 * Returns 0 (partitioned) or 1 (whole-row). */
tf_status tf_autotune_xsweep(int length, int batch, const char *cache_path);
int tf_xsweep_choice(int nx, int ny);

/* Description of the calling thread's most recent error (never NULL). */
const char *tf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* THINFILM_H */
