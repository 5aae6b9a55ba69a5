/* Sanitizer driver for the CPU oracle (test infrastructure): compiles the oracle source into
 * the same translation unit and runs its entry points on small grids of every model, so that
 * AddressSanitizer and UndefinedBehaviorSanitizer watch every access. Exit status 0 when all
 * calls return OR_OK; sanitizer reports abort the run. */
#include "../oracle/tf_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static double lcg(unsigned long long *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*s >> 11) / 9007199254740992.0;
}

static int run(const or_model *M, double h0, double ds, double dt, int nx, int ny, double theta)
{
    const size_t N = (size_t)nx * ny;
    double *u = malloc(N * sizeof(double)), *u0 = malloc(N * sizeof(double));
    double *lam = malloc(N * sizeof(double)), *lam_n = malloc(N * sizeof(double));
    double *out = malloc(N * sizeof(double));
    unsigned long long s = 12345;
    for (size_t k = 0; k < N; ++k) {
        u[k] = h0 * (1.0 + 0.02 * (lcg(&s) - 0.5));
        u0[k] = u[k];
        lam[k] = lcg(&s) - 0.5;
    }
    or_scheme S = {theta, 1e-12, 1e-9, 1.0, 0.5, 1.1, 5000, 5, 0};
    or_step_info info;
    int succ = 0, st = OR_OK;
    double d = dt;
    for (int k = 0; k < 3 && st == OR_OK; ++k) st = or_step(M, &S, nx, ny, ds, u, &d, &succ, &info);
    double g = 0.0;
    int it = 0;
    if (st == OR_OK) st = or_adjoint_step(M, nx, ny, ds, dt, theta, u0, u, lam, lam_n, M->kind == OR_POWERLAW ? &g : NULL,
                                          1e-12, 10000, &it);
    if (st == OR_OK) st = or_jacobian_apply_t(M, nx, ny, ds, u, lam, out);
    if (st == OR_OK) st = or_flux_divergence(M, nx, ny, ds, u, out);
    double sum, hmin;
    or_mass(nx, ny, u, &sum, &hmin);
    free(u); free(u0); free(lam); free(lam_n); free(out);
    return st;
}

int main(void)
{
    or_model pl = {0};
    pl.kind = OR_POWERLAW; pl.kappa = 10.0; pl.b = 0.1; pl.n = 3.0; pl.m = 2.0;
    or_model p52 = pl;
    p52.n = 5.0;
    or_model lin = {0};
    lin.kind = OR_LINEAR; lin.c0 = 1.0; lin.c1 = 1.0;
    or_model nlc = {0};
    nlc.kind = OR_NLC; nlc.cap = 0.0857; nlc.K = 36.0; nlc.N = 1.67; nlc.beta = 1.0; nlc.w = 0.05; nlc.b = 0.01;
    or_model pol = {0};
    pol.kind = OR_POLYMER; pol.cap = 0.00581; pol.Cst = 1.181; pol.Aox = 41.25; pol.Asi = -243.75; pol.d = 191.0;
    struct { const or_model *M; double h0, ds, dt; } cases[] = {
        {&pl, 1.0, 0.67, 0.1}, {&p52, 1.0, 0.67, 0.1}, {&lin, 1.0, 0.55, 0.1}, {&nlc, 0.5, 0.26, 0.5}, {&pol, 3.9, 0.25, 0.01}};
    const int shapes[][2] = {{2, 2}, {5, 3}, {9, 7}, {16, 11}};
    for (int c = 0; c < 5; ++c)
        for (int s = 0; s < 4; ++s)
            for (int t = 0; t < 2; ++t) {
                const int st = run(cases[c].M, cases[c].h0, cases[c].ds, cases[c].dt, shapes[s][0], shapes[s][1],
                                   t ? 0.5 : 1.0);
                if (st != OR_OK) {
                    fprintf(stderr, "case %d shape %dx%d theta %s: status %d\n", c, shapes[s][0], shapes[s][1],
                            t ? "1/2" : "1", st);
                    return 1;
                }
            }
    double band[5 * 6] = {0}, rhs[6], x[6];
    for (int p = 0; p < 6; ++p) {
        band[5 * p + 2] = 4.0;
        band[5 * p + 1] = band[5 * p + 3] = -1.0;
        band[5 * p + 0] = band[5 * p + 4] = 0.5;
        rhs[p] = p;
    }
    if (or_band_solve(6, band, rhs, x) != OR_OK) return 1;
    printf("oracle sanitizer run: ok\n");
    return 0;
}
