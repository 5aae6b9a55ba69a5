// Host runtime and C ABI of libthinfilm (see include/thinfilm.h).
//
// The Newton / time-step control of Fig. FlowChartTime (Lam, Cummings & Kondic,
// arXiv:1806.10550) runs on the host: after every iteration the kernels leave a
// 64-byte reduction record {max|v/u_k|, max|G|, flags} on the device, which is copied
// to pinned memory and read after one stream synchronisation (the paper's per-block
// flag array reduced to a single record).
//
// Buffer rotation: the accepted state u^n stays untouched while iterates alternate
// between the two buffers that do not hold u^n (the caller's h is one of the three),
// so u_(0) = u^n needs no copy and a rejected attempt restarts from u^n at no cost.
// The accepted state is copied back into h when a call returns.
#include "tf_internal.h"
#include "../../include/thinfilm.h"

#include <cmath>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err = "no error";

tf_status fail(tf_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define TF_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(TF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

enum ProfKind { P_REL_Y, P_CHAIN_Y, P_SOLVE_Y, P_REL_X, P_CHAIN_X, P_SOLVE_X, P_RHS, P_MASS, P_XROW, P_NKIND };
const char *kProfNames = "relations_y,chain_y,solve_y,relations_x,chain_x,solve_x,rhs_theta,mass,xrow";

constexpr int RES_SLOTS = 4;
constexpr int RES_STRIDE = tf::RES_SPREAD * tf::RES_WORDS; // words per reduction slot

} // namespace

namespace tf_detail {
void set_error(const std::string &msg) { g_err = msg; }

// Model records of the linear, NLC and polymer models (see tf::Model); false with a message
// for parameters the models do not admit (M is then left unchanged).
bool linear_model(double c0, double c1, tf::Model *M, std::string *err)
{
    if (!(c0 > 0.0) || !std::isfinite(c0) || !std::isfinite(c1)) {
        *err = "need finite c0 > 0 and c1";
        return false;
    }
    tf::Model m{};
    m.kind = tf::MODEL_LINEAR;
    m.cap = c0;
    m.Cm = c1;
    *M = m;
    return true;
}

bool nlc_model(double C, double K, double N, double beta, double w, double b, tf::Model *M, std::string *err)
{
    const double v[6] = {C, K, N, beta, w, b};
    for (double x : v)
        if (!std::isfinite(x)) {
            *err = "NLC parameters must be finite";
            return false;
        }
    if (!(C > 0.0) || !(w > 0.0) || !(b > 0.0) || !(K >= 0.0) || !(N >= 0.0)) {
        *err = "need C > 0, w > 0, b > 0, K >= 0 and N >= 0";
        return false;
    }
    tf::Model m{};
    m.kind = tf::MODEL_NLC;
    m.cap = C;
    m.K = K;
    m.N = N;
    m.beta2 = beta * beta;
    m.w = w;
    m.iw = 1.0 / w;
    m.b = b;
    *M = m;
    return true;
}

bool polymer_model(double C, double Cst, double Aox, double Asi, double d, tf::Model *M, std::string *err)
{
    const double v[5] = {C, Cst, Aox, Asi, d};
    for (double x : v)
        if (!std::isfinite(x)) {
            *err = "polymer parameters must be finite";
            return false;
        }
    if (!(C > 0.0) || !(d >= 0.0)) {
        *err = "need C > 0 and d >= 0";
        return false;
    }
    tf::Model m{};
    m.kind = tf::MODEL_POLYMER;
    m.cap = C;
    // Pi = -psi' = 8 Cst h^-9 - (Aox/(6 pi)) h^-3 + ((Aox - Asi)/(6 pi)) (h+d)^-3
    m.C8 = 8.0 * Cst;
    m.a2 = Aox / (6.0 * M_PI);
    m.c2 = (Aox - Asi) / (6.0 * M_PI);
    m.d = d;
    *M = m;
    return true;
}
} // namespace tf_detail

struct tf_grid {
    int nx = 0, ny = 0;
    double ds = 0.0;
    hipStream_t stream = nullptr;
    int device = 0;
    tf::Model M{};
    bool model_set = false;
    tf_scheme S{};
    int diag_mass = 0;
    double *h = nullptr, *cur = nullptr;
    double *buf[2] = {nullptr, nullptr};
    double *w = nullptr, *bn = nullptr, *rel = nullptr, *ext = nullptr, *chain = nullptr;
    double *partials = nullptr, *hpart = nullptr;
    double *mpart = nullptr;   // per x-solve tile mass records {s, c, min, -} of the last iterate
    double *mout = nullptr;    // {sum, min} combined from mpart
    unsigned long long *res = nullptr, *hres = nullptr;
    int Px = 0, Py = 0;
    int xsweep = TF_XSWEEP_PARTITIONED; // x-sweep variant (TF_XSWEEP_*)
    long iter = 0;
    int successes = 0;
    double t = 0.0;
    bool state_ok = false;
    bool prof = false;
    struct Ev { int kind; hipEvent_t a, b; };
    std::vector<Ev> ev;
    double prof_ms[P_NKIND] = {};
    long prof_n[P_NKIND] = {};
};

namespace {

template <class F>
tf_status timed(tf_grid *g, int kind, F &&launch)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (g->prof) {
        TF_HIP(hipEventCreate(&a));
        TF_HIP(hipEventRecord(a, g->stream));
    }
    const hipError_t e = launch();
    if (e != hipSuccess) return fail(TF_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
    if (g->prof) {
        TF_HIP(hipEventCreate(&b));
        TF_HIP(hipEventRecord(b, g->stream));
        g->ev.push_back({kind, a, b});
    }
    return TF_OK;
}

// Collect finished event pairs (called right after a stream synchronisation).
void prof_flush(tf_grid *g)
{
    for (auto &e : g->ev) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
            g->prof_ms[e.kind] += ms;
            g->prof_n[e.kind] += 1;
        }
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    g->ev.clear();
}

tf::PassParams base_params(const tf_grid *g, double dt)
{
    tf::PassParams P{};
    P.nx = g->nx;
    P.ny = g->ny;
    P.ids2 = 1.0 / (g->ds * g->ds);
    P.f0s = P.ids2 * g->M.cap;
    P.ka = 0.5 * g->S.theta * dt * P.ids2;
    P.K0 = 3.0 * P.ka * P.ids2 * g->M.cap;
    P.K1 = P.ka * g->M.Dn;
    P.M = g->M;
    P.res_spread = tf::RES_SPREAD;
    return P;
}

// One ADI-Newton iteration: y sweep (relations, chain, solve) into w, x sweep into
// u_kp1. The reduction record of slot `slot` receives max|G| (y relations pass) and
// max|v/u_k| and flags (x solve pass); slot (slot+2)%RES_SLOTS is cleared for later.
tf_status enqueue_iteration(tf_grid *g, const double *bnp, const double *uk, double *ukp1, double dt, int slot,
                            bool diag = false)
{
    tf::PassParams P = base_params(g, dt);
    P.u = uk;
    P.rel = g->rel;
    P.ext = g->ext;
    unsigned long long *res = g->res + (size_t)slot * RES_STRIDE;
    unsigned long long *clr = g->res + (size_t)((slot + 2) % RES_SLOTS) * RES_STRIDE;
    tf_status st;
    // y sweep: (I + c J_y) w = -G(u_k)
    P.in2 = bnp;
    P.out = g->w;
    P.res = res;
    P.res_clear = clr;
    P.tiles_x = (g->nx + tf::TILE - 1) / tf::TILE;
    P.tiles_y = g->Py;
    if ((st = timed(g, P_REL_Y, [&] { return tf::launch_pass(0, false, P, g->stream); })) != TF_OK) return st;
    tf::ChainParams C{g->nx, g->Py, g->rel, g->chain, g->ext};
    if ((st = timed(g, P_CHAIN_Y, [&] { return tf::launch_chain(C, g->stream); })) != TF_OK) return st;
    P.res = nullptr;
    P.res_clear = nullptr;
    if ((st = timed(g, P_SOLVE_Y, [&] { return tf::launch_pass(0, true, P, g->stream); })) != TF_OK) return st;
    // x sweep: (I + c J_x) v = w, u_{k+1} = u_k + v
    P.in2 = g->w;
    P.out = ukp1;
    P.tiles_x = g->Px;
    P.tiles_y = (g->ny + tf::TILE - 1) / tf::TILE;
    if (g->xsweep == TF_XSWEEP_ROW) {
        // one whole-row kernel: assembly, elimination, in-row tree, back-substitution, update
        P.res = res;
        P.mass = diag ? g->mpart : nullptr;
        return timed(g, P_XROW, [&] { return tf::launch_xrow(P, g->stream); });
    }
    if ((st = timed(g, P_REL_X, [&] { return tf::launch_pass(1, false, P, g->stream); })) != TF_OK) return st;
    tf::ChainParams Cx{g->ny, g->Px, g->rel, g->chain, g->ext};
    if ((st = timed(g, P_CHAIN_X, [&] { return tf::launch_chain(Cx, g->stream); })) != TF_OK) return st;
    P.res = res;
    P.mass = diag ? g->mpart : nullptr; // mass diagnostic of u_{k+1}, formed as it is stored
    if ((st = timed(g, P_SOLVE_X, [&] { return tf::launch_pass(1, true, P, g->stream); })) != TF_OK) return st;
    return TF_OK;
}

tf_status read_result(tf_grid *g, int slot, double *e, double *r, int *flags)
{
    TF_HIP(hipMemcpyAsync(g->hres, g->res + (size_t)slot * RES_STRIDE, RES_STRIDE * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, g->stream));
    TF_HIP(hipStreamSynchronize(g->stream));
    if (g->prof) prof_flush(g);
    // combine the copies: maxima of non-negative doubles compare as their bit patterns
    unsigned long long em = 0, rm = 0, fl = 0;
    for (int c = 0; c < tf::RES_SPREAD; ++c) {
        const unsigned long long *w = g->hres + (size_t)c * tf::RES_WORDS;
        em = std::max(em, w[tf::RES_EMAX]);
        rm = std::max(rm, w[tf::RES_RMAX]);
        fl |= w[tf::RES_FLAGS];
    }
    double ev, rv;
    std::memcpy(&ev, &em, sizeof(double));
    std::memcpy(&rv, &rm, sizeof(double));
    *e = ev;
    *r = rv;
    *flags = (int)fl;
    return TF_OK;
}

tf_status rhs_theta(tf_grid *g, const double *un, double dt)
{
    const double ids = 1.0 / g->ds, ids2 = ids * ids;
    const double beta = -(1.0 - g->S.theta) * dt;
    return timed(g, P_RHS, [&] {
        return tf::launch_flux_divergence(g->nx, g->ny, ids, ids2, g->M, un, 1.0, beta, un, g->bn, g->stream);
    });
}

tf_status mass_of(tf_grid *g, const double *u, double *mass, double *hmin, bool *nan)
{
    const size_t n = (size_t)g->nx * g->ny;
    const int nb = tf::mass_blocks(n);
    tf_status st = timed(g, P_MASS, [&] { return tf::launch_mass(u, n, g->partials, nb, g->stream); });
    if (st != TF_OK) return st;
    TF_HIP(hipMemcpyAsync(g->hpart, g->partials, (size_t)nb * 4 * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    TF_HIP(hipStreamSynchronize(g->stream));
    if (g->prof) prof_flush(g);
    double s = 0.0, c = 0.0, m = INFINITY;
    bool isn = false;
    for (int b = 0; b < nb; ++b) {
        const double x = g->hpart[4 * b], cx = g->hpart[4 * b + 1];
        const double t = s + x;
        c += (std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s) + cx;
        s = t;
        m = std::fmin(m, g->hpart[4 * b + 2]);
        if (g->hpart[4 * b + 3] != 0.0) isn = true;
    }
    *mass = s + c;
    *hmin = m;
    if (nan) *nan = isn;
    return TF_OK;
}

int x_tiles(const tf_grid *g) { return g->Px * ((g->ny + tf::TILE - 1) / tf::TILE); }
// Mass records the x sweep leaves (one per x-solve tile or per whole-row workgroup).
int mass_records(const tf_grid *g)
{
    return g->xsweep == TF_XSWEEP_ROW ? tf::xrow_blocks(g->nx, g->ny) : x_tiles(g);
}

// Mass and minimum of the last iterate from the records its x solve left per tile (Sec.
// "Conservation of Mass"), combined on the device in a fixed order: no extra read of h.
tf_status fused_mass(tf_grid *g, double *mass, double *hmin)
{
    tf_status st = timed(g, P_MASS, [&] { return tf::launch_mass_tiles(g->mpart, mass_records(g), g->mout, g->stream); });
    if (st != TF_OK) return st;
    TF_HIP(hipMemcpyAsync(g->hpart, g->mout, 2 * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    TF_HIP(hipStreamSynchronize(g->stream));
    if (g->prof) prof_flush(g);
    *mass = g->hpart[0];
    *hmin = g->hpart[1];
    return TF_OK;
}

double *pick_buffer(tf_grid *g, const double *a, const double *b)
{
    double *cand[3] = {g->h, g->buf[0], g->buf[1]};
    for (double *c : cand)
        if (c != a && c != b) return c;
    return nullptr;
}

tf_status ensure_ready(tf_grid *g)
{
    if (!g->model_set) return fail(TF_ESTATE, "model not set (tf_set_model)");
    if (g->h == nullptr) return fail(TF_ESTATE, "no state bound (tf_bind_state)");
    return TF_OK;
}

tf_status validate_state(tf_grid *g)
{
    if (g->state_ok) return TF_OK;
    double m, hmin;
    bool isn;
    tf_status st = mass_of(g, g->cur, &m, &hmin, &isn);
    if (st != TF_OK) return st;
    if (isn || !(hmin > 0.0)) return fail(TF_ENONPOS, "state holds h <= 0 or NaN");
    g->state_ok = true;
    return TF_OK;
}

tf_status copy_back(tf_grid *g)
{
    if (g->cur != g->h) {
        TF_HIP(hipMemcpyAsync(g->h, g->cur, (size_t)g->nx * g->ny * sizeof(double), hipMemcpyDeviceToDevice,
                              g->stream));
        g->cur = g->h;
    }
    TF_HIP(hipStreamSynchronize(g->stream));
    if (g->prof) prof_flush(g);
    return TF_OK;
}

// One accepted step with the control of Fig. FlowChartTime (state stays in g->cur).
tf_status do_step(tf_grid *g, double *dt_inout, tf_step_info *info)
{
    double dt = *dt_inout;
    if (!(dt > 0.0)) return fail(TF_EINVAL, "dt must be positive");
    tf_status st = validate_state(g);
    if (st != TF_OK) return st;
    double *un = g->cur;
    int rejections = 0, total = 0, iters = 0;
    double e = 0.0, r = 0.0;
    tf_status status = TF_ENOCONV;
    for (;;) {
        const double *bnp = un;
        if (g->S.theta < 1.0) {
            if ((st = rhs_theta(g, un, dt)) != TF_OK) return st;
            bnp = g->bn;
        }
        double *uk = un;
        bool accepted = false;
        for (iters = 1; iters <= g->S.max_newton; ++iters) {
            double *dst = pick_buffer(g, un, uk);
            const int slot = (int)(g->iter % RES_SLOTS);
            if ((st = enqueue_iteration(g, bnp, uk, dst, dt, slot, info != nullptr && g->diag_mass)) != TF_OK)
                return st;
            g->iter++;
            int flags = 0;
            if ((st = read_result(g, slot, &e, &r, &flags)) != TF_OK) return st;
            ++total;
            if (flags != 0) break; // an iterate left the admissible set (h <= 0 or NaN)
            uk = dst;
            if (e < g->S.tol) { accepted = true; break; }
        }
        if (accepted) {
            g->cur = uk;
            status = TF_OK;
            break;
        }
        ++rejections;
        g->successes = 0;
        if (!g->S.adaptive) break;
        dt *= g->S.dt_shrink;
        if (dt < g->S.dt_min) break;
    }
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->dt_used = dt;
        info->e_final = e;
        info->r_final = r;
        info->newton_iters = iters;
        info->rejections = rejections;
        info->total_iters = total;
        info->status = status;
    }
    if (status != TF_OK) {
        *dt_inout = dt;
        return fail(status, "Newton iteration did not converge (dt below dt_min or fixed dt)");
    }
    g->t += dt;
    if (info) info->t = g->t;
    g->successes += 1;
    if (g->S.adaptive && g->successes >= g->S.grow_after) {
        dt = std::fmin(dt * g->S.dt_grow, g->S.dt_max);
        g->successes = 0;
    }
    *dt_inout = dt;
    if (info && g->diag_mass) {
        // the accepted state is the last iterate: its x solve left the mass records
        double m, hm;
        if ((st = fused_mass(g, &m, &hm)) != TF_OK) return st;
        info->mass = m;
        info->hmin = hm;
    }
    return TF_OK;
}

bool is_int(double x) { return std::isfinite(x) && std::floor(x) == x; }

} // namespace

namespace tf_detail {
bool grid_view(const tf_grid *g, GridView *v)
{
    if (g == nullptr || !g->model_set) return false;
    v->nx = g->nx;
    v->ny = g->ny;
    v->ds = g->ds;
    v->theta = g->S.theta;
    v->M = g->M;
    v->stream = g->stream;
    v->rel = g->rel;
    v->ext = g->ext;
    v->chain = g->chain;
    v->xsweep = g->xsweep;
    return true;
}
} // namespace tf_detail

extern "C" {

const char *tf_last_error(void) { return g_err.c_str(); }

const char *tf_profile_names(void) { return kProfNames; }

tf_status tf_create(int nx, int ny, double ds, void *stream, tf_grid **out)
{
    if (out == nullptr) return fail(TF_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 4 || ny < 4) return fail(TF_EINVAL, "nx and ny must be >= 4");
    if (!(ds > 0.0) || !std::isfinite(ds)) return fail(TF_EINVAL, "ds must be positive and finite");
    if ((double)nx * (double)ny > 4.0e9) return fail(TF_EINVAL, "grid too large");
    tf_grid *g = new (std::nothrow) tf_grid();
    if (g == nullptr) return fail(TF_ENOMEM, "host allocation failed");
    g->nx = nx;
    g->ny = ny;
    g->ds = ds;
    g->stream = (hipStream_t)stream;
    g->S = tf_scheme{1.0, 1e-10, 1e-6, 1.0, 0.5, 1.1, 5000, 5, 0};
    g->Px = tf::seg_count(nx);
    g->Py = tf::seg_count(ny);
    g->xsweep = tf::xsweep_choice(nx, ny) == 1 ? TF_XSWEEP_ROW : TF_XSWEEP_PARTITIONED;
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return fail(TF_EDEVICE, "hipGetDevice failed");
    }
    const size_t N = (size_t)nx * ny;
    const size_t lines_seg = std::max((size_t)g->Py * nx, (size_t)g->Px * ny);
    bool ok = hipMalloc(&g->buf[0], N * sizeof(double)) == hipSuccess
              && hipMalloc(&g->buf[1], N * sizeof(double)) == hipSuccess
              && hipMalloc(&g->w, N * sizeof(double)) == hipSuccess
              && hipMalloc(&g->rel, lines_seg * tf::NREL * sizeof(double)) == hipSuccess
              && hipMalloc(&g->ext, lines_seg * tf::NEXT * sizeof(double)) == hipSuccess
              && hipMalloc(&g->chain, lines_seg * tf::NCHAIN * sizeof(double)) == hipSuccess
              && hipMalloc(&g->partials, 4096 * 4 * sizeof(double)) == hipSuccess
              && hipMalloc(&g->mpart, (size_t)std::max(x_tiles(g), tf::xrow_supported(nx) ? tf::xrow_blocks(nx, ny) : 0)
                                          * 4 * sizeof(double)) == hipSuccess
              && hipMalloc(&g->mout, 2 * sizeof(double)) == hipSuccess
              && hipMalloc(&g->res, RES_SLOTS * RES_STRIDE * sizeof(unsigned long long)) == hipSuccess
              && hipHostMalloc(&g->hres, RES_STRIDE * sizeof(unsigned long long), hipHostMallocDefault) == hipSuccess
              && hipHostMalloc(&g->hpart, 4096 * 4 * sizeof(double), hipHostMallocDefault) == hipSuccess;
    if (ok) ok = hipMemsetAsync(g->res, 0, RES_SLOTS * RES_STRIDE * sizeof(unsigned long long), g->stream) == hipSuccess
                 && hipStreamSynchronize(g->stream) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        tf_destroy(g);
        return fail(TF_ENOMEM, "device allocation failed");
    }
    *out = g;
    return TF_OK;
}

tf_status tf_destroy(tf_grid *g)
{
    if (g == nullptr) return TF_OK;
    (void)hipStreamSynchronize(g->stream);
    tf_detail::release_adjoint(g);
    for (auto &e : g->ev) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    (void)hipFree(g->buf[0]);
    (void)hipFree(g->buf[1]);
    (void)hipFree(g->w);
    (void)hipFree(g->bn);
    (void)hipFree(g->rel);
    (void)hipFree(g->ext);
    (void)hipFree(g->chain);
    (void)hipFree(g->partials);
    (void)hipFree(g->mpart);
    (void)hipFree(g->mout);
    (void)hipFree(g->res);
    if (g->hres) (void)hipHostFree(g->hres);
    if (g->hpart) (void)hipHostFree(g->hpart);
    delete g;
    return TF_OK;
}

tf_status tf_set_model(tf_grid *g, double kappa, double b, double n, double m)
{
    if (g == nullptr) return fail(TF_EINVAL, "grid is NULL");
    if (!(b > 0.0) || !std::isfinite(b) || !std::isfinite(kappa)) return fail(TF_EINVAL, "need b > 0 and finite kappa");
    if (!is_int(n) || !is_int(m) || !(n > m) || m < 1 || n > 16)
        return fail(TF_EINVAL, "exponents must be integers with 16 >= n > m >= 1");
    tf::Model M{};
    M.kappa = kappa;
    M.b = b;
    M.n = (int)n;
    M.m = (int)m;
    M.Cn = kappa * n * std::pow(b, n);
    M.Cm = kappa * m * std::pow(b, m);
    M.Dn = kappa * n * (n - 2.0) * std::pow(b, n);
    M.Dm = kappa * m * (m - 2.0) * std::pow(b, m);
    M.p32 = (M.n == 3 && M.m == 2);
    M.kind = tf::MODEL_POWER;
    M.cap = 1.0;
    g->M = M;
    g->model_set = true;
    g->state_ok = false;
    return TF_OK;
}

tf_status tf_set_model_linear(tf_grid *g, double c0, double c1)
{
    if (g == nullptr) return fail(TF_EINVAL, "grid is NULL");
    std::string err;
    if (!tf_detail::linear_model(c0, c1, &g->M, &err)) return fail(TF_EINVAL, err);
    g->model_set = true;
    g->state_ok = false;
    return TF_OK;
}

tf_status tf_set_model_nlc(tf_grid *g, double C, double K, double N, double beta, double w, double b)
{
    if (g == nullptr) return fail(TF_EINVAL, "grid is NULL");
    std::string err;
    if (!tf_detail::nlc_model(C, K, N, beta, w, b, &g->M, &err)) return fail(TF_EINVAL, err);
    g->model_set = true;
    g->state_ok = false;
    return TF_OK;
}

tf_status tf_set_model_polymer(tf_grid *g, double C, double Cst, double Aox, double Asi, double d)
{
    if (g == nullptr) return fail(TF_EINVAL, "grid is NULL");
    std::string err;
    if (!tf_detail::polymer_model(C, Cst, Aox, Asi, d, &g->M, &err)) return fail(TF_EINVAL, err);
    g->model_set = true;
    g->state_ok = false;
    return TF_OK;
}

tf_status tf_set_scheme(tf_grid *g, const tf_scheme *s)
{
    if (g == nullptr || s == nullptr) return fail(TF_EINVAL, "NULL argument");
    if (!(s->theta >= 0.5 && s->theta <= 1.0)) return fail(TF_EINVAL, "theta must lie in [0.5, 1]");
    if (!(s->tol > 0.0) || s->max_newton < 1) return fail(TF_EINVAL, "need tol > 0 and max_newton >= 1");
    if (s->adaptive && (!(s->dt_shrink > 0.0 && s->dt_shrink < 1.0) || !(s->dt_grow >= 1.0) || !(s->dt_min > 0.0)
                        || !(s->dt_max >= s->dt_min) || s->grow_after < 1))
        return fail(TF_EINVAL, "inconsistent adaptive-dt parameters");
    if (s->theta < 1.0 && g->bn == nullptr) {
        if (hipMalloc(&g->bn, (size_t)g->nx * g->ny * sizeof(double)) != hipSuccess) {
            g->bn = nullptr;
            return fail(TF_ENOMEM, "device allocation failed");
        }
    }
    g->S = *s;
    return TF_OK;
}

tf_status tf_get_scheme(const tf_grid *g, tf_scheme *s)
{
    if (g == nullptr || s == nullptr) return fail(TF_EINVAL, "NULL argument");
    *s = g->S;
    return TF_OK;
}

tf_status tf_set_xsweep(tf_grid *g, int variant)
{
    if (g == nullptr) return fail(TF_EINVAL, "grid is NULL");
    if (variant == TF_XSWEEP_AUTO)
        variant = tf::xsweep_choice(g->nx, g->ny) == 1 ? TF_XSWEEP_ROW : TF_XSWEEP_PARTITIONED;
    if (variant != TF_XSWEEP_PARTITIONED && variant != TF_XSWEEP_ROW)
        return fail(TF_EINVAL, "unknown x-sweep variant");
    if (variant == TF_XSWEEP_ROW && !tf::xrow_supported(g->nx))
        return fail(TF_EINVAL, "the whole-row x sweep needs 4 <= nx <= " + std::to_string(tf::XR_MAX_NX));
    g->xsweep = variant;
    return TF_OK;
}

int tf_get_xsweep(const tf_grid *g) { return g == nullptr ? -1 : g->xsweep; }

tf_status tf_set_diagnostics(tf_grid *g, int mass_every_step)
{
    if (g == nullptr) return fail(TF_EINVAL, "grid is NULL");
    g->diag_mass = mass_every_step != 0;
    return TF_OK;
}

tf_status tf_bind_state(tf_grid *g, double *h_dev)
{
    if (g == nullptr) return fail(TF_EINVAL, "grid is NULL");
    g->h = h_dev;
    g->cur = h_dev;
    g->t = 0.0;
    g->successes = 0;
    g->state_ok = false;
    return TF_OK;
}

tf_status tf_get_clock(const tf_grid *g, double *t, int *successes)
{
    if (g == nullptr || t == nullptr || successes == nullptr) return fail(TF_EINVAL, "NULL argument");
    *t = g->t;
    *successes = g->successes;
    return TF_OK;
}

tf_status tf_set_clock(tf_grid *g, double t, int successes)
{
    if (g == nullptr) return fail(TF_EINVAL, "grid is NULL");
    if (!std::isfinite(t) || successes < 0) return fail(TF_EINVAL, "need finite t and successes >= 0");
    g->t = t;
    g->successes = successes;
    return TF_OK;
}

tf_status tf_step(tf_grid *g, double *dt_inout, tf_step_info *info)
{
    if (g == nullptr || dt_inout == nullptr) return fail(TF_EINVAL, "NULL argument");
    tf_status st = ensure_ready(g);
    if (st != TF_OK) return st;
    st = do_step(g, dt_inout, info);
    const tf_status cb = copy_back(g);
    return st != TF_OK ? st : cb;
}

tf_status tf_advance(tf_grid *g, int nsteps, double *dt_inout, tf_step_info *log)
{
    if (g == nullptr || dt_inout == nullptr || nsteps < 0) return fail(TF_EINVAL, "bad argument");
    tf_status st = ensure_ready(g);
    if (st != TF_OK) return st;
    for (int s = 0; s < nsteps && st == TF_OK; ++s) st = do_step(g, dt_inout, log ? &log[s] : nullptr);
    const tf_status cb = copy_back(g);
    return st != TF_OK ? st : cb;
}

tf_status tf_advance_keep(tf_grid *g, int nsteps, double *dt_inout, double *const *states, tf_step_info *log)
{
    if (g == nullptr || dt_inout == nullptr || nsteps < 0 || (nsteps > 0 && states == nullptr))
        return fail(TF_EINVAL, "bad argument");
    for (int s = 0; s < nsteps; ++s)
        if (states[s] == nullptr) return fail(TF_EINVAL, "NULL state buffer");
    tf_status st = ensure_ready(g);
    if (st != TF_OK) return st;
    const size_t bytes = (size_t)g->nx * g->ny * sizeof(double);
    for (int s = 0; s < nsteps && st == TF_OK; ++s) {
        st = do_step(g, dt_inout, log ? &log[s] : nullptr);
        if (st == TF_OK) {
            const hipError_t e = hipMemcpyAsync(states[s], g->cur, bytes, hipMemcpyDeviceToDevice, g->stream);
            if (e != hipSuccess) st = fail(TF_EDEVICE, std::string("state copy: ") + hipGetErrorString(e));
        }
    }
    const tf_status cb = copy_back(g);
    return st != TF_OK ? st : cb;
}

tf_status tf_mass(tf_grid *g, double *mass, double *hmin)
{
    if (g == nullptr || mass == nullptr || hmin == nullptr) return fail(TF_EINVAL, "NULL argument");
    if (g->h == nullptr) return fail(TF_ESTATE, "no state bound");
    return mass_of(g, g->cur, mass, hmin, nullptr);
}

tf_status tf_newton_iteration(tf_grid *g, const double *u_n, const double *u_k, double *u_kp1, double dt, double *e,
                              double *r, int *flags)
{
    if (g == nullptr || u_n == nullptr || u_k == nullptr || u_kp1 == nullptr || e == nullptr || r == nullptr
        || flags == nullptr)
        return fail(TF_EINVAL, "NULL argument");
    if (u_kp1 == u_k || u_kp1 == u_n) return fail(TF_EINVAL, "u_kp1 must not alias u_k or u_n");
    if (!(dt > 0.0)) return fail(TF_EINVAL, "dt must be positive");
    if (!g->model_set) return fail(TF_ESTATE, "model not set");
    const double *bnp = u_n;
    tf_status st;
    if (g->S.theta < 1.0) {
        if ((st = rhs_theta(g, u_n, dt)) != TF_OK) return st;
        bnp = g->bn;
    }
    const int slot = (int)(g->iter % RES_SLOTS);
    if ((st = enqueue_iteration(g, bnp, u_k, u_kp1, dt, slot)) != TF_OK) return st;
    g->iter++;
    return read_result(g, slot, e, r, flags);
}

tf_status tf_flux_divergence(tf_grid *g, const double *u, double *out)
{
    if (g == nullptr || u == nullptr || out == nullptr) return fail(TF_EINVAL, "NULL argument");
    if (!g->model_set) return fail(TF_ESTATE, "model not set");
    const double ids = 1.0 / g->ds;
    const hipError_t e =
        tf::launch_flux_divergence(g->nx, g->ny, ids, ids * ids, g->M, u, 0.0, 1.0, nullptr, out, g->stream);
    if (e != hipSuccess) return fail(TF_EDEVICE, hipGetErrorString(e));
    TF_HIP(hipStreamSynchronize(g->stream));
    return TF_OK;
}

tf_status tf_model_coeffs(tf_grid *g, const double *h, int n, double *out)
{
    if (g == nullptr || (n > 0 && (h == nullptr || out == nullptr))) return fail(TF_EINVAL, "NULL argument");
    if (n < 0) return fail(TF_EINVAL, "n must be >= 0");
    if (!g->model_set) return fail(TF_ESTATE, "model not set");
    const hipError_t e = tf::launch_model_coeffs(g->M, h, n, out, g->stream);
    if (e != hipSuccess) return fail(TF_EDEVICE, hipGetErrorString(e));
    TF_HIP(hipStreamSynchronize(g->stream));
    return TF_OK;
}

tf_status tf_profile(tf_grid *g, int on)
{
    if (g == nullptr) return fail(TF_EINVAL, "grid is NULL");
    TF_HIP(hipStreamSynchronize(g->stream));
    prof_flush(g);
    for (int k = 0; k < P_NKIND; ++k) {
        g->prof_ms[k] = 0.0;
        g->prof_n[k] = 0;
    }
    g->prof = on != 0;
    return TF_OK;
}

int tf_profile_read(tf_grid *g, double *ms, long *count, int n)
{
    if (g == nullptr) return 0;
    if (hipStreamSynchronize(g->stream) == hipSuccess) prof_flush(g);
    const int k = n < P_NKIND ? n : P_NKIND;
    for (int i = 0; i < k; ++i) {
        if (ms) ms[i] = g->prof_ms[i];
        if (count) count[i] = g->prof_n[i];
    }
    return P_NKIND;
}

} // extern "C"
