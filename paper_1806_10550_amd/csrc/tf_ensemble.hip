// Ensemble of films (ragged sizes, per-film kappa and ds) advanced in lockstep by one
// captured HIP graph per Newton iteration (see include/thinfilm.h, tf_ensemble_*).
//
// Every film keeps its own Newton / dt state on the device (FilmState); the work-list
// kernels read it, so the same graph serves all iterations of all films: films that
// have converged (or failed) leave their tiles immediately. After each batch of graph
// replays the host reads one integer, the number of films still iterating.
#include "tf_internal.h"
#include "../../include/thinfilm.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

namespace tf_detail {
void set_error(const std::string &msg);
}

namespace {

tf_status efail(tf_status s, const std::string &msg)
{
    tf_detail::set_error(msg);
    return s;
}

#define TF_EHIP(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return efail(TF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool is_int(double x) { return std::isfinite(x) && std::floor(x) == x; }

} // namespace

struct tf_ensemble {
    int nfilms = 0;
    hipStream_t user = nullptr, stream = nullptr;
    tf_scheme S{};
    std::vector<tf::FilmDesc> desc;
    long long ncells = 0, nrec = 0;
    int ny_items = 0, nx_items = 0, ncy_items = 0, ncx_items = 0, nxr_items = 0;
    tf::FilmDesc *d_desc = nullptr;
    tf::FilmState *d_state = nullptr, *h_state = nullptr;
    // [y tiles | x tiles | y chain blocks | x chain blocks | whole-row blocks]; the x tiles and
    // x chain blocks cover the films whose x sweep is partitioned, the row blocks the others
    int *d_items = nullptr;
    std::vector<int> xsweep;  // per film: 1 = whole-row x sweep, 0 = partitioned
    int *d_active = nullptr, *h_active = nullptr;
    double *buf0 = nullptr, *buf1 = nullptr, *buf2 = nullptr, *w = nullptr;
    double *rel = nullptr, *ext = nullptr, *chain = nullptr;
    double *bn = nullptr;  // packed b^n (allocated when a scheme with theta < 1 is set)
    int km = tf::KM_P32; // model form of the sweep kernels (one model for every film)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int prev_iters = 4;
};

namespace {

tf::EnsParams params(const tf_ensemble *e, int which)
{
    tf::EnsParams p{};
    p.desc = e->d_desc;
    p.state = e->d_state;
    p.buf0 = e->buf0;
    p.buf1 = e->buf1;
    p.buf2 = e->buf2;
    p.w = e->w;
    p.rel = e->rel;
    p.ext = e->ext;
    p.chain = e->chain;
    p.bn = e->bn;
    p.theta = e->S.theta;
    const int off_y = 0, off_x = 3 * e->ny_items, off_cy = off_x + 3 * e->nx_items, off_cx = off_cy + 2 * e->ncy_items;
    const int off_xr = off_cx + 2 * e->ncx_items;
    switch (which) {
    case 0: p.items = e->d_items + off_y; p.nitems = e->ny_items; break;
    case 1: p.items = e->d_items + off_x; p.nitems = e->nx_items; break;
    case 2: p.items = e->d_items + off_cy; p.nitems = e->ncy_items; break;
    case 3: p.items = e->d_items + off_cx; p.nitems = e->ncx_items; break;
    default: p.items = e->d_items + off_xr; p.nitems = e->nxr_items; break;
    }
    return p;
}

tf_status enqueue_iteration(tf_ensemble *e)
{
    const tf::EnsScheme S{e->S.theta, e->S.tol, e->S.dt_min, e->S.dt_max, e->S.dt_shrink, e->S.dt_grow,
                          e->S.max_newton, e->S.grow_after, e->S.adaptive};
    if (e->S.theta < 1.0) TF_EHIP(tf::launch_bn_ens(params(e, 0), e->stream));
    TF_EHIP(tf::launch_pass_ens(0, false, e->km, params(e, 0), e->stream));
    TF_EHIP(tf::launch_chain_ens(params(e, 2), 0, e->stream));
    TF_EHIP(tf::launch_pass_ens(0, true, e->km, params(e, 0), e->stream));
    if (e->nx_items > 0) {
        TF_EHIP(tf::launch_pass_ens(1, false, e->km, params(e, 1), e->stream));
        TF_EHIP(tf::launch_chain_ens(params(e, 3), 1, e->stream));
        TF_EHIP(tf::launch_pass_ens(1, true, e->km, params(e, 1), e->stream));
    }
    if (e->nxr_items > 0) TF_EHIP(tf::launch_xrow_ens(e->km, params(e, 4), e->stream));
    TF_EHIP(tf::launch_ens_control(e->d_state, e->nfilms, S, e->d_active, e->stream));
    return TF_OK;
}

void drop_graph(tf_ensemble *e)
{
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    e->exec = nullptr;
    e->graph = nullptr;
}

tf_status ensure_graph(tf_ensemble *e)
{
    if (e->exec) return TF_OK;
    TF_EHIP(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
    const tf_status st = enqueue_iteration(e);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(e->stream, &g);
    if (st != TF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (ce != hipSuccess) return efail(TF_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    e->graph = g;
    TF_EHIP(hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0));
    return TF_OK;
}

// Replace every film's model by M (kernel form km) and upload the film table.
tf_status set_all_models(tf_ensemble *e, const tf::Model &M, int km)
{
    for (auto &d : e->desc) d.M = M;
    TF_EHIP(hipMemcpyAsync(e->d_desc, e->desc.data(), e->nfilms * sizeof(tf::FilmDesc), hipMemcpyHostToDevice,
                           e->stream));
    TF_EHIP(hipStreamSynchronize(e->stream));
    e->km = km;
    drop_graph(e);
    return TF_OK;
}

// Work lists of one iteration (see tf_ensemble::d_items); the x sweep of film f is
// whole-row when xsweep[f] == 1.
void build_items(tf_ensemble *e, std::vector<int> &items)
{
    std::vector<int> items_y, items_x, items_cy, items_cx, items_xr;
    for (int f = 0; f < e->nfilms; ++f) {
        const tf::FilmDesc &d = e->desc[f];
        const int tyx = (d.nx + tf::TILE - 1) / tf::TILE;
        for (int ty = 0; ty < d.Py; ++ty)
            for (int tx = 0; tx < tyx; ++tx) { items_y.push_back(f); items_y.push_back(tx); items_y.push_back(ty); }
        for (int lb = 0; lb < (d.nx + 63) / 64; ++lb) { items_cy.push_back(f); items_cy.push_back(lb); }
        if (e->xsweep[f] == 1) {
            for (int rb = 0; rb < tf::xrow_blocks(d.nx, d.ny); ++rb) { items_xr.push_back(f); items_xr.push_back(rb); }
        } else {
            const int txy = (d.ny + tf::TILE - 1) / tf::TILE;
            for (int ty = 0; ty < txy; ++ty)
                for (int tx = 0; tx < d.Px; ++tx) { items_x.push_back(f); items_x.push_back(tx); items_x.push_back(ty); }
            for (int lb = 0; lb < (d.ny + 63) / 64; ++lb) { items_cx.push_back(f); items_cx.push_back(lb); }
        }
    }
    e->ny_items = (int)items_y.size() / 3;
    e->nx_items = (int)items_x.size() / 3;
    e->ncy_items = (int)items_cy.size() / 2;
    e->ncx_items = (int)items_cx.size() / 2;
    e->nxr_items = (int)items_xr.size() / 2;
    items.clear();
    items.insert(items.end(), items_y.begin(), items_y.end());
    items.insert(items.end(), items_x.begin(), items_x.end());
    items.insert(items.end(), items_cy.begin(), items_cy.end());
    items.insert(items.end(), items_cx.begin(), items_cx.end());
    items.insert(items.end(), items_xr.begin(), items_xr.end());
}

// Rows of all films: the x sweep of an ensemble is one launch over every film's rows, so the
// automatic variant choice takes this as its batch.
int total_rows(const tf_ensemble *e)
{
    long long n = 0;
    for (const auto &d : e->desc) n += d.ny;
    return (int)std::min(n, (long long)1 << 30);
}

// Work-list capacity for any choice of x-sweep variants.
size_t max_items(const tf_ensemble *e)
{
    size_t n = 0;
    for (const auto &d : e->desc) {
        n += 3 * (size_t)d.Py * ((d.nx + tf::TILE - 1) / tf::TILE) + 2 * (size_t)((d.nx + 63) / 64);
        n += std::max(3 * (size_t)((d.ny + tf::TILE - 1) / tf::TILE) * d.Px + 2 * (size_t)((d.ny + 63) / 64),
                      tf::xrow_supported(d.nx) ? 2 * (size_t)tf::xrow_blocks(d.nx, d.ny) : 0);
    }
    return n;
}

} // namespace

extern "C" {

tf_status tf_ensemble_create(int nfilms, const int *nx, const int *ny, const double *ds, const double *kappa, double b,
                             double n, double m, void *stream, tf_ensemble **out)
{
    if (out == nullptr) return efail(TF_EINVAL, "out is NULL");
    *out = nullptr;
    if (nfilms < 1 || nx == nullptr || ny == nullptr || ds == nullptr || kappa == nullptr)
        return efail(TF_EINVAL, "need nfilms >= 1 and per-film arrays");
    if (!(b > 0.0) || !is_int(n) || !is_int(m) || !(n > m) || m < 1 || n > 16)
        return efail(TF_EINVAL, "need b > 0 and integer exponents 16 >= n > m >= 1");
    tf_ensemble *e = new (std::nothrow) tf_ensemble();
    if (e == nullptr) return efail(TF_ENOMEM, "host allocation failed");
    e->nfilms = nfilms;
    e->user = (hipStream_t)stream;
    e->S = tf_scheme{1.0, 1e-10, 1e-6, 1.0, 0.5, 1.1, 5000, 5, 0};
    const bool p32 = ((int)n == 3 && (int)m == 2);
    e->km = p32 ? tf::KM_P32 : tf::KM_POWER;
    for (int f = 0; f < nfilms; ++f) {
        if (nx[f] < 4 || ny[f] < 4 || !(ds[f] > 0.0) || !std::isfinite(kappa[f])) {
            delete e;
            return efail(TF_EINVAL, "film " + std::to_string(f) + ": need nx, ny >= 4, ds > 0, finite kappa");
        }
        tf::FilmDesc d{};
        d.nx = nx[f];
        d.ny = ny[f];
        d.Px = tf::seg_count(nx[f]);
        d.Py = tf::seg_count(ny[f]);
        d.ds = ds[f];
        tf::Model M{};
        M.kappa = kappa[f];
        M.b = b;
        M.n = (int)n;
        M.m = (int)m;
        M.Cn = kappa[f] * n * std::pow(b, n);
        M.Cm = kappa[f] * m * std::pow(b, m);
        M.Dn = kappa[f] * n * (n - 2.0) * std::pow(b, n);
        M.Dm = kappa[f] * m * (m - 2.0) * std::pow(b, m);
        M.p32 = p32;
        M.kind = tf::MODEL_POWER;
        M.cap = 1.0;
        d.M = M;
        d.off = e->ncells;
        d.roff = e->nrec;
        e->ncells += (long long)nx[f] * ny[f];
        e->nrec += std::max((long long)d.Py * nx[f], (long long)d.Px * ny[f]);
        e->desc.push_back(d);
    }
    e->xsweep.assign(nfilms, 0);
    for (int f = 0; f < nfilms; ++f) e->xsweep[f] = tf::xsweep_choice(nx[f], total_rows(e));
    std::vector<int> items;
    build_items(e, items);
    const size_t N = (size_t)e->ncells, R = (size_t)e->nrec;
    bool ok = hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) == hipSuccess
              && hipMalloc(&e->d_desc, nfilms * sizeof(tf::FilmDesc)) == hipSuccess
              && hipMalloc(&e->d_state, nfilms * sizeof(tf::FilmState)) == hipSuccess
              && hipHostMalloc(&e->h_state, nfilms * sizeof(tf::FilmState), hipHostMallocDefault) == hipSuccess
              && hipMalloc(&e->d_items, max_items(e) * sizeof(int)) == hipSuccess
              && hipMalloc(&e->d_active, sizeof(int)) == hipSuccess
              && hipHostMalloc(&e->h_active, sizeof(int), hipHostMallocDefault) == hipSuccess
              && hipMalloc(&e->buf1, N * sizeof(double)) == hipSuccess
              && hipMalloc(&e->buf2, N * sizeof(double)) == hipSuccess
              && hipMalloc(&e->w, N * sizeof(double)) == hipSuccess
              && hipMalloc(&e->rel, R * tf::NREL * sizeof(double)) == hipSuccess
              && hipMalloc(&e->ext, R * tf::NEXT * sizeof(double)) == hipSuccess
              && hipMalloc(&e->chain, R * tf::NCHAIN * sizeof(double)) == hipSuccess;
    if (ok) {
        std::memset(e->h_state, 0, nfilms * sizeof(tf::FilmState));
        ok = hipMemcpyAsync(e->d_desc, e->desc.data(), nfilms * sizeof(tf::FilmDesc), hipMemcpyHostToDevice, e->stream)
                 == hipSuccess
             && hipMemcpyAsync(e->d_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice, e->stream)
                    == hipSuccess
             && hipMemcpyAsync(e->d_state, e->h_state, nfilms * sizeof(tf::FilmState), hipMemcpyHostToDevice,
                               e->stream) == hipSuccess
             && hipStreamSynchronize(e->stream) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        tf_ensemble_destroy(e);
        return efail(TF_ENOMEM, "device allocation failed");
    }
    *out = e;
    return TF_OK;
}

tf_status tf_ensemble_destroy(tf_ensemble *e)
{
    if (e == nullptr) return TF_OK;
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    drop_graph(e);
    (void)hipFree(e->d_desc);
    (void)hipFree(e->d_state);
    (void)hipFree(e->d_items);
    (void)hipFree(e->d_active);
    (void)hipFree(e->buf1);
    (void)hipFree(e->buf2);
    (void)hipFree(e->w);
    (void)hipFree(e->rel);
    (void)hipFree(e->ext);
    (void)hipFree(e->chain);
    (void)hipFree(e->bn);
    if (e->h_state) (void)hipHostFree(e->h_state);
    if (e->h_active) (void)hipHostFree(e->h_active);
    if (e->stream) (void)hipStreamDestroy(e->stream);
    delete e;
    return TF_OK;
}

long long tf_ensemble_size(const tf_ensemble *e) { return e ? e->ncells : 0; }

tf_status tf_ensemble_offsets(const tf_ensemble *e, long long *offsets)
{
    if (e == nullptr || offsets == nullptr) return efail(TF_EINVAL, "NULL argument");
    for (int f = 0; f < e->nfilms; ++f) offsets[f] = e->desc[f].off;
    return TF_OK;
}

tf_status tf_ensemble_set_scheme(tf_ensemble *e, const tf_scheme *s)
{
    if (e == nullptr || s == nullptr) return efail(TF_EINVAL, "NULL argument");
    if (!(s->theta >= 0.5 && s->theta <= 1.0)) return efail(TF_EINVAL, "theta must lie in [0.5, 1]");
    if (!(s->tol > 0.0) || s->max_newton < 1) return efail(TF_EINVAL, "need tol > 0 and max_newton >= 1");
    if (s->adaptive && (!(s->dt_shrink > 0.0 && s->dt_shrink < 1.0) || !(s->dt_grow >= 1.0) || !(s->dt_min > 0.0)
                        || !(s->dt_max >= s->dt_min) || s->grow_after < 1))
        return efail(TF_EINVAL, "inconsistent adaptive-dt parameters");
    if (s->theta < 1.0 && e->bn == nullptr) {
        if (hipMalloc(&e->bn, (size_t)e->ncells * sizeof(double)) != hipSuccess) {
            e->bn = nullptr;
            return efail(TF_ENOMEM, "device allocation failed");
        }
    }
    e->S = *s;
    drop_graph(e);
    return TF_OK;
}

tf_status tf_ensemble_set_xsweep(tf_ensemble *e, int variant)
{
    if (e == nullptr) return efail(TF_EINVAL, "ensemble is NULL");
    if (variant != TF_XSWEEP_AUTO && variant != TF_XSWEEP_PARTITIONED && variant != TF_XSWEEP_ROW)
        return efail(TF_EINVAL, "unknown x-sweep variant");
    for (int f = 0; f < e->nfilms; ++f) {
        const tf::FilmDesc &d = e->desc[f];
        const bool row4 = tf::xrow_supported(d.nx) && d.nx <= tf::XR_ROW4_MAX_NX;
        e->xsweep[f] = variant == TF_XSWEEP_AUTO ? tf::xsweep_choice(d.nx, total_rows(e))
                     : (variant == TF_XSWEEP_ROW && row4 ? 1 : 0);
    }
    std::vector<int> items;
    build_items(e, items);
    TF_EHIP(hipStreamSynchronize(e->stream));
    TF_EHIP(hipMemcpyAsync(e->d_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice, e->stream));
    TF_EHIP(hipStreamSynchronize(e->stream));
    drop_graph(e);
    return TF_OK;
}

int tf_ensemble_xsweep(const tf_ensemble *e, int film)
{
    return (e == nullptr || film < 0 || film >= e->nfilms) ? -1 : e->xsweep[film];
}

tf_status tf_ensemble_set_model_linear(tf_ensemble *e, double c0, double c1)
{
    if (e == nullptr) return efail(TF_EINVAL, "ensemble is NULL");
    tf::Model M;
    std::string err;
    if (!tf_detail::linear_model(c0, c1, &M, &err)) return efail(TF_EINVAL, err);
    return set_all_models(e, M, tf::KM_LINEAR);
}

tf_status tf_ensemble_set_model_nlc(tf_ensemble *e, double C, double K, double N, double beta, double w, double b)
{
    if (e == nullptr) return efail(TF_EINVAL, "ensemble is NULL");
    tf::Model M;
    std::string err;
    if (!tf_detail::nlc_model(C, K, N, beta, w, b, &M, &err)) return efail(TF_EINVAL, err);
    return set_all_models(e, M, tf::KM_NLC);
}

tf_status tf_ensemble_set_model_polymer(tf_ensemble *e, double C, double Cst, double Aox, double Asi, double d)
{
    if (e == nullptr) return efail(TF_EINVAL, "ensemble is NULL");
    tf::Model M;
    std::string err;
    if (!tf_detail::polymer_model(C, Cst, Aox, Asi, d, &M, &err)) return efail(TF_EINVAL, err);
    return set_all_models(e, M, tf::KM_POLYMER);
}

tf_status tf_ensemble_bind(tf_ensemble *e, double *packed_dev)
{
    if (e == nullptr) return efail(TF_EINVAL, "ensemble is NULL");
    e->buf0 = packed_dev;
    drop_graph(e);
    std::memset(e->h_state, 0, e->nfilms * sizeof(tf::FilmState));
    TF_EHIP(hipMemcpyAsync(e->d_state, e->h_state, e->nfilms * sizeof(tf::FilmState), hipMemcpyHostToDevice,
                           e->stream));
    if (packed_dev != nullptr) TF_EHIP(tf::launch_ens_validate(e->d_desc, e->d_state, e->nfilms, e->buf0, e->stream));
    TF_EHIP(hipStreamSynchronize(e->stream));
    return TF_OK;
}

tf_status tf_ensemble_step(tf_ensemble *e, int nsteps, double *dt_per_film, int *status_per_film, int *iters_per_film)
{
    if (e == nullptr || dt_per_film == nullptr || nsteps < 0) return efail(TF_EINVAL, "bad argument");
    if (e->buf0 == nullptr) return efail(TF_ESTATE, "no packed state bound (tf_ensemble_bind)");
    for (int f = 0; f < e->nfilms; ++f)
        if (!(dt_per_film[f] > 0.0)) return efail(TF_EINVAL, "dt must be positive for every film");
    // order after the caller's stream
    hipEvent_t ev;
    TF_EHIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    TF_EHIP(hipEventRecord(ev, e->user));
    TF_EHIP(hipStreamWaitEvent(e->stream, ev, 0));
    (void)hipEventDestroy(ev);
    // load the per-film dt, clear iteration totals
    TF_EHIP(hipMemcpyAsync(e->h_state, e->d_state, e->nfilms * sizeof(tf::FilmState), hipMemcpyDeviceToHost,
                           e->stream));
    TF_EHIP(hipStreamSynchronize(e->stream));
    for (int f = 0; f < e->nfilms; ++f) {
        e->h_state[f].dt = dt_per_film[f];
        e->h_state[f].total = 0;
    }
    TF_EHIP(hipMemcpyAsync(e->d_state, e->h_state, e->nfilms * sizeof(tf::FilmState), hipMemcpyHostToDevice,
                           e->stream));
    tf_status st = ensure_graph(e);
    if (st != TF_OK) return st;
    for (int s = 0; s < nsteps; ++s) {
        TF_EHIP(tf::launch_ens_begin(e->d_state, e->nfilms, e->stream));
        int done = 0;
        int batch = std::max(1, std::min(e->prev_iters, 16));
        for (;;) {
            for (int b = 0; b < batch; ++b) TF_EHIP(hipGraphLaunch(e->exec, e->stream));
            done += batch;
            TF_EHIP(hipMemcpyAsync(e->h_active, e->d_active, sizeof(int), hipMemcpyDeviceToHost, e->stream));
            TF_EHIP(hipStreamSynchronize(e->stream));
            if (*e->h_active == 0) break;
            batch = 1;
        }
        e->prev_iters = done;
    }
    TF_EHIP(tf::launch_ens_commit(e->d_desc, e->d_state, e->nfilms, e->buf0, e->buf1, e->buf2, e->stream));
    TF_EHIP(hipMemcpyAsync(e->h_state, e->d_state, e->nfilms * sizeof(tf::FilmState), hipMemcpyDeviceToHost,
                           e->stream));
    TF_EHIP(hipStreamSynchronize(e->stream));
    tf_status result = TF_OK;
    for (int f = 0; f < e->nfilms; ++f) {
        dt_per_film[f] = e->h_state[f].dt;
        if (status_per_film) status_per_film[f] = e->h_state[f].status;
        if (iters_per_film) iters_per_film[f] = e->h_state[f].total;
        if (result == TF_OK && e->h_state[f].status != 0) result = e->h_state[f].status;
    }
    if (result != TF_OK) return efail(result, "at least one film failed (see status_per_film)");
    return TF_OK;
}

tf_status tf_ensemble_film_info(const tf_ensemble *e, int film, tf_step_info *info)
{
    if (e == nullptr || info == nullptr || film < 0 || film >= e->nfilms) return efail(TF_EINVAL, "bad argument");
    const tf::FilmState &s = e->h_state[film];
    std::memset(info, 0, sizeof(*info));
    info->t = s.t;
    info->dt_used = s.dt_used;
    info->e_final = s.e_last;
    info->r_final = s.r_last;
    info->newton_iters = s.newton;
    info->rejections = s.rejections;
    info->status = s.status;
    info->total_iters = s.total;
    return TF_OK;
}

} // extern "C"
