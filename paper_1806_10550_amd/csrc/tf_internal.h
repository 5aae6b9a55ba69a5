// Internal declarations shared by the HIP kernels (tf_kernels.hip) and the host
// runtime (tf_api.hip) of libthinfilm. Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>

namespace tf {

// Geometry of the partitioned line solver.
//   A line (a grid column for the y sweep, a grid row for the x sweep) is cut into
//   segments of TILE cells; 64 neighbouring lines times one segment form a tile that
//   one workgroup owns. Inside a tile each of the NSUB waves eliminates a
//   sub-segment of at most SUB cells for all 64 lines (one line per lane).
constexpr int TILE = 64;
constexpr int NSUB = 4;
constexpr int SUB = TILE / NSUB;
constexpr int HALO = 2;
constexpr int TW = TILE + 2 * HALO;      // haloed tile width (68)
constexpr int UPITCH = TW + 1;           // LDS row pitch of the haloed u tile (odd: no bank conflicts)
constexpr int WPITCH = TILE + 1;         // LDS row pitch of the second input tile
constexpr int NREL = 20;                 // doubles per (segment, line) relation record
constexpr int NEXT = 4;                  // doubles per (segment, line) boundary record
constexpr int NCHAIN = 12;               // doubles per (segment, line) chain record
constexpr int BLOCK = 64 * NSUB;

// Whole-row x sweep (tf_xrow.hip): each lane eliminates XR_CPL consecutive cells of a row;
// a workgroup of 4 or 8 waves holds one row (of up to XR_MAX_NX cells) or several shorter
// rows, in xr_lds(waves) doubles of LDS: 4-wave workgroups (rows up to 4096 cells) fit two
// to a CU, so that one's memory phases overlap the other's arithmetic.
constexpr int XR_CPL = 16;
constexpr int XR_WAVES = 8;                          // waves of the largest workgroup
constexpr int XR_MAX_NX = XR_CPL * 64 * XR_WAVES;
__host__ __device__ constexpr int xr_lds(int waves) { return waves * 2400; }
constexpr int XR_ROW4_MAX_NX = XR_CPL * 64 * 4;      // rows a 4-wave workgroup holds

// Geometry of the whole-row sweep and of the whole-line solver (host and device).
// A row of nx cells is held by S = ceil(nx / 16) lanes; lane s owns the 16 positions
// q = nx - 16 (S - s) + k, k < 16 (lane 0 may start before the row). Staged rows number
// their positions w = q + 16 S - nx = 16 s + k from lane 0's first one (w >= -2 covers the two
// cells before it) and store them at xr_at(w): one padding double every 16, so that lanes
// reading their cells in step (stride 17 doubles) hit distinct banks, and lane s's block
// starts at 17 s + 3, so that a lane's accesses sit at constant offsets xr_off(t) of its
// block (t = k + d, -2 <= t).
__host__ __device__ inline int xr_at(int w) { return w + 3 + (w >> 4); }
__host__ __device__ constexpr int xr_off(int t) { return t + (t >> 4); }
__host__ __device__ inline int xr_base(int s) { return 17 * s + 3; }

// Geometry of one launch (host computed, identical for every row of the grid).
struct XRowGeom {
    int S;        // sub-segments (lanes) per row
    int W;        // waves per row
    int R;        // rows per workgroup
    int pu, p2;   // LDS doubles per row: staged u row; X row / tree / output staging
    int waves;    // waves per workgroup (4 or 8)
};

// Staging loads per thread: 16 S + 4 <= 64 W XR_CPL + 4 cells over 64 W threads.
constexpr int XR_STAGE = XR_CPL + 1;

__host__ __device__ inline XRowGeom xrow_geom(int nx)
{
    XRowGeom g{};
    g.S = (nx + XR_CPL - 1) / XR_CPL;
    g.W = (g.S + 63) / 64;
    g.pu = xr_at(XR_CPL * g.S + 1) + 1;                // u row: w = -2 .. 16 S + 1
    const int px = xr_at(XR_CPL * g.S) + 1, pt = NREL * g.S; // u(j-1) + u(j+1): w = -1 .. 16 S
    g.p2 = px > pt ? px : pt;
    g.waves = g.W <= 4 ? 4 : XR_WAVES;
    g.R = g.waves / g.W;
    if (g.R < 1) g.R = 1;
    while (g.R > 1 && g.R * (g.pu + g.p2) > xr_lds(g.waves)) --g.R;
    return g;
}

// Segments of a line of n >= 2 cells: TILE cells each, except that a last segment of
// a single cell borrows one from its neighbour (every segment has >= 2 cells).
__host__ __device__ inline int seg_count(int n) { return (n + TILE - 1) / TILE; }
__host__ __device__ inline int seg_start(int q, int n)
{
    const int P = seg_count(n);
    if (q >= P) return n;
    int s = q * TILE;
    if (q == P - 1 && P > 1 && n - s < 2) s -= 1;
    return s;
}

// Even reflection across the boundary faces (no-flux ghosts), clamped so that a
// ragged tile never reads outside the grid.
__host__ __device__ __forceinline__ int crefl(int k, int n)
{
    if (k < 0) k = -1 - k;
    if (k >= n) k = 2 * n - 1 - k;
    return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous run
// of tiles so that neighbouring tiles share halos in the same L2.
__host__ __device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Thin-film models (eq. GeneralDisPreForm): f0 = cap h^3, f1 = h^3 Pi'(h).
// MODEL_POWER: Pi = kappa f(h), f = (b/h)^n - (b/h)^m with integer n, m, cap = 1; in terms
//   of r = 1/h:
//     f1  = Cm r^(m-2) - Cn r^(n-2),  Cm = kappa m b^m, Cn = kappa n b^n
//     f1' = Dn r^(n-1) - Dm r^(m-1),  Dn = kappa n (n-2) b^n, Dm = kappa m (m-2) b^m
// MODEL_LINEAR: the linear test model f0 = c0, f1 = c1 (Sec. "Thin Film Models"); c0 is held
//   in cap, c1 in Cm.
// MODEL_NLC: Pi = K[(b/h)^3 - (b/h)^2] + N/2 (m(h)/h)^2, m(h) = g(h) h^2/(h^2 + beta^2),
//   g = (1 + tanh((h - 2b)/w))/2 (eqs. DisjPressNLC, mh_model).
// MODEL_POLYMER: Pi = -psi', psi = Cst h^-8 - Aox/(12 pi h^2) + (Aox - Asi)/(12 pi (h+d)^2)
//   (eq. DisjPressPolymer), stored as Pi = C8 h^-9 - a2 h^-3 + c2 (h+d)^-3.
enum ModelKind { MODEL_POWER = 0, MODEL_LINEAR = 1, MODEL_NLC = 2, MODEL_POLYMER = 3 };
// Model form compiled into the sweep kernels (one instantiation each): the power law with
// n = 3, m = 2, any other power law, the linear model, NLC, polymer.
enum KernelModel { KM_P32 = 0, KM_POWER = 1, KM_LINEAR = 2, KM_NLC = 3, KM_POLYMER = 4 };
struct Model {
    double kappa, b;
    int n, m;
    double Cn, Cm, Dn, Dm;
    bool p32; // power law with n == 3 && m == 2: f1 = Cm - Cn r, f1' = Dn r^2
    int kind;
    double cap;                // C in f0 = C h^3 (c0 of the linear model)
    double K, N, beta2, w, iw; // NLC (with b); iw = 1/w
    double C8, a2, c2, d;      // polymer
};

// Parameters of one sweep pass (K1 relations / K3 solve) over a grid or a packed film.
struct PassParams {
    int nx, ny;
    double ids2;        // 1/ds^2
    double f0s;         // cap / ds^2 (scale of h^3 in the cell's f0; the linear model's f0 / ds^2)
    double ka;          // c / (2 ds^2) with c = theta dt
    double K0, K1;      // 3 ka cap / ds^2 (scale of h^2 in g0) and ka Dn (of r^2 in g1, n=3, m=2)
    Model M;
    const double *u;    // u_k
    const double *in2;  // y sweep: b^n (= u^n for backward Euler); x sweep: w
    double *out;        // y sweep: w; x sweep: u_{k+1}
    double *rel;        // [P][NREL][nlines]
    const double *ext;  // [P][NEXT][nlines]
    unsigned long long *res;        // reduction slot: res_spread records {emax, rmax, flags, ...}
    unsigned long long *res_clear;  // slot zeroed by block 0 (may be null)
    int res_spread;                 // copies of the reduction record in a slot (>= 1)
    int tiles_x, tiles_y;
    // x solve only, nullable: per tile (ty * tiles_x + tx) the compensated sum {s, c} and the
    // minimum of the u_{k+1} cells it writes (the mass diagnostic of the iterate, 4 doubles)
    double *mass;
};

struct ChainParams {
    int nlines, P;
    const double *rel;
    double *chain;
    double *ext;
};

enum ResultWord { RES_EMAX = 0, RES_RMAX = 1, RES_FLAGS = 2, RES_WORDS = 8 };
constexpr int ENS_RES_SPREAD = 16;    // copies of each film's reduction record in the ensemble
// A grid's reduction record is spread over RES_SPREAD copies (workgroup b updates copy
// b % RES_SPREAD) so that the atomics of thousands of workgroups do not all meet at
// one address; the host combines the copies.
constexpr int RES_SPREAD = 64;

// ---- ensemble of films packed in one buffer --------------------------------------------
struct FilmDesc {          // constant per film
    int nx, ny, Px, Py;
    double ds;
    Model M;
    long long off;         // first cell of the film in the packed field buffers
    long long roff;        // first (segment, line) record of the film in the interface scratch
};

struct FilmState {         // per-film Newton / time-step state, updated on the device
    double dt, t, dt_used, e_last, r_last;
    int k, cur, it, nxt;   // iteration in the attempt; buffer index of u^n, u_k, u_{k+1} (0,1,2)
    int active, status, successes, rejections, newton, total;
    // reduction words of the current iteration: ENS_RES_SPREAD copies of RES_WORDS words
    // (RES_EMAX..), so that the waves of a large film do not all update one address
    unsigned long long red[ENS_RES_SPREAD * RES_WORDS];
};

struct EnsScheme {
    double theta, tol, dt_min, dt_max, dt_shrink, dt_grow;
    int max_newton, grow_after, adaptive;
};

struct EnsParams {
    const FilmDesc *desc;
    FilmState *state;
    const int *items;      // tiles: (film, tx, ty); chain blocks: (film, line block)
    int nitems;
    double *buf0, *buf1, *buf2; // packed u buffers; index 0 is the caller's state
    double *w, *rel, *ext, *chain;
    double *bn;            // packed b^n = u^n - (1 - theta) dt D(u^n) (theta < 1 only)
    double theta;
};
enum ResultFlag { FLAG_NONPOS = 1, FLAG_NAN = 2 };

// Launchers (tf_kernels.hip). Each returns the launch status.
// out = D(u) evaluated with f0 = 0 (the f1 part only; with kappa = 1 this is dD/dkappa)
hipError_t launch_flux_divergence_f1(int nx, int ny, double ids, double ids2, const Model &M, const double *u,
                                     double *out, hipStream_t s);
hipError_t launch_pass(int dir, bool solve, const PassParams &p, hipStream_t s);
// Whole-row x sweep: reads u (u_k) and in2 (w), writes out (u_{k+1}), the reduction record
// (res: max|v/u_k|, flags) and, when mass is set, one mass record per workgroup.
bool xrow_supported(int nx);
int xrow_blocks(int nx, int ny);           // workgroups of one launch (= mass records)
hipError_t launch_xrow(const PassParams &p, hipStream_t s);
// Stored-band solves of whole lines (4 ..= XR_ROW4_MAX_NX cells) in one kernel: pm true
// position-major (plain or transposed; mode 0 out = x, mode 1 out += x with the maxima in
// red[0..1]), pm false line-major (transposed, mode 0 only). stop (nullable): a device word;
// when it is nonzero as the kernel starts, the kernel does nothing.
bool sbline_supported(int np);
hipError_t launch_sbline(bool trans, bool pm, int mode, int nl, int np, const double *bands, const double *rhs,
                         double *out, unsigned long long *red, hipStream_t s,
                         const unsigned long long *stop = nullptr);
// x-sweep variant for a film of nx x ny cells (0: partitioned, 1: whole-row): the autotuned
// choice for the nearest shape, else the built-in rule (tf_adjoint.hip).
int xsweep_choice(int nx, int ny);
// Whole-row x sweep over the ensemble's row films (items: (film, row block); every such film
// has nx <= XR_ROW4_MAX_NX); km: the KernelModel every film shares.
hipError_t launch_xrow_ens(int km, const EnsParams &e, hipStream_t s);
hipError_t launch_model_coeffs(const Model &M, const double *h, int n, double *out, hipStream_t s);
hipError_t launch_chain(const ChainParams &c, hipStream_t s);
hipError_t launch_flux_divergence(int nx, int ny, double ids, double ids2, const Model &M,
                                  const double *u, double alpha, double beta, const double *add,
                                  double *out, hipStream_t s);
hipError_t launch_mass(const double *u, size_t n, double *partials, int nblocks, hipStream_t s);
// Combine ntiles per-tile mass records {s, c, min, -} (PassParams::mass) in a fixed order into
// out = {sum, min}.
hipError_t launch_mass_tiles(const double *part, int ntiles, double *out, hipStream_t s);
hipError_t launch_pass_ens(int dir, bool solve, int km, const EnsParams &e, hipStream_t s);
// b^n of every active film at the first iteration of an attempt (items: the y-sweep tiles)
hipError_t launch_bn_ens(const EnsParams &e, hipStream_t s);
hipError_t launch_chain_ens(const EnsParams &e, int dir, hipStream_t s);
hipError_t launch_ens_control(FilmState *st, int nfilms, const EnsScheme &S, int *active_count, hipStream_t s);
hipError_t launch_ens_begin(FilmState *st, int nfilms, hipStream_t s);
hipError_t launch_ens_commit(const FilmDesc *desc, FilmState *st, int nfilms, double *buf0, double *buf1,
                             double *buf2, hipStream_t s);
hipError_t launch_ens_validate(const FilmDesc *desc, FilmState *st, int nfilms, const double *buf0, hipStream_t s);
int mass_blocks(size_t n);

} // namespace tf

struct tf_grid;
namespace tf_detail {
struct GridView {
    int nx, ny;
    double ds, theta;
    tf::Model M;
    hipStream_t stream;
    double *rel, *ext, *chain;
    int xsweep;               // x-sweep variant (TF_XSWEEP_PARTITIONED / TF_XSWEEP_ROW)
};
bool grid_view(const tf_grid *g, GridView *v);   // false if the model is not set
void release_adjoint(const tf_grid *g);           // frees adjoint scratch of a grid
void set_error(const std::string &msg);
bool linear_model(double c0, double c1, tf::Model *M, std::string *err);
bool nlc_model(double C, double K, double N, double beta, double w, double b, tf::Model *M, std::string *err);
bool polymer_model(double C, double Cst, double Aox, double Asi, double d, tf::Model *M, std::string *err);
} // namespace tf_detail
