// Host-side bounds check of the kernels' geometry: the segment partition of a line, the
// sub-segments of a tile, the even reflection of ghost indices, the workgroup -> tile map,
// the y-sweep column tiles, the LDS layout and staging indices of the tile passes, and the
// geometry of the whole-row sweep and whole-line solver (lane sub-segments, padding, LDS
// regions, staging coverage, tree slots). The functions checked are the ones the kernels
// call (tf_internal.h, host and device); the tile-pass staging loops are restated from
// stage_tile. Exhaustive over line lengths; prints "geometry check: ok" or the first failure.
#include "../paper_1806_10550_amd/csrc/tf_internal.h"

#include <cstdio>
#include <cstdlib>
#include <vector>

using namespace tf;

static int failures = 0;
#define CHECK(cond, ...)                                                                    \
    do {                                                                                    \
        if (!(cond)) {                                                                      \
            if (failures++ < 20) {                                                          \
                std::printf("FAIL %s:%d: %s: ", __FILE__, __LINE__, #cond);                 \
                std::printf(__VA_ARGS__);                                                   \
                std::printf("\n");                                                          \
            }                                                                               \
        }                                                                                   \
    } while (0)

// segments of a line and the sub-segments of each tile (tile_body: nsub = min(NSUB, npos/2))
static void check_segments()
{
    for (int n = 2; n <= 20000; ++n) {
        const int P = seg_count(n);
        CHECK(seg_start(0, n) == 0 && seg_start(P, n) == n, "n=%d", n);
        for (int q = 0; q < P; ++q) {
            const int len = seg_start(q + 1, n) - seg_start(q, n);
            CHECK(len >= 2 && len <= TILE, "n=%d q=%d len=%d", n, q, len);
        }
    }
    for (int npos = 2; npos <= TILE; ++npos) {
        const int nsub = npos / 2 < NSUB ? npos / 2 : NSUB;
        int covered = 0;
        for (int wave = 0; wave < NSUB; ++wave) {
            const int ps = (wave * npos) / nsub;
            const int len = wave < nsub ? ((wave + 1) * npos) / nsub - ps : 0;
            if (wave < nsub) {
                CHECK(ps == covered, "npos=%d wave=%d", npos, wave);
                CHECK(len >= 2 && len <= SUB, "npos=%d wave=%d len=%d", npos, wave, len);
            }
            covered += len;
        }
        CHECK(covered == npos, "npos=%d covered=%d", npos, covered);
    }
}

// ghost indices: the even reflection for one layer beyond each end, clamped beyond that
static void check_reflection()
{
    for (int n = 1; n <= 300; ++n)
        for (int k = -TILE - 8; k <= n + TILE + 8; ++k) {
            const int r = crefl(k, n);
            CHECK(r >= 0 && r < n, "k=%d n=%d r=%d", k, n, r);
            if (k >= -n && k < 2 * n) {
                const int e = k < 0 ? -1 - k : (k >= n ? 2 * n - 1 - k : k);
                CHECK(r == e, "k=%d n=%d r=%d e=%d", k, n, r, e);
            }
        }
}

// workgroup -> tile: a bijection of [0, n) that gives each XCD (b mod 8) a contiguous run
static void check_xcd_map()
{
    for (int n = 1; n <= 5000; ++n) {
        std::vector<int> seen(n, 0);
        for (int b = 0; b < n; ++b) {
            const int t = xcd_tile(b, n);
            CHECK(t >= 0 && t < n, "b=%d n=%d t=%d", b, n, t);
            if (t >= 0 && t < n) seen[t]++;
        }
        for (int t = 0; t < n; ++t) CHECK(seen[t] == 1, "n=%d tile %d hit %d times", n, t, seen[t]);
        for (int b = 8; b < n; ++b) CHECK(xcd_tile(b, n) == xcd_tile(b - 8, n) + 1, "n=%d b=%d", n, b);
    }
}

// y-sweep tiles own TILE columns, one per lane: every grid column exactly once
static void check_column_tiles()
{
    for (int nx = 4; nx <= 5000; ++nx) {
        const int tiles = (nx + TILE - 1) / TILE;
        int covered = 0;
        for (int tx = 0; tx < tiles; ++tx) {
            const int x0 = tx * TILE, x1 = x0 + TILE < nx ? x0 + TILE : nx;
            CHECK(x0 == covered && x1 > x0, "nx=%d tx=%d", nx, tx);
            covered = x1;
            CHECK(x1 - x0 <= 64, "nx=%d tx=%d owned=%d", nx, tx, x1 - x0);
        }
        CHECK(covered == nx, "nx=%d", nx);
    }
}

// LDS indices of the tile staging (stage_tile): u tile rows RU0.. and its extra columns,
// the second input tile; every index inside its region, every cell the sweeps read staged
static void check_tile_staging()
{
    const int NU = TW * UPITCH, NW = TILE * WPITCH;
    for (int dir = 0; dir < 2; ++dir) {
        const int LX0 = HALO, RU0 = dir == 0 ? 0 : 1, NRU = dir == 0 ? TW : TW - 2;
        const int KU = (NRU + NSUB - 1) / NSUB, KB = TILE / NSUB, XPR = 2 * HALO;
        const int NX = NRU * XPR, KX = (NX + BLOCK - 1) / BLOCK;
        std::vector<int> hit(NU, 0);
        for (int wave = 0; wave < NSUB; ++wave)
            for (int lane = 0; lane < 64; ++lane) {
                for (int k = 0; k < KU; ++k) {
                    const int ly = RU0 + wave + NSUB * k;
                    if (ly < RU0 + NRU) {
                        const int i = ly * UPITCH + LX0 + lane;
                        CHECK(i >= 0 && i < NU, "dir=%d u index %d", dir, i);
                        if (i >= 0 && i < NU) hit[i]++;
                    }
                }
                for (int k = 0; k < KB; ++k) {
                    const int i = (wave + NSUB * k) * WPITCH + lane;
                    CHECK(i >= 0 && i < NW, "dir=%d b index %d", dir, i);
                }
                for (int k = 0; k < KX; ++k) {
                    const int idx = (wave + NSUB * k) * 64 + lane;
                    if (idx < NX) {
                        const int ly = RU0 + idx / XPR, q = idx % XPR;
                        const int lx = q < HALO ? q : TILE + q;
                        const int i = ly * UPITCH + lx;
                        CHECK(lx < TW && i >= 0 && i < NU, "dir=%d extra index %d", dir, i);
                        if (i >= 0 && i < NU) hit[i]++;
                    }
                }
            }
        // the cells the sweeps read, each staged exactly once: the cell quantities of (line l,
        // position q) read u at (l, q), (l +- 1, q) and (l, q +- 1); the sweeps form them for
        // every lane at positions -1..TILE, the y sweep's edge record for the lines -1, 0,
        // TILE-1 and TILE at positions 0..TILE-1
        std::vector<int> need(NU, 0);
        auto at = [&](int l, int q) {
            const int i = dir == 0 ? (q + HALO) * UPITCH + (l + HALO) : (l + HALO) * UPITCH + (q + HALO);
            CHECK(i >= 0 && i < NU, "dir=%d read (%d,%d) outside the tile", dir, l, q);
            if (i >= 0 && i < NU) need[i] = 1;
        };
        auto cell = [&](int l, int q) { at(l, q); at(l - 1, q); at(l + 1, q); at(l, q - 1); at(l, q + 1); };
        for (int l = 0; l < TILE; ++l)
            for (int q = -1; q <= TILE; ++q) cell(l, q);
        if (dir == 0)
            for (int q = 0; q < TILE; ++q) { cell(-1, q); cell(0, q); cell(TILE - 1, q); cell(TILE, q); }
        for (int i = 0; i < NU; ++i)
            if (need[i]) CHECK(hit[i] == 1, "dir=%d cell (%d,%d) staged %d times", dir, i / UPITCH, i % UPITCH, hit[i]);
    }
}

// whole-row sweep / whole-line solver: lanes cover the row (lane 0 may start up to
// XR_CPL-1 padding positions early), every LDS index inside its region, the staging loop
// covers the row and its ghosts, and every tree merge and split names two slots of the row
static void check_rows()
{
    for (int nx = 4; nx <= XR_MAX_NX; ++nx) {
        const XRowGeom g = xrow_geom(nx);
        CHECK(g.S * XR_CPL >= nx && (g.S - 1) * XR_CPL < nx, "nx=%d S=%d", nx, g.S);
        CHECK(g.W * 64 >= g.S && g.W <= g.waves && (g.waves == 4 || g.waves == XR_WAVES), "nx=%d", nx);
        CHECK(g.R >= 1 && g.R * g.W <= g.waves, "nx=%d R=%d W=%d", nx, g.R, g.W);
        const bool fits = g.R * (g.pu + g.p2) <= xr_lds(g.waves);
        CHECK(fits, "nx=%d LDS %d > %d", nx, g.R * (g.pu + g.p2), xr_lds(g.waves));
        const int p0_lane0 = nx - XR_CPL * g.S;
        CHECK(p0_lane0 <= 0 && p0_lane0 > -XR_CPL, "nx=%d p0=%d", nx, p0_lane0);
        const int W16 = XR_CPL * g.S, sh = W16 - nx;
        // staging: thread i of the row group stages w = i - 2 (u row, -2 .. 16 S + 1) and
        // w = i - 1 (neighbour rows, -1 .. 16 S) over XR_STAGE rounds of 64 W threads
        CHECK(64 * g.W * XR_STAGE >= W16 + 4, "nx=%d staging covers %d", nx, 64 * g.W * XR_STAGE);
        CHECK(xr_at(-2) == 0 && xr_at(W16 + 1) < g.pu, "nx=%d u row", nx);
        CHECK(xr_at(-1) >= 0 && xr_at(W16) < g.p2, "nx=%d neighbour rows", nx);
        CHECK(NREL * g.S <= g.p2, "nx=%d records", nx);                    // record tree
        {
            // staged positions map to distinct slots; staged cells reflect into the row
            std::vector<int> seen(g.pu, 0);
            for (int w = -2; w <= W16 + 1; ++w) {
                const int a = xr_at(w);
                if (a >= 0 && a < g.pu) seen[a]++;
                const int q = w - sh < -2 ? -2 : w - sh, c = crefl(q, nx);
                CHECK(c >= 0 && c < nx, "nx=%d w=%d reflects to %d", nx, w, c);
            }
            for (int a = 0; a < g.pu; ++a) CHECK(seen[a] <= 1, "nx=%d slot %d staged %d times", nx, a, seen[a]);
        }
        // a lane's accesses: cells at relative positions t = -1 .. 16 read t - 1 .. t + 1 of the
        // u row and t of the neighbour rows, at constant offsets of its block; parked factors and
        // the solution use t = 0 .. 15
        for (int s = 0; s < g.S; ++s)
            for (int t = -2; t <= XR_CPL + 1; ++t) {
                const int a = xr_base(s) + xr_off(t);
                CHECK(a == xr_at(XR_CPL * s + t), "nx=%d s=%d t=%d offset", nx, s, t);
                CHECK(a >= 0 && a < g.pu, "nx=%d s=%d t=%d u row index %d", nx, s, t, a);
                if (t >= -1 && t <= XR_CPL) CHECK(a < g.p2, "nx=%d s=%d t=%d neighbour index %d", nx, s, t, a);
            }
        // the output loop reads position i < nx at xr_at(i + sh), inside the lanes' blocks
        CHECK(xr_at(sh) >= xr_base(0) && xr_at(nx - 1 + sh) < xr_base(g.S - 1) + XR_CPL, "nx=%d output", nx);
        int levels = 0;
        while ((1 << levels) < g.S) ++levels;
        for (int l = 1; l <= levels; ++l) {
            const int half = 1 << (l - 1);
            const int nm = (g.S - half + 2 * half - 1) / (2 * half);
            for (int b = 0; b < nm; ++b) {
                const int a = b * 2 * half, c = a + half;
                CHECK(a >= 0 && c < g.S, "nx=%d level %d merge %d: slots %d %d", nx, l, b, a, c);
            }
            // no pair of neighbouring blocks is left unmerged at this level
            CHECK(nm * 2 * half + half >= g.S, "nx=%d level %d nm=%d", nx, l, nm);
        }
        const int mx = g.waves * 64; // threads of the largest workgroup
        CHECK(64 * g.W * g.R <= mx, "nx=%d block", nx);
    }
}

int main()
{
    check_segments();
    check_reflection();
    check_xcd_map();
    check_column_tiles();
    check_tile_staging();
    check_rows();
    if (failures) {
        std::printf("geometry check: %d failures\n", failures);
        return 1;
    }
    std::printf("geometry check: ok\n");
    return 0;
}
