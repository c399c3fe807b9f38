// Host runtime of the MI355X pressure solver: arena allocator, slot table,
// hipGraph capture of the iteration, polling, and the C ABI of pcg.h.
//
// One Engine drives any number of resident solves ("slots").  Device memory
// comes from a caller-owned arena: a fixed head (batch header, slot table,
// slot states, error flag) followed by one block per slot carved by a
// first-fit allocator.  The iteration is captured once as a hipGraph of
// check_every x [K1, K2] launches that read the slot table from device
// memory, so slots can join and leave between replays without re-capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "pcg.h"
#include "pcg_types.h"

namespace pcgmi {
hipError_t launch_iter(int family, int which, int mode, int grid,
                       const BatchHeader *hdr, const Slot *slots, hipStream_t s);
hipError_t launch_classify(const double *r64, uint8_t *cls, int64_t n, int round,
                           unsigned long long *words, hipStream_t s);
hipError_t launch_encode(const double *rho, const uint8_t *mask, double *r64,
                         float *r32, int64_t n, int *bad, hipStream_t s);
hipError_t launch_copy(const double *src, double *dst, size_t n, hipStream_t s);
hipError_t launch_pack_mask(const uint8_t *mask, uint32_t *bits, int nx,
                            int words_per_row, int64_t nwords, hipStream_t s);
hipError_t launch_triad(double *a, const double *b, const double *c, double sc, size_t n,
                        hipStream_t s);
hipError_t launch_check_frac(const double *ax, const double *ay, const double *az,
                             const double *vol, const double *rho64, int64_t nu, int64_t nv,
                             int64_t nw, int64_t n, int *bad, hipStream_t s);
hipError_t launch_project(const Slot *slot, const double *p, double s, double wt,
                          const double *const a[3], const double *const b[3],
                          double *const out[3], int blocks, hipStream_t st);
hipError_t launch_rhs(const Slot *slot, double h, double dt, const double *const a[3],
                      const double *const b[3], double *rhs, int blocks, hipStream_t st);
hipError_t launch_divnorm(const Slot *slot, double inv_h, const double *u,
                          const double *v, const double *w, double *part, int blocks,
                          hipStream_t st);
hipError_t static_scratch(void **ptr, size_t *bytes);
}  // namespace pcgmi

using namespace pcgmi;

namespace {

thread_local std::string g_hip_err;

int hip_fail(hipError_t e, const char *what)
{
    g_hip_err = std::string(what) + ": " + hipGetErrorString(e);
    return PCG_EHIP;
}

#define HIP_TRY(expr)                                      \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return hip_fail(_e, #expr);  \
    } while (0)

// Average ms of `reps` launches after one untimed launch, on stream s.
template <class F>
int time_launches(hipStream_t s, int32_t reps, F &&launch, double *ms_out)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "timed probe launches");
    *ms_out = ms / reps;
    return PCG_OK;
}

constexpr size_t kAlign = 256;
constexpr int kDefaultCheckEvery = 32;
constexpr int kDefaultGridMax = 1024;
constexpr int kBatchGrid = 512;
constexpr double kDefaultInnerTol = 1e-4;
// largest byte span pass A addresses within one tile (32-bit offsets)
constexpr int64_t kMaxTileBytes = 0xffffffffll;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// ---- tile shape table (autotuned values can be installed at run time) ----

struct TileRule {
    int64_t max_cells;  // rule applies to grids with at most this many cells
    int tz;             // planes per tile
    int grid;           // workgroups for a single-solve context (0 = default)
};

// Built-in table: the autotuner's choice on gfx950 (package tile_table.json).
std::vector<TileRule> g_rules[2] = {  // single solves: FP64, FP32+IR
    { { 7524, 2, 256 }, { 21283, 2, 256 }, { 60198, 4, 1024 }, { 170267, 4, 768 }, { 481589, 8, 1024 }, { 1362140, 16, 2048 }, { 3852714, 16, 768 }, { 10897121, 64, 512 }, { 30821713, 128, 768 }, { 87176971, 32, 512 }, { INT64_MAX, 256, 512 } },
    { { 7524, 2, 256 }, { 21283, 2, 1024 }, { 60198, 2, 2048 }, { 170267, 4, 768 }, { 481589, 4, 1024 }, { 1362140, 8, 256 }, { 3852714, 16, 256 }, { 10897121, 32, 768 }, { 30821713, 32, 768 }, { 87176971, 16, 512 }, { INT64_MAX, 256, 1024 } },
};

// Batches: longer tiles (the resident solves fill the device together).
std::vector<TileRule> g_rules_batch[2] = {
    { { 7524, 8, 0 }, { 21283, 16, 0 }, { 60198, 16, 0 }, { 170267, 32, 0 }, { 481589, 32, 0 }, { 1362140, 32, 0 }, { 3852714, 16, 0 }, { INT64_MAX, 64, 0 } },
    { { 7524, 8, 0 }, { 21283, 8, 0 }, { 60198, 8, 0 }, { 170267, 16, 0 }, { 481589, 16, 0 }, { 1362140, 16, 0 }, { 3852714, 16, 0 }, { INT64_MAX, 32, 0 } },
};

// Single solves on 2-D plane tiles (their own optimum: a tile also runs the
// plane below it in the one-sweep form, and its plane holds 512 cells).
std::vector<TileRule> g_rules_plane[2] = {
    { { 681070, 4, 1024 }, { 1362140, 8, 768 }, { 3852714, 16, 1024 }, { 7705428, 48, 1024 }, { 11863283, 32, 1024 }, { 30821713, 64, 1024 }, { 87176971, 24, 512 }, { INT64_MAX, 256, 512 } },
    { { 1048576, 4, 768 }, { 3852714, 8, 1024 }, { 10897121, 24, 1024 }, { 23726566, 32, 512 }, { 67108864, 64, 512 }, { INT64_MAX, 256, 768 } },
};

// Single solves on narrow plane tiles (64 x 4, one cell a thread): the
// autotuner's choice on odd-row grids, longer tiles than the wide ones at
// the same size (a narrow plane holds half the cells of a wide FP64 one and
// a quarter of a wide FP32 one).
std::vector<TileRule> g_rules_narrow[2] = {
    { { 99343, 4, 512 }, { 516205, 8, 512 }, { 1409802, 24, 1024 }, { 1989340, 16, 1024 }, { 3669049, 24, 1024 }, { 10748808, 64, 1024 }, { 30521679, 128, 512 }, { INT64_MAX, 64, 512 } },
    { { 99343, 4, 1024 }, { 516205, 8, 768 }, { 1409802, 16, 1024 }, { 1989340, 16, 1024 }, { 3669049, 24, 1024 }, { 10748808, 64, 512 }, { 30521679, 128, 1024 }, { INT64_MAX, 48, 512 } },
};

// Table kinds: 0 single solves, 1 batches, 2 single solves on plane tiles,
// 3 single solves on narrow plane tiles.
enum { kTableSingle = 0, kTableBatch = 1, kTablePlane = 2, kTableNarrow = 3 };

std::vector<TileRule> &rules_of(int prec, int table)
{
    std::vector<TileRule> *t = table == kTableBatch    ? g_rules_batch
                               : table == kTablePlane  ? g_rules_plane
                               : table == kTableNarrow ? g_rules_narrow
                                                       : g_rules;
    return t[prec == PCG_PREC_FP32_IR ? 1 : 0];
}

// Batches use the batch table whatever their tile form; single solves the
// table of theirs (group: 0 consecutive cells, 1 narrow, else wide plane
// tiles).
const TileRule &rule_for(int64_t n, int prec, bool batch, int group)
{
    const int table = batch ? kTableBatch
                      : group == 1 ? kTableNarrow
                      : group > 1 ? kTablePlane : kTableSingle;
    const auto &rules = rules_of(prec, table);
    for (const auto &r : rules)
        if (n <= r.max_cells) return r;
    return rules.back();
}

// ---- first-fit allocator over [0, size) ----

class Arena {
public:
    void reset(size_t base, size_t size)
    {
        free_.clear();
        if (size > base) free_[base] = size - base;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(bytes, kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes, kAlign);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

private:
    std::map<size_t, size_t> free_;
};

struct Geometry {
    int nx, ny, nz, tz, plane_tiles, ztiles, cpt;
    int tx, ty, tiles_x;    // 2-D plane tiles (tx > 0) or consecutive cells
    int64_t n, ntiles;
};

// Whether a grid runs 2-D plane tiles (the LDS-staged sweep): no cut-cell
// fractions, not switched off, rows of whole groups (an even length for
// FP64, a multiple of four for FP32), and rows that hold whole tiles (128
// cells for FP64, two per thread; 256 for FP32, four) or, in single-solve
// contexts with walls on x, keep enough of their tiles' lanes busy
// (PCG_PLANE_TILES takes any share, also in batches); a periodic y axis
// holds whole tile rows.  With the walls unknown (bc null: workspace
// sizing) the periodic conditions are taken as met, which sizes for the
// larger tile count.
// They are taken on every grid that allows them: with one sweep per
// iteration they measured faster than the consecutive-cell tiles on every
// grid of whole tiles tried (FP64 per iteration: 128^3 45 against 61 us,
// 256^3 187 against 239, the 512 x 128 x 128 strut 113 against 137, 384^3
// 555 against 761, 512^3 1167 against 1650; FP32 inner iterations: 256^3
// 117 against 159, 512^3 643 against 864).  On rows of nx x 256 x 256
// grids that leave the last tile partly empty, FP64 per iteration: nx 192
// (three quarters of the lanes busy) 169 against 221 us, 224 175 against
// 230, 320 311 against 361, but 160 (five eighths) 215 against 197 and 136
// 214 against 179; FP32: nx 136 (just over half) 104 against 118, 160
// 106 against 131, 320 230 against 244; on smaller grids at their tuned
// tile heights, FP64 96^3 35 against 40, 192^3 127 against 131; FP32
// 128 x 64 x 64 (half) 27 against 29, 128^3 49 against 47.  Hence the
// shares below.  A batch of 64 small FP32 solves whose rows are multiples
// of four ran 160 ms with its partly filled members on plane tiles against
// 142 with none: batches keep such rows on consecutive tiles.
constexpr double kRaggedUse[2] = {0.7, 0.5};   // FP64, FP32

// Narrow plane tiles (64 x 4, one cell a thread, one sweep per iteration)
// where the wide ones are not taken: in batches, for single solves whose
// consecutive-cell tiles would run one cell a thread (rows of an odd length)
// or that have at most kNarrowCells cells, and wherever PCG_NARROW_TILES
// asks; not with two sweeps, consecutive tiles asked for, or fractions.
// Measured against consecutive-cell tiles, per iteration at the tuned tile
// heights (FP64, FP32): 33^3 17.0 against 20.8 us and 17.0 against 21.7,
// 64^3 22.5 against 25.8 and 23.4 against 25.0, odd rows 127^3 54 against
// 83 and 46 against 64, 255^3 234 against 302 and 188 against 351, 383^3
// 750 against 995 and 594 against 758, 447^3 1148 against 1583 and 982
// against 1379; but against the grouped tiles of rows of pairs or quads
// past 2^18 cells they lose (160 x 256 x 256 FP64 223 against 195,
// 120 x 256 x 256 FP32 112 against 94, 100 x 300 x 300 FP32 176 against
// 128).  The 64-solve FP32+IR batch 159 against 175 ms (one launch per
// iteration once every member sweeps), the served capacity 136 against 132
// solves/s.
constexpr int64_t kNarrowCells = 1 << 18;

bool narrow_allowed(const pcg_grid_t &g, int flags, bool batch)
{
    if (flags & (PCG_TWO_SWEEPS | PCG_FLAT_TILES | PCG_FRACTIONS)) return false;
    if ((flags & PCG_NARROW_TILES) || batch) return true;
    // consecutive-cell tiles group cells in pairs or quads on rows of even
    // length, one cell a thread otherwise
    return g.nx % 2 != 0 || (int64_t)g.nx * g.ny * g.nz <= kNarrowCells;
}

// The group width of a grid's plane tiles (cells a thread, of adjacent
// columns): 0 for consecutive-cell tiles, 2 (FP64) or 4 (FP32) for the wide
// tiles above, 1 for the narrow tiles.
int plane_group(const pcg_grid_t &g, int prec, int flags, const pcg_bc_t *bc, bool batch)
{
    if (flags & (PCG_FLAT_TILES | PCG_FRACTIONS)) return 0;
    if (bc && bc->kind[2] == PCG_BC_PERIODIC && g.ny > 1 && g.ny % kTileY != 0) return 0;
    const bool f32 = prec == PCG_PREC_FP32_IR;
    const bool px = bc && bc->kind[0] == PCG_BC_PERIODIC && g.nx > 1;
    const int nw = f32 ? 4 : 2;
    const int width = nw * kBlock / kTileY;
    if (g.nx % nw == 0) {
        if (g.nx % width == 0) return nw;
        const int tiles = (g.nx + width - 1) / width;
        if (!px && ((flags & PCG_PLANE_TILES) ||
                    (!batch && g.nx >= kRaggedUse[f32] * tiles * width)))
            return nw;
    }
    if (narrow_allowed(g, flags, batch) && (!px || g.nx % (kBlock / kTileY) == 0)) return 1;
    return 0;
}

Geometry make_geometry(const pcg_grid_t &g, int prec, int tz_opt, bool batch, int group)
{
    const bool tiles2d = group > 0;
    Geometry G;
    G.nx = g.nx; G.ny = g.ny; G.nz = g.nz;
    G.n = (int64_t)g.nx * g.ny * g.nz;
    G.tz = tz_opt > 0 ? tz_opt : rule_for(G.n, prec, batch, group).tz;
    if (G.tz > g.nz) G.tz = g.nz;
    const int64_t plane = (int64_t)g.nx * g.ny;
    // pass A addresses a tile's tz + 2 planes of 8-byte values with 32-bit
    // byte offsets
    const int64_t tz_cap = kMaxTileBytes / (plane * 8) - 2;
    if (G.tz > tz_cap) G.tz = (int)std::max<int64_t>(1, tz_cap);
    // adjacent columns per thread: two when rows have an even length, four
    // for FP32 passes when it is a multiple of four
    G.cpt = tiles2d ? group
                    : (prec == PCG_PREC_FP32_IR && g.nx % 4 == 0) ? 4 : (g.nx % 2 == 0 ? 2 : 1);
    const int64_t per_tile = (int64_t)G.cpt * kBlock;
    if (tiles2d) {
        G.tx = G.cpt * kBlock / kTileY;    // 128 (FP64 pairs), 256 (FP32 quads) or 64
        G.ty = kTileY;
        G.tiles_x = (g.nx + G.tx - 1) / G.tx;
        G.plane_tiles = G.tiles_x * ((g.ny + kTileY - 1) / kTileY);
    } else {
        G.tx = G.ty = G.tiles_x = 0;
        G.plane_tiles = (int)((plane + per_tile - 1) / per_tile);
    }
    G.ztiles = (g.nz + G.tz - 1) / G.tz;
    G.ntiles = (int64_t)G.plane_tiles * G.ztiles;
    return G;
}

// Bytes of the four fraction arrays of a grid (FP64 MAC faces and cells).
size_t frac_bytes(const Geometry &G)
{
    const size_t nx = G.nx, ny = G.ny, nz = G.nz;
    return align_up(8 * (nx + 1) * ny * nz, kAlign) + align_up(8 * nx * (ny + 1) * nz, kAlign) +
           align_up(8 * nx * ny * (nz + 1), kAlign) + align_up(8 * nx * ny * nz, kAlign);
}

// Whether the iterations of a grid (FP64, or the FP32 inner ones) run as
// one sweep each: on plane tiles unless switched off.  Measured on the
// 512^3 wedge against the two LDS-staged passes: FP64 1.167 against 1.559
// ms per iteration, FP32 0.643 against 0.834.
bool one_sweep(const Geometry &G, int prec, int flags)
{
    (void)prec;
    return !(flags & PCG_TWO_SWEEPS) && G.tx > 0;
}

size_t slot_bytes(const Geometry &G, int prec, bool frac = false, bool sweep = false)
{
    const size_t n = (size_t)G.n;
    const size_t es = prec == PCG_PREC_FP32_IR ? 4 : 8;
    size_t b = frac ? frac_bytes(G) : 0;
    b += align_up(8 * n, kAlign);                    // rho64
    if (prec == PCG_PREC_FP32_IR) b += align_up(4 * n, kAlign);  // rho32
    b += 4 * align_up(es * n, kAlign);               // z and three directions
    if (sweep) b += align_up(es * n, kAlign);        // second z of the one-sweep form
    if (prec == PCG_PREC_FP32_IR) b += align_up(4 * n, kAlign);  // d32
    b += align_up(kMaxPartials * 8 * (size_t)G.ntiles, kAlign);  // partials
    b += align_up(n, kAlign);                                      // classes
    b += align_up(kClasses * kClasses * 12, kAlign);              // tables
    return b;
}

// Workspace of one solve of a grid whose walls are not known yet: a
// periodic y axis may still send a grid that allows plane tiles to
// consecutive-cell tiles, whose tile count (and so partial sums) differs,
// so the larger of the two forms.
size_t grid_bytes(const pcg_grid_t &g, int prec, int tz_opt, bool batch, int flags, bool frac)
{
    const Geometry flat = make_geometry(g, prec, tz_opt, batch, 0);
    size_t b = slot_bytes(flat, prec, frac, false);
    auto cover = [&](int group) {
        const Geometry G = make_geometry(g, prec, tz_opt, batch, group);
        b = std::max(b, slot_bytes(G, prec, frac, one_sweep(G, prec, flags)));
    };
    const int group = plane_group(g, prec, flags, nullptr, batch);
    if (group) cover(group);
    // a periodic x axis turns down wide tiles on rows of partial ones, which
    // then take the narrow ones (more tiles, and so more partial sums)
    const int width = (prec == PCG_PREC_FP32_IR ? 4 : 2) * kBlock / kTileY;
    if (group > 1 && g.nx % width != 0 && narrow_allowed(g, flags, batch)) cover(1);
    return b;
}

size_t head_bytes(int max_slots)
{
    return align_up(sizeof(BatchHeader), kAlign) +
           align_up(sizeof(Slot) * max_slots, kAlign) +
           align_up(sizeof(SlotState) * max_slots, kAlign) + kAlign;  // + error flag
}

int check_grid(const pcg_grid_t *g)
{
    if (!g) return PCG_EINVAL;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return PCG_EINVAL;
    if (!(g->h > 0.0) || !std::isfinite(g->h)) return PCG_EINVAL;
    const int64_t n = (int64_t)g->nx * g->ny * g->nz;
    if (n >= ((int64_t)1 << 31)) return PCG_EUNSUPPORTED;
    // a tile of one plane and its two neighbours must fit pass A's 32-bit
    // byte offsets
    if ((int64_t)g->nx * g->ny * 8 * 3 > kMaxTileBytes) return PCG_EUNSUPPORTED;
    return PCG_OK;
}

// Dirichlet walls as a bit mask (bit f: wall f) and periodic axes (bit 0: x,
// bit 1: y).  Periodic walls pair up on x or y; periodic z is not supported.
int check_bc(const pcg_bc_t *bc, int *mask_out, int *per_out = nullptr)
{
    if (!bc) return PCG_EINVAL;
    int m = 0, per = 0;
    for (int f = 0; f < 6; ++f) {
        const int k = bc->kind[f];
        if (k != PCG_BC_NEUMANN && k != PCG_BC_DIRICHLET && k != PCG_BC_PERIODIC)
            return PCG_EINVAL;
        if (k == PCG_BC_DIRICHLET) m |= 1 << f;
    }
    for (int a = 0; a < 3; ++a) {
        const bool lo = bc->kind[2 * a] == PCG_BC_PERIODIC;
        const bool hi = bc->kind[2 * a + 1] == PCG_BC_PERIODIC;
        if (lo != hi) return PCG_EINVAL;
        if (lo && a == 2) return PCG_EUNSUPPORTED;
        if (lo) per |= 1 << a;
    }
    *mask_out = m;
    if (per_out) *per_out = per;
    return PCG_OK;
}

int check_opts(const pcg_opts_t *o)
{
    if (!o) return PCG_OK;
    if (o->precision != PCG_PREC_FP64 && o->precision != PCG_PREC_FP32_IR) return PCG_EINVAL;
    if (o->check_every < 0 || o->inner_maxit < 0 || o->tz < 0 || o->grid_blocks < 0) return PCG_EINVAL;
    if (o->inner_tol < 0.0 || o->inner_tol >= 1.0 || std::isnan(o->inner_tol)) return PCG_EINVAL;
    if (o->flags & ~(PCG_WARM_START | PCG_SKIP_CONNECTIVITY_CHECK | PCG_NO_DENSITY_CLASSES |
                     PCG_FRACTIONS | PCG_FLAT_TILES | PCG_PLANE_TILES | PCG_TWO_SWEEPS |
                     PCG_NARROW_TILES))
        return PCG_EINVAL;
    return PCG_OK;
}

// Connected fluid regions and how many of them touch no Dirichlet wall.
// Flood fill over x-runs of fluid cells: the mask, one bit per cell, is split
// row by row into maximal runs a 32-bit word at a time, then a breadth-first
// search per region moves between runs of neighbouring rows (y and z) that
// overlap in x, and across periodic walls (the first and last run of a row
// for x, the first and last row of a plane for y).  Work is linear in the
// words for the split and in the runs for the search.
struct FluidRegions {
    int64_t regions = 0;
    int64_t unanchored = 0;
};

// Bit layout of a packed mask: words_per_row(nx) 32-bit words per row, bit j
// of word w the cell x = 32 w + j, 1 = hull, the bits past the row's end set.
int words_per_row(int nx) { return (nx + 31) / 32; }

// The same packing on the host (for a host mask).
std::vector<uint32_t> pack_mask_host(const uint8_t *m, int nx, int64_t nrows)
{
    const int wpr = words_per_row(nx);
    std::vector<uint32_t> bits((size_t)(nrows * wpr));
    for (int64_t r = 0; r < nrows; ++r)
        for (int w = 0; w < wpr; ++w) {
            const int x0 = 32 * w, cnt = std::min(32, nx - x0);
            const uint8_t *row = m + r * nx + x0;
            uint32_t v = cnt < 32 ? ~0u << cnt : 0u;
            for (int j = 0; j < cnt; ++j) v |= (uint32_t)(row[j] != 0) << j;
            bits[(size_t)(r * wpr + w)] = v;
        }
    return bits;
}

// First cell >= i of a row whose bit is `hull` (1) or fluid (0), or the end
// of the row's words.
static int next_cell(const uint32_t *w, int wpr, int i, bool hull)
{
    int iw = i >> 5;
    if (iw >= wpr) return 32 * wpr;
    uint32_t v = (hull ? w[iw] : ~w[iw]) & (~0u << (i & 31));
    while (!v) {
        if (++iw == wpr) return 32 * wpr;
        v = hull ? w[iw] : ~w[iw];
    }
    return 32 * iw + __builtin_ctz(v);
}

FluidRegions fluid_regions(const uint32_t *bits, int nx, int ny, int nz, int bcmask,
                           int permask)
{
    const int64_t nrows = (int64_t)ny * nz;
    const int wpr = words_per_row(nx);
    std::vector<int64_t> row_start(nrows + 1, 0);
    std::vector<int32_t> ra, rb;  // run [ra, rb) in x
    std::vector<int64_t> run_row;
    ra.reserve(nrows * 2);
    rb.reserve(nrows * 2);
    run_row.reserve(nrows * 2);
    for (int64_t r = 0; r < nrows; ++r) {
        row_start[r] = (int64_t)ra.size();
        const uint32_t *w = bits + r * wpr;
        int i = 0;
        while (true) {
            const int a = next_cell(w, wpr, i, false);
            if (a >= nx) break;
            i = std::min(next_cell(w, wpr, a, true), nx);
            ra.push_back(a);
            rb.push_back(i);
            run_row.push_back(r);
        }
    }
    row_start[nrows] = (int64_t)ra.size();
    const int64_t nruns = (int64_t)ra.size();
    const bool perx = (permask & 1) && nx > 1, pery = (permask & 2) && ny > 1;
    FluidRegions out;
    std::vector<uint8_t> seen(nruns, 0);
    std::vector<int64_t> queue;
    queue.reserve(1024);
    auto push = [&](int64_t u) {
        if (!seen[u]) { seen[u] = 1; queue.push_back(u); }
    };
    for (int64_t u0 = 0; u0 < nruns; ++u0) {
        if (seen[u0]) continue;
        queue.clear();
        push(u0);
        bool anchored = false;
        for (size_t h = 0; h < queue.size(); ++h) {
            const int64_t u = queue[h];
            const int64_t r = run_row[u];
            const int j = (int)(r % ny), k = (int)(r / ny);
            anchored = anchored || ((bcmask & 4) && j == 0) || ((bcmask & 8) && j == ny - 1) ||
                       ((bcmask & 16) && k == 0) || ((bcmask & 32) && k == nz - 1) ||
                       ((bcmask & 1) && ra[u] == 0) || ((bcmask & 2) && rb[u] == nx);
            int64_t nb[4] = { j > 0 ? r - 1 : (pery ? r + ny - 1 : -1),
                              j < ny - 1 ? r + 1 : (pery ? r - (ny - 1) : -1),
                              k > 0 ? r - ny : -1, k < nz - 1 ? r + ny : -1 };
            for (int e = 0; e < 4; ++e) {
                if (nb[e] < 0) continue;
                const int64_t b0 = row_start[nb[e]], b1 = row_start[nb[e] + 1];
                // first run of the neighbouring row ending after ra[u]
                int64_t v = std::upper_bound(rb.begin() + b0, rb.begin() + b1, ra[u]) - rb.begin();
                for (; v < b1 && ra[v] < rb[u]; ++v) push(v);
            }
            if (perx) {
                const int64_t f0 = row_start[r], f1 = row_start[r + 1] - 1;
                if (ra[u] == 0 && rb[f1] == nx) push(f1);
                if (rb[u] == nx && ra[f0] == 0) push(f0);
            }
        }
        ++out.regions;
        if (!anchored) ++out.unanchored;
    }
    return out;
}

// Solvability of a wall and hull layout: 0 when every fluid region touches
// a Dirichlet wall, 1 for a single region touching none (singular: the
// constant is the null vector), PCG_ESINGULAR otherwise.
int classify_regions(const FluidRegions &f)
{
    if (f.unanchored == 0) return 0;
    if (f.regions == 1) return 1;
    return PCG_ESINGULAR;
}

struct SlotHost {
    bool used = false;      // holds a prepared density field
    bool ready = false;     // its coefficients are valid (a failed rebuild clears it)
    bool running = false;   // in the slot table
    bool finished = false;  // completion observed on the host
    Geometry geo{};
    int bcmask = 0;
    int permask = 0;
    bool singular = false;   // no Dirichlet wall reaches the fluid
    double h2 = 0.0;
    size_t off = 0, bytes = 0;
    double *rho64 = nullptr;
    float *rho32 = nullptr;
    void *z = nullptr, *dir0 = nullptr, *dir1 = nullptr, *dir2 = nullptr;
    void *z2 = nullptr;          // one-sweep iterations only
    float *d32 = nullptr;
    double *partials = nullptr;
    uint8_t *cls = nullptr;      // arena: class per cell
    double *tab64 = nullptr;     // arena: kClasses^2 coefficients
    float *tab32 = nullptr;
    bool classes = false;        // class coding in use
    int nclasses = 0;            // fluid classes when coded
    double *ax = nullptr, *ay = nullptr, *az = nullptr, *vol = nullptr;  // arena, if reserved
    bool has_frac = false;       // cut-cell fractions in use (coefficient mode 2)
    const double *rhs = nullptr;
    double *x = nullptr;
    Clock::time_point t0;
    double ms = 0.0;
};

// Coefficient mode of a slot, as the kernels derive it from its description
// (kernel template argument MODE): 0 per-cell density, 1 density classes,
// 2 per-cell density with cut-cell fractions, 3 classes and 4 per-cell
// density on 2-D plane tiles.
constexpr int kModes = 5;
int slot_mode(const SlotHost &S)
{
    if (S.has_frac) return 2;
    if (S.geo.tx > 0) return S.classes ? 3 : 4;
    return S.classes ? 1 : 0;
}

}  // namespace

// Host mirrors of an arena's head for an engine that must not allocate
// (pinned host memory is an allocation): owned by the caller, alive as long
// as the engine.  One slot.
struct HostMirror {
    BatchHeader hdr;
    Slot slots[1];
    SlotState states[1];
    alignas(8) int bad[64];   // error flag + class search words, 256 bytes
};

struct Engine {
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    int prec = PCG_PREC_FP64;
    int check_every = kDefaultCheckEvery;
    int grid = 0;
    int grid_opt = 0;
    int tz_opt = 0;
    int inner_maxit = 0;
    double inner_tol = kDefaultInnerTol;
    bool frac_space = false;  // slots reserve room for cut-cell fractions
    int flags = 0;            // option flags of the context or batch
    char *arena = nullptr;
    size_t arena_bytes = 0;
    int max_slots = 0;
    BatchHeader *d_hdr = nullptr;
    Slot *d_slots = nullptr;
    SlotState *d_states = nullptr;
    int *d_bad = nullptr;
    BatchHeader *h_hdr = nullptr;
    Slot *h_slots = nullptr;
    SlotState *h_states = nullptr;
    int *h_bad = nullptr;
    Arena alloc;
    std::vector<SlotHost> slots;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool table_dirty = true;
    int view_id = -1;       // slot whose projection view is in d_slots[0]
    int64_t total_tiles = 0;
    int nrunning = 0;
    bool is_batch = false;  // created by pcg_batch_create (batch tile table)
    int modes = 0;          // bit m: a running slot uses coefficient mode m (slot_mode)
    int graph_modes = -1;   // modes the captured graph was built for
    bool k2only = false;    // second-half launches only (every solve in one sweep)
    int graph_k2only = -1;  // the same for the captured graph
    int fail_after = 0;     // test hook: the step call that reports a failure
    HostMirror *mirror = nullptr;  // caller-owned host mirrors: no pinned memory,
                                   // no capture stream, launches without graphs
    // timing mode
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<float> t_k1, t_k2;

    ~Engine() { teardown(); }

    void teardown()
    {
        // copies staged through the pinned host buffers may still be queued
        // on the caller's stream: let them finish before the buffers go
        if (h_hdr || h_slots || h_states || h_bad) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        for (auto e : ev) (void)hipEventDestroy(e);
        ev.clear();
        if (cap) (void)hipStreamDestroy(cap);
        cap = nullptr;
        if (!mirror) {
            if (h_hdr) (void)hipHostFree(h_hdr);
            if (h_slots) (void)hipHostFree(h_slots);
            if (h_states) (void)hipHostFree(h_states);
            if (h_bad) (void)hipHostFree(h_bad);
        }
        h_hdr = nullptr; h_slots = nullptr; h_states = nullptr; h_bad = nullptr;
    }

    int init(void *arena_ptr, size_t bytes, int nslots, const pcg_opts_t *o,
             void *hip_stream, HostMirror *hm = nullptr)
    {
        if (hm && nslots != 1) return PCG_EINVAL;
        if (!arena_ptr || nslots < 1) return PCG_EINVAL;
        if (((uintptr_t)arena_ptr) % kAlign) return PCG_EINVAL;
        int st = check_opts(o);
        if (st) return st;
        if (o) {
            prec = o->precision;
            if (o->check_every > 0) check_every = o->check_every;
            inner_maxit = o->inner_maxit;
            if (o->inner_tol > 0.0) inner_tol = o->inner_tol;
            tz_opt = o->tz;
            grid_opt = o->grid_blocks;
            frac_space = (o->flags & PCG_FRACTIONS) != 0;
            flags = o->flags;
        }
        arena = (char *)arena_ptr;
        arena_bytes = bytes;
        max_slots = nslots;
        const size_t hb = head_bytes(nslots);
        if (bytes < hb) return PCG_ENOMEM;
        size_t off = 0;
        d_hdr = (BatchHeader *)(arena + off);
        off += align_up(sizeof(BatchHeader), kAlign);
        d_slots = (Slot *)(arena + off);
        off += align_up(sizeof(Slot) * nslots, kAlign);
        d_states = (SlotState *)(arena + off);
        off += align_up(sizeof(SlotState) * nslots, kAlign);
        d_bad = (int *)(arena + off);
        alloc.reset(hb, bytes);
        slots.assign(nslots, SlotHost{});
        stream = (hipStream_t)hip_stream;
        if (hm) {
            mirror = hm;
            h_hdr = &hm->hdr;
            h_slots = hm->slots;
            h_states = hm->states;
            h_bad = hm->bad;
        } else {
            HIP_TRY(hipHostMalloc((void **)&h_hdr, sizeof(BatchHeader), hipHostMallocDefault));
            HIP_TRY(hipHostMalloc((void **)&h_slots, sizeof(Slot) * nslots, hipHostMallocDefault));
            HIP_TRY(hipHostMalloc((void **)&h_states, sizeof(SlotState) * nslots, hipHostMallocDefault));
            HIP_TRY(hipHostMalloc((void **)&h_bad, 256, hipHostMallocDefault));  // flag + class search words
        }
        std::memset(h_states, 0, sizeof(SlotState) * nslots);
        for (int i = 0; i < nslots; ++i) h_states[i].phase = PH_IDLE;
        HIP_TRY(hipMemcpyAsync(d_states, h_states, sizeof(SlotState) * nslots,
                               hipMemcpyHostToDevice, stream));
        h_hdr->total_tiles = 0;
        h_hdr->nslots = 0;
        h_hdr->chunked = 0;
        HIP_TRY(hipMemcpyAsync(d_hdr, h_hdr, sizeof(BatchHeader), hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        if (!mirror) HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        return PCG_OK;
    }

    bool batch_mode() const { return is_batch; }

    static void set_frac(Slot &d, const SlotHost &S)
    {
        d.ax = S.has_frac ? S.ax : nullptr;
        d.ay = S.has_frac ? S.ay : nullptr;
        d.az = S.has_frac ? S.az : nullptr;
        d.vol = S.has_frac ? S.vol : nullptr;
    }

    // Cut-cell fractions for a prepared slot that is not running: copy the
    // caller's arrays into the slot's reserved space and validate them on the
    // device (areas in [0, 1], fluid volumes in (0, 1]); all NULL clears.
    int set_fractions(int id, const double *ax, const double *ay, const double *az,
                      const double *vol)
    {
        if (id < 0 || id >= max_slots || !slots[id].used) return PCG_EINVAL;
        SlotHost &S = slots[id];
        if (S.running) return PCG_EBUSY;
        const int given = (ax != nullptr) + (ay != nullptr) + (az != nullptr) + (vol != nullptr);
        if (given != 0 && given != 4) return PCG_EINVAL;
        if (view_id == id) view_id = -1;
        table_dirty = true;
        S.has_frac = false;
        if (!given) return PCG_OK;
        if (!S.ax) return PCG_EINVAL;   // no room reserved (PCG_FRACTIONS not set)
        const size_t nx = S.geo.nx, ny = S.geo.ny, nz = S.geo.nz;
        const size_t nu = (nx + 1) * ny * nz, nv = nx * (ny + 1) * nz, nw = nx * ny * (nz + 1),
                     n = nx * ny * nz;
        *h_bad = 0;
        hipError_t e = hipMemcpyAsync(d_bad, h_bad, sizeof(int), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(S.ax, ax, 8 * nu, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(S.ay, ay, 8 * nv, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(S.az, az, 8 * nw, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(S.vol, vol, 8 * n, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess)
            e = launch_check_frac(S.ax, S.ay, S.az, S.vol, S.rho64, (int64_t)nu, (int64_t)nv,
                                  (int64_t)nw, (int64_t)n, d_bad, stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h_bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "fractions");
        if (*h_bad) return PCG_EDOMAIN;
        S.has_frac = true;
        return PCG_OK;
    }

    // Device description of a prepared slot for the projection kernels:
    // written into the head's spare slot entry when no solve runs.
    int slot_view(int id, Slot **d_slot)
    {
        SlotHost &S = slots[id];
        if (!S.used || !S.ready) return PCG_EINVAL;
        if (view_id == id) { *d_slot = d_slots; return PCG_OK; }
        Slot &d = h_slots[0];
        std::memset(&d, 0, sizeof(Slot));
        d.nx = S.geo.nx; d.ny = S.geo.ny; d.nz = S.geo.nz;
        d.bcmask = S.bcmask;
        d.permask = S.permask;
        d.h2 = S.h2;
        d.rho64 = S.rho64;
        d.cls = S.classes && !S.has_frac ? S.cls : nullptr;
        d.tab64 = S.tab64;
        d.ntiles = S.geo.ntiles;
        set_frac(d, S);
        HIP_TRY(hipMemcpyAsync(d_slots, h_slots, sizeof(Slot), hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        table_dirty = true;      // the solve path rebuilds the table before use
        view_id = id;
        *d_slot = d_slots;
        return PCG_OK;
    }

    size_t footprint(const pcg_grid_t &g) const
    {
        return grid_bytes(g, prec, tz_opt, batch_mode(), flags, frac_space);
    }

    // Reserve a slot and its memory, encode the density.  Does not start a solve.
    int prepare(const pcg_grid_t *grid_, const double *rho, const uint8_t *mask,
                const pcg_bc_t *bc, int flags, int *slot_out)
    {
        int st = check_grid(grid_);
        if (st) return st;
        int bm = 0, per = 0;
        st = check_bc(bc, &bm, &per);
        if (st) return st;
        if (!rho) return PCG_EINVAL;
        int id = -1;
        for (int i = 0; i < max_slots; ++i)
            if (!slots[i].used) { id = i; break; }
        if (id < 0) return PCG_EBUSY;
        const Geometry geo = make_geometry(*grid_, prec, tz_opt, batch_mode(),
                                           plane_group(*grid_, prec, flags | this->flags, bc,
                                                       batch_mode()));
        const bool sweep = one_sweep(geo, prec, flags | this->flags);
        const size_t need = slot_bytes(geo, prec, frac_space, sweep);
        size_t off = 0;
        if (!alloc.alloc(need, &off)) return max_slots == 1 ? PCG_ENOMEM : PCG_EBUSY;

        SlotHost &S = slots[id];
        S = SlotHost{};
        S.geo = geo;
        S.bcmask = bm;
        S.permask = per;
        S.h2 = grid_->h * grid_->h;
        S.off = off;
        S.bytes = need;
        const size_t n = (size_t)geo.n;
        const size_t es = prec == PCG_PREC_FP32_IR ? 4 : 8;
        char *p = arena + off;
        S.rho64 = (double *)p; p += align_up(8 * n, kAlign);
        if (prec == PCG_PREC_FP32_IR) { S.rho32 = (float *)p; p += align_up(4 * n, kAlign); }
        S.z = p; p += align_up(es * n, kAlign);
        if (sweep) { S.z2 = p; p += align_up(es * n, kAlign); }
        S.dir0 = p; p += align_up(es * n, kAlign);
        S.dir1 = p; p += align_up(es * n, kAlign);
        S.dir2 = p; p += align_up(es * n, kAlign);
        if (prec == PCG_PREC_FP32_IR) { S.d32 = (float *)p; p += align_up(4 * n, kAlign); }
        S.partials = (double *)p;
        p += align_up(kMaxPartials * 8 * (size_t)geo.ntiles, kAlign);
        S.cls = (uint8_t *)p;
        p += align_up(n, kAlign);
        S.tab64 = (double *)p;
        S.tab32 = (float *)(p + kClasses * kClasses * 8);
        p += align_up(kClasses * kClasses * 12, kAlign);
        if (frac_space) {
            const size_t nx = geo.nx, ny = geo.ny, nz = geo.nz;
            S.ax = (double *)p; p += align_up(8 * (nx + 1) * ny * nz, kAlign);
            S.ay = (double *)p; p += align_up(8 * nx * (ny + 1) * nz, kAlign);
            S.az = (double *)p; p += align_up(8 * nx * ny * (nz + 1), kAlign);
            S.vol = (double *)p;
        }

        st = encode_slot(S, rho, mask, flags);
        if (st) { alloc.release(off, need); S = SlotHost{}; return st; }
        S.used = true;
        *slot_out = id;
        return PCG_OK;
    }

    // Check connectivity (unless skipped), encode and validate the densities,
    // then (unless switched off) run the chained class rounds; one host round
    // trip reads both results.  Overwrites the slot's coefficients: on any
    // error the slot is left not ready.
    int encode_slot(SlotHost &S, const double *rho, const uint8_t *mask, int flags)
    {
        S.ready = false;
        S.classes = false;
        S.nclasses = 0;
        if (view_id >= 0 && &slots[view_id] == &S) view_id = -1;
        const Geometry &geo = S.geo;
        // connectivity: every fluid region touches a Dirichlet wall, or a
        // single region touches none (singular); unchecked, the walls decide
        S.singular = S.bcmask == 0;
        if (!(flags & PCG_SKIP_CONNECTIVITY_CHECK) && mask) {
            // packed on the device into the slot's z vector (4 n bytes or
            // more; unused until the solve initialises it), then read back
            const int wpr = words_per_row(geo.nx);
            const int64_t nwords = (int64_t)geo.ny * geo.nz * wpr;
            std::vector<uint32_t> h((size_t)nwords);
            uint32_t *dbits = (uint32_t *)S.z;
            hipError_t e = launch_pack_mask(mask, dbits, geo.nx, wpr, nwords, stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(h.data(), dbits, (size_t)nwords * 4, hipMemcpyDeviceToHost,
                                   stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return hip_fail(e, "mask bits");
            const int kind = classify_regions(
                fluid_regions(h.data(), geo.nx, geo.ny, geo.nz, S.bcmask, S.permask));
            if (kind < 0) return kind;
            S.singular = kind == 1;
        }
        const bool want_classes = !(flags & PCG_NO_DENSITY_CLASSES);
        *h_bad = 0;
        hipError_t e = hipMemcpyAsync(d_bad, h_bad, sizeof(int), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = launch_encode(rho, mask, S.rho64, S.rho32, geo.n, d_bad, stream);
        if (e == hipSuccess && want_classes) e = classify_launch(S);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_bad, d_bad, want_classes ? 8 + 8 * kRounds : sizeof(int),
                               hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "encode");
        if (*h_bad) return PCG_EDOMAIN;
        if (want_classes) {
            int st = classify_finish(S);
            if (st) return st;
        }
        S.ready = true;
        table_dirty = true;      // coefficient mode and pointers may have changed
        return PCG_OK;
    }

    // New densities (and hull) for a prepared slot that is not running.
    int refresh(int id, const double *rho, const uint8_t *mask, int flags)
    {
        if (id < 0 || id >= max_slots || !slots[id].used || !rho) return PCG_EINVAL;
        SlotHost &S = slots[id];
        if (S.running) return PCG_EBUSY;
        return encode_slot(S, rho, mask, flags);
    }

    // Code the densities as classes when there are at most kMaxFluidClasses
    // distinct fluid values.  kMaxFluidClasses + 2 chained device rounds (no
    // host round trip between them) find the distinct values in increasing
    // order and label the cells; one copy brings the values back, and the
    // face coefficient table is computed here exactly as 2/(rho_a + rho_b)
    // in FP64 (and FP32).
    static constexpr int kRounds = kMaxFluidClasses + 2;

    hipError_t classify_launch(SlotHost &S)
    {
        unsigned long long *d_words = (unsigned long long *)(d_bad + 2);
        unsigned long long *h_words = (unsigned long long *)(h_bad + 2);
        for (int r = 0; r < kRounds; ++r) h_words[r] = ~0ull;
        hipError_t e = hipMemcpyAsync(d_words, h_words, 8 * kRounds, hipMemcpyHostToDevice, stream);
        for (int r = 0; r < kRounds && e == hipSuccess; ++r)
            e = launch_classify(S.rho64, S.cls, S.geo.n, r, d_words, stream);
        return e;
    }

    // After classify_launch and a synchronize: read the distinct values and
    // build the coefficient tables.
    int classify_finish(SlotHost &S)
    {
        const unsigned long long *h_words = (const unsigned long long *)(h_bad + 2);
        std::vector<double> pal;
        for (int r = 0; r < kRounds && h_words[r] != ~0ull; ++r) {
            double v;
            std::memcpy(&v, &h_words[r], 8);
            pal.push_back(v);
        }
        // a value in words[kMaxFluidClasses] means a 15th distinct density
        if ((int)pal.size() > kMaxFluidClasses) return PCG_OK;
        double rho[kClasses];
        for (int a = 0; a < kClasses; ++a) rho[a] = 0.0;
        for (size_t a = 0; a < pal.size(); ++a) rho[a] = pal[a];
        rho[kClsWallD] = 0.0;
        rho[kClsSolid] = INFINITY;
        std::vector<double> t64(kClasses * kClasses);
        std::vector<float> t32(kClasses * kClasses);
        for (int a = 0; a < kClasses; ++a)
            for (int b = 0; b < kClasses; ++b) {
                const bool live = (a < (int)pal.size() || a >= kClsWallD) &&
                                  (b < (int)pal.size() || b >= kClsWallD);
                const double sum = rho[a] + rho[b];
                t64[a * kClasses + b] = live && std::isfinite(sum) && sum > 0.0 ? 2.0 / sum : 0.0;
                const float sf = (float)rho[a] + (float)rho[b];
                t32[a * kClasses + b] = live && std::isfinite(sf) && sf > 0.0f ? 2.0f / sf : 0.0f;
            }
        // on the engine's stream (not the null stream, which would wait for
        // every other stream of the device); the host tables live until the
        // copies have finished
        HIP_TRY(hipMemcpyAsync(S.tab64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemcpyAsync(S.tab32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        S.classes = true;
        S.nclasses = (int)pal.size();
        return PCG_OK;
    }

    // Start a solve on a prepared slot.
    int start(int id, const double *rhs, double *x, double tol, int maxit, int flags)
    {
        if (id < 0 || id >= max_slots || !slots[id].used || !slots[id].ready) return PCG_EINVAL;
        if (!rhs || !x) return PCG_EINVAL;
        if (!(tol > 0.0) || !std::isfinite(tol) || maxit < 0) return PCG_EINVAL;
        SlotHost &S = slots[id];
        if (S.running) return PCG_EBUSY;
        S.rhs = rhs;
        S.x = x;
        S.finished = false;
        S.ms = 0.0;
        SlotState &h = h_states[id];
        std::memset(&h, 0, sizeof(SlotState));
        h.phase = prec == PCG_PREC_FP64 ? K1_INIT64 : K1_IR_INIT;
        if (S.singular) {   // the source's fluid mean first
            h.after = h.phase;
            h.phase = K1_MEAN_B;
            h.singular = 1;
        }
        h.status = PCG_PENDING;
        h.tol = tol;
        h.maxit = maxit;
        h.inner_maxit = inner_maxit > 0 ? inner_maxit : INT32_MAX;
        h.inner_tol2 = inner_tol * inner_tol;
        h.warm = (flags & PCG_WARM_START) ? 1 : 0;
        h.fused = S.z2 ? 1 : 0;
        h.scale = 1.0;
        HIP_TRY(hipMemcpyAsync(d_states + id, &h, sizeof(SlotState), hipMemcpyHostToDevice, stream));
        S.running = true;
        S.t0 = Clock::now();
        table_dirty = true;
        return PCG_OK;
    }

    void release(int id)
    {
        SlotHost &S = slots[id];
        if (!S.used) return;
        alloc.release(S.off, S.bytes);
        if (S.running) table_dirty = true;
        if (view_id == id) view_id = -1;
        S = SlotHost{};
        h_states[id].phase = PH_IDLE;
    }

    int upload_table()
    {
        if (!table_dirty) return PCG_OK;
        int64_t tb = 0;
        int ns = 0;
        int m = 0;
        bool all_fused = true;
        for (int id = 0; id < max_slots; ++id) {
            SlotHost &S = slots[id];
            if (!S.used || !S.running) continue;
            Slot &d = h_slots[ns++];
            std::memset(&d, 0, sizeof(Slot));
            d.nx = S.geo.nx; d.ny = S.geo.ny; d.nz = S.geo.nz;
            d.bcmask = S.bcmask;
        d.permask = S.permask;
            d.plane_tiles = S.geo.plane_tiles;
            d.cpt = S.geo.cpt;
            d.tx = S.geo.tx;
            d.ty = S.geo.ty;
            d.tiles_x = S.geo.tiles_x;
            d.ztiles = S.geo.ztiles;
            d.tz = S.geo.tz;
            d.tile_begin = tb;
            d.ntiles = S.geo.ntiles;
            d.h2 = S.h2;
            d.rhs = S.rhs;
            d.x = S.x;
            d.rho64 = S.rho64;
            d.rho32 = S.rho32;
            d.z = S.z;
            d.z2 = S.z2;
            d.dir0 = S.dir0;
            d.dir1 = S.dir1;
            d.dir2 = S.dir2;
            d.d32 = S.d32;
            d.partials = S.partials;
            d.st = d_states + id;
            d.cls = S.classes && !S.has_frac ? S.cls : nullptr;
            set_frac(d, S);
            d.tab64 = S.tab64;
            d.tab32 = S.tab32;
            m |= 1 << slot_mode(S);
            tb += S.geo.ntiles;
            all_fused = all_fused && S.z2 != nullptr;
        }
        h_hdr->total_tiles = tb;
        h_hdr->nslots = ns;
        h_hdr->chunked = ns > 1 ? 1 : 0;
        // every solve in one sweep per iteration: second-half launches only
        // (timed runs keep both positions, so each is timed on its own)
        k2only = ns > 0 && all_fused && !timing;
        h_hdr->k2only = k2only ? 1 : 0;
        total_tiles = tb;
        nrunning = ns;
        modes = m;
        view_id = -1;
        if (ns) HIP_TRY(hipMemcpyAsync(d_slots, h_slots, sizeof(Slot) * ns, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipMemcpyAsync(d_hdr, h_hdr, sizeof(BatchHeader), hipMemcpyHostToDevice, stream));
        table_dirty = false;
        return PCG_OK;
    }

    int choose_grid() const
    {
        // batches: workgroups take contiguous tile ranges when several solves
        // are resident; two workgroups per CU measured best there
        int g = grid_opt > 0 ? grid_opt : (max_slots == 1 ? kDefaultGridMax : kBatchGrid);
        if (max_slots == 1) {
            int64_t t = 0, n = 0;
            int group = 0;
            for (auto &S : slots)
                if (S.used) {
                    t = std::max<int64_t>(t, S.geo.ntiles);
                    n = S.geo.n;
                    group = S.geo.tx > 0 ? S.geo.cpt : 0;
                }
            if (grid_opt <= 0 && n > 0 && rule_for(n, prec, false, group).grid > 0)
                g = rule_for(n, prec, false, group).grid;
            if (t > 0 && t < g) g = (int)t;
        }
        g = std::max(8, (g + 7) / 8 * 8);
        return g;
    }

    int capture()
    {
        const int g = choose_grid();
        if (exec && g == grid && modes == graph_modes && (int)k2only == graph_k2only)
            return PCG_OK;
        if (exec) { (void)hipGraphExecDestroy(exec); exec = nullptr; }
        if (graph) { (void)hipGraphDestroy(graph); graph = nullptr; }
        grid = g;
        HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipSuccess;
        for (int i = 0; i < check_every && err == hipSuccess; ++i)
            err = launch_iteration(cap);
        hipGraph_t gph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cap, &gph);
        if (err != hipSuccess) { if (gph) (void)hipGraphDestroy(gph); return hip_fail(err, "capture launch"); }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        graph = gph;
        HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        graph_modes = modes;
        graph_k2only = k2only;
        return PCG_OK;
    }

    // The launches of iteration position w, once per coefficient mode in
    // use: 1 the first-half actions (K1: pass A; the first mode's launch,
    // kernel position 3, also serves every slot's set-up, FP64 residual and
    // flush actions), 2 pass B (K2).  Position 0 launches nothing: a kernel
    // boundary of its own measured 1-12 % of an iteration (512^3 .. 160^3).
    hipError_t launch_position(int w, hipStream_t s)
    {
        hipError_t e = hipSuccess;
        if (w == 0) return e;
        bool first = true;
        for (int m = 0; m < kModes && e == hipSuccess; ++m) {
            if (!(modes & (1 << m))) continue;
            // second-half launches only: both positions launch kernel 2
            const int which = k2only ? 2 : ((w == 1 && first) ? 3 : w);
            e = launch_iter(prec, which, m, grid, d_hdr, d_slots, s);
            first = false;
        }
        return e;
    }

    // One iteration: K1, then K2, of each coefficient mode in use.
    hipError_t launch_iteration(hipStream_t s)
    {
        hipError_t e = hipSuccess;
        for (int w = 0; w < 3 && e == hipSuccess; ++w) e = launch_position(w, s);
        return e;
    }

    // Direct launches with an event around each kernel position (timing
    // mode): K1 and K2 durations include every coefficient mode in use.
    int timed_chunk()
    {
        const int ne = 3 * check_every + 1;
        while ((int)ev.size() < ne) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            ev.push_back(e);
        }
        HIP_TRY(hipEventRecord(ev[0], stream));
        for (int i = 0; i < check_every; ++i)
            for (int w = 0; w < 3; ++w) {
                HIP_TRY(launch_position(w, stream));
                HIP_TRY(hipEventRecord(ev[3 * i + w + 1], stream));
            }
        HIP_TRY(hipEventSynchronize(ev[ne - 1]));
        for (int i = 0; i < check_every; ++i) {
            float a = 0.f, b = 0.f;
            HIP_TRY(hipEventElapsedTime(&a, ev[3 * i + 1], ev[3 * i + 2]));
            HIP_TRY(hipEventElapsedTime(&b, ev[3 * i + 2], ev[3 * i + 3]));
            t_k1.push_back(a);
            t_k2.push_back(b);
        }
        return PCG_OK;
    }

    // Stop tracking a solve the host gave up on (a runtime error, or a solve
    // that stopped advancing): wait for the stream, then mark the slot not
    // running with `code` as its final status, so the slot can start again.
    void abandon(int id, int code)
    {
        (void)hipStreamSynchronize(stream);
        SlotHost &S = slots[id];
        if (!S.running) return;
        S.running = false;
        S.finished = true;
        S.ms = ms_since(S.t0);
        h_states[id].status = code;
        h_states[id].phase = PH_DONE;
        table_dirty = true;
    }

    // Run `replays` graphs (or timed chunks), then refresh the status mirror.
    int step(int replays)
    {
        if (fail_after > 0 && --fail_after == 0) {
            g_hip_err = "failure injected by pcg_inject_failure";
            return PCG_EHIP;
        }
        int st = upload_table();
        if (st) return st;
        if (nrunning == 0) return PCG_OK;
        if (mirror) {
            grid = choose_grid();    // launched directly: no graph to capture
        } else {
            st = capture();
            if (st) return st;
        }
        for (int r = 0; r < replays; ++r) {
            if (timing) {
                st = timed_chunk();
                if (st) return st;
            } else if (mirror) {
                for (int i = 0; i < check_every; ++i) HIP_TRY(launch_iteration(stream));
            } else {
                HIP_TRY(hipGraphLaunch(exec, stream));
            }
        }
        HIP_TRY(hipMemcpyAsync(h_states, d_states, sizeof(SlotState) * max_slots,
                               hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        for (int id = 0; id < max_slots; ++id) {
            SlotHost &S = slots[id];
            if (!S.used || !S.running) continue;
            if (h_states[id].phase == PH_DONE) {
                S.running = false;
                S.finished = true;
                S.ms = ms_since(S.t0);
                table_dirty = true;
            }
        }
        return PCG_OK;
    }

    int running_count() const
    {
        int n = 0;
        for (auto &S : slots) n += S.running ? 1 : 0;
        return n;
    }

    void fill_stats(int id, pcg_stats_t *out) const
    {
        const SlotState &h = h_states[id];
        out->status = h.status;
        out->iters = h.iter;
        out->outer_iters = h.outer;
        const double bb = h.bb;
        out->rel_res_true = bb > 0 ? std::sqrt(h.rr_true / bb) : 0.0;
        out->rel_res_recursive = bb > 0 ? std::sqrt(h.rr / bb) : 0.0;
        if (prec == PCG_PREC_FP32_IR) out->rel_res_recursive = out->rel_res_true;
        out->ms = slots[id].ms;
    }
};

struct pcg_ctx {
    Engine eng;
    int slot = -1;
    int flags = 0;
    double last_k1 = 0.0, last_k2 = 0.0;
    int last_n = 0;
    bool have_timing = false;
};

struct pcg_batch {
    Engine eng;
};

namespace {

// Poll a started solve until it finishes and fill its statistics.  Every
// step advances a running solve (its iteration count or its phase): one that
// stops moving is reported instead of polled forever.  A host-side failure
// ends the solve with that status (statistics included) and leaves the slot
// able to start again.
int run_to_end(Engine &eng, int slot, Clock::time_point t0, pcg_stats_t *stats)
{
    auto fail = [&](int code) {
        eng.abandon(slot, code);
        if (stats) {
            eng.fill_stats(slot, stats);
            stats->ms = ms_since(t0);
        }
        return code;
    };
    int last_iter = -1, last_phase = -1, still = 0;
    while (eng.slots[slot].running) {
        const int st = eng.step(1);
        if (st) return fail(st);
        const SlotState &h = eng.h_states[slot];
        if (h.iter == last_iter && h.phase == last_phase) {
            if (++still >= 4) {
                g_hip_err = "solve made no progress";
                return fail(PCG_EHIP);
            }
        } else {
            still = 0;
        }
        last_iter = h.iter;
        last_phase = h.phase;
    }
    pcg_stats_t s;
    eng.fill_stats(slot, &s);
    s.ms = ms_since(t0);
    if (stats) *stats = s;
    return s.status;
}

void average_nonempty(const std::vector<float> &t, double *avg, int *n)
{
    // launches that did work dominate; an early-exit launch (solve already
    // finished) is far shorter than the median working launch
    if (t.empty()) { *avg = 0.0; *n = 0; return; }
    std::vector<float> s(t);
    std::sort(s.begin(), s.end());
    const float med = s[s.size() / 2];
    double sum = 0.0;
    int c = 0;
    for (float v : t)
        if (v >= 0.25f * med) { sum += v; ++c; }
    *avg = c ? sum / c : 0.0;
    *n = c;
}

}  // namespace

// ======================================================================
// C ABI
// ======================================================================

extern "C" {

int pcg_workspace_bytes(const pcg_grid_t *grid, const pcg_opts_t *opts,
                        size_t *out_bytes)
{
    if (!out_bytes) return PCG_EINVAL;
    int st = check_grid(grid);
    if (st) return st;
    st = check_opts(opts);
    if (st) return st;
    const int prec = opts ? opts->precision : PCG_PREC_FP64;
    const int flags = opts ? opts->flags : 0;
    *out_bytes = head_bytes(1) + grid_bytes(*grid, prec, opts ? opts->tz : 0, false, flags,
                                            (flags & PCG_FRACTIONS) != 0);
    return PCG_OK;
}

int pcg_setup(pcg_ctx_t **out, const pcg_grid_t *grid, const double *rho,
              const uint8_t *solid_mask, const pcg_bc_t *bc,
              const pcg_opts_t *opts, void *workspace, size_t ws_bytes,
              void *hip_stream)
{
    if (!out) return PCG_EINVAL;
    *out = nullptr;
    int st = check_grid(grid);
    if (st) return st;
    int bm = 0;
    st = check_bc(bc, &bm);
    if (st) return st;
    st = check_opts(opts);
    if (st) return st;
    if (!rho || !workspace) return PCG_EINVAL;
    size_t need = 0;
    pcg_workspace_bytes(grid, opts, &need);
    if (ws_bytes < need) return PCG_ENOMEM;
    pcg_ctx *c = new (std::nothrow) pcg_ctx();
    if (!c) return PCG_ENOMEM;
    st = c->eng.init(workspace, ws_bytes, 1, opts, hip_stream);
    if (st) { delete c; return st; }
    c->flags = opts ? opts->flags : 0;
    st = c->eng.prepare(grid, rho, solid_mask, bc, c->flags, &c->slot);
    if (st) { delete c; return st; }
    *out = c;
    return PCG_OK;
}

int pcg_solve(pcg_ctx_t *c, const double *rhs, double *p, double tol,
              int32_t maxit, pcg_stats_t *stats)
{
    if (!c) return PCG_EINVAL;
    return pcg_solve_ex(c, rhs, p, tol, maxit, c->flags & PCG_WARM_START, stats);
}

int pcg_solve_ex(pcg_ctx_t *c, const double *rhs, double *p, double tol,
                 int32_t maxit, int32_t flags, pcg_stats_t *stats)
{
    if (!c) return PCG_EINVAL;
    if (flags & ~PCG_WARM_START) return PCG_EINVAL;
    const auto t0 = Clock::now();
    int st = c->eng.start(c->slot, rhs, p, tol, maxit, flags);
    if (st) return st;
    c->eng.t_k1.clear();
    c->eng.t_k2.clear();
    st = run_to_end(c->eng, c->slot, t0, stats);
    if (st < 0) return st;
    if (c->eng.timing) {
        average_nonempty(c->eng.t_k1, &c->last_k1, &c->last_n);
        int n2 = 0;
        average_nonempty(c->eng.t_k2, &c->last_k2, &n2);
        c->have_timing = true;
    }
    return st;
}

int pcg_solve_static(const pcg_grid_t *grid, const double *rho, const uint8_t *solid_mask,
                     const pcg_bc_t *bc, const pcg_opts_t *opts, const double *rhs, double *p,
                     double tol, int32_t maxit, pcg_stats_t *stats, void *hip_stream)
{
    int st = check_grid(grid);
    if (st) return st;
    int bm = 0;
    st = check_bc(bc, &bm);
    if (st) return st;
    st = check_opts(opts);
    if (st) return st;
    const int flags = opts ? opts->flags : 0;
    if (flags & PCG_FRACTIONS) return PCG_EINVAL;   // fractions need a context
    if (!rho || !rhs || !p) return PCG_EINVAL;
    if (!(tol > 0.0) || !std::isfinite(tol) || maxit < 0) return PCG_EINVAL;
    size_t need = 0;
    st = pcg_workspace_bytes(grid, opts, &need);
    if (st) return st;
    void *scr = nullptr;
    size_t cap = 0;
    hipError_t e = static_scratch(&scr, &cap);
    if (e != hipSuccess) return hip_fail(e, "static scratch address");
    if (need > cap) {
        g_hip_err = "pcg_solve_static: the grid needs " + std::to_string(need) +
                    " bytes of device memory, more than the " + std::to_string(cap) +
                    "-byte static scratch";
        return PCG_ENOMEM;
    }
    const auto t0 = Clock::now();
    HostMirror hm;
    Engine eng;
    st = eng.init(scr, cap, 1, opts, hip_stream, &hm);
    if (st) return st;
    int slot = -1;
    st = eng.prepare(grid, rho, solid_mask, bc, flags, &slot);
    if (st) return st;
    st = eng.start(slot, rhs, p, tol, maxit, flags & PCG_WARM_START);
    if (st) return st;
    return run_to_end(eng, slot, t0, stats);
}

int pcg_check_connectivity(const uint8_t *host_mask, const pcg_grid_t *grid,
                           const pcg_bc_t *bc)
{
    int st = check_grid(grid);
    if (st) return st;
    int bm = 0, per = 0;
    st = check_bc(bc, &bm, &per);
    if (st) return st;
    if (!host_mask) return bm ? PCG_OK : PCG_SINGULAR;   // one region
    const std::vector<uint32_t> bits =
        pack_mask_host(host_mask, grid->nx, (int64_t)grid->ny * grid->nz);
    const int kind = classify_regions(
        fluid_regions(bits.data(), grid->nx, grid->ny, grid->nz, bm, per));
    return kind < 0 ? kind : kind == 1 ? PCG_SINGULAR : PCG_OK;
}

int pcg_set_tile_rules(int32_t precision, int32_t table, int32_t n,
                       const int64_t *max_cells, const int32_t *tz, const int32_t *grid)
{
    if (precision != PCG_PREC_FP64 && precision != PCG_PREC_FP32_IR) return PCG_EINVAL;
    if (table < kTableSingle || table > kTableNarrow) return PCG_EINVAL;
    if (n < 1 || n > 64 || !max_cells || !tz) return PCG_EINVAL;
    std::vector<TileRule> rules;
    for (int i = 0; i < n; ++i) {
        if (tz[i] < 1 || max_cells[i] < 1) return PCG_EINVAL;
        if (i > 0 && max_cells[i] <= max_cells[i - 1]) return PCG_EINVAL;
        const int g = grid ? grid[i] : 0;
        if (g < 0) return PCG_EINVAL;
        rules.push_back({ max_cells[i], tz[i], g });
    }
    rules.back().max_cells = INT64_MAX;   // the last rule covers every size
    rules_of(precision, table) = rules;
    return PCG_OK;
}

int pcg_get_tile_rules(int32_t precision, int32_t table, int32_t cap,
                       int64_t *max_cells, int32_t *tz, int32_t *grid, int32_t *n_out)
{
    if (precision != PCG_PREC_FP64 && precision != PCG_PREC_FP32_IR) return PCG_EINVAL;
    if (table < kTableSingle || table > kTableNarrow) return PCG_EINVAL;
    if (!n_out || cap < 0) return PCG_EINVAL;
    const auto &rules = rules_of(precision, table);
    *n_out = (int32_t)rules.size();
    for (int i = 0; i < cap && i < (int)rules.size(); ++i) {
        if (max_cells) max_cells[i] = rules[i].max_cells;
        if (tz) tz[i] = rules[i].tz;
        if (grid) grid[i] = rules[i].grid;
    }
    return PCG_OK;
}

static int project_blocks(const SlotHost &S)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>((S.geo.n + 255) / 256, 4096));
}

int pcg_project(pcg_ctx_t *c, const double *p, double dt, double *u, double *v,
                double *w)
{
    return pcg_project_ex(c, p, dt, u, v, w, nullptr, nullptr, nullptr, 1.0, u, v, w);
}

int pcg_project_ex(pcg_ctx_t *c, const double *p, double dt, const double *au,
                   const double *av, const double *aw, const double *bu,
                   const double *bv, const double *bw, double weight, double *u,
                   double *v, double *w)
{
    if (!c || !p || !au || !av || !aw || !u || !v || !w) return PCG_EINVAL;
    if (!std::isfinite(dt) || !std::isfinite(weight)) return PCG_EINVAL;
    const bool add = bu || bv || bw;
    if (add && !(bu && bv && bw)) return PCG_EINVAL;
    Slot *ds = nullptr;
    int st = c->eng.slot_view(c->slot, &ds);
    if (st) return st;
    const SlotHost &S = c->eng.slots[c->slot];
    const double h = std::sqrt(S.h2);
    const double *a[3] = { au, av, aw };
    const double *b[3] = { bu, bv, bw };
    double *o[3] = { u, v, w };
    HIP_TRY(launch_project(ds, p, dt / h, weight, a, add ? b : nullptr, o,
                           project_blocks(S), c->eng.stream));
    return PCG_OK;
}

int pcg_rhs(pcg_ctx_t *c, double dt, const double *au, const double *av,
            const double *aw, const double *bu, const double *bv, const double *bw,
            double *rhs)
{
    if (!c || !au || !av || !aw || !rhs) return PCG_EINVAL;
    if (!std::isfinite(dt) || dt == 0.0) return PCG_EINVAL;
    const bool add = bu || bv || bw;
    if (add && !(bu && bv && bw)) return PCG_EINVAL;
    Slot *ds = nullptr;
    int st = c->eng.slot_view(c->slot, &ds);
    if (st) return st;
    const SlotHost &S = c->eng.slots[c->slot];
    const double *a[3] = { au, av, aw };
    const double *b[3] = { bu, bv, bw };
    HIP_TRY(launch_rhs(ds, std::sqrt(S.h2), dt, a, add ? b : nullptr, rhs,
                       project_blocks(S), c->eng.stream));
    return PCG_OK;
}

int pcg_set_fractions(pcg_ctx_t *c, const double *ax, const double *ay, const double *az,
                      const double *vol)
{
    if (!c) return PCG_EINVAL;
    return c->eng.set_fractions(c->slot, ax, ay, az, vol);
}

int pcg_update_density(pcg_ctx_t *c, const double *rho, const uint8_t *solid_mask,
                       int32_t flags)
{
    if (!c || !rho) return PCG_EINVAL;
    if (flags & ~(PCG_SKIP_CONNECTIVITY_CHECK | PCG_NO_DENSITY_CLASSES)) return PCG_EINVAL;
    return c->eng.refresh(c->slot, rho, solid_mask, flags);
}

int pcg_divergence(pcg_ctx_t *c, const double *u, const double *v, const double *w,
                   double *out)
{
    if (!c || !u || !v || !w || !out) return PCG_EINVAL;
    Slot *ds = nullptr;
    int st = c->eng.slot_view(c->slot, &ds);
    if (st) return st;
    const SlotHost &S = c->eng.slots[c->slot];
    // one partial pair per workgroup, in the slot's partial-sum buffer
    const int64_t blocks = std::max<int64_t>(
        1, std::min<int64_t>({ (S.geo.n + 255) / 256, 2048,
                               (int64_t)(kMaxPartials * S.geo.ntiles / 2) }));
    HIP_TRY(launch_divnorm(ds, 1.0 / std::sqrt(S.h2), u, v, w, S.partials, (int)blocks,
                           c->eng.stream));
    std::vector<double> part(2 * blocks);
    HIP_TRY(hipMemcpyAsync(part.data(), S.partials, part.size() * 8, hipMemcpyDeviceToHost,
                           c->eng.stream));
    HIP_TRY(hipStreamSynchronize(c->eng.stream));
    double ss = 0.0, mx = 0.0;
    for (int64_t b = 0; b < blocks; ++b) {
        ss += part[2 * b];
        mx = std::max(mx, part[2 * b + 1]);
    }
    out[0] = std::sqrt(ss);
    out[1] = mx;
    return PCG_OK;
}

int pcg_density_classes(const pcg_ctx_t *c, int32_t *nclasses)
{
    if (!c || !nclasses) return PCG_EINVAL;
    const SlotHost &S = c->eng.slots[c->slot];
    *nclasses = S.classes && !S.has_frac ? std::max(1, S.nclasses) : 0;
    return PCG_OK;
}

int pcg_tile_form(const pcg_ctx_t *c, int32_t *tx, int32_t *ty, int32_t *sweeps)
{
    if (!c || !tx || !ty || !sweeps) return PCG_EINVAL;
    const SlotHost &S = c->eng.slots[c->slot];
    *tx = S.geo.tx;
    *ty = S.geo.ty;
    *sweeps = S.z2 ? 1 : 2;
    return PCG_OK;
}

int pcg_destroy(pcg_ctx_t *c)
{
    delete c;
    return PCG_OK;
}

const char *pcg_strerror(int code)
{
    switch (code) {
    case PCG_OK: return "ok";
    case PCG_MAXIT: return "iteration limit reached";
    case PCG_PENDING: return "solve still running";
    case PCG_SINGULAR: return "one fluid region and no Dirichlet wall: solvable up to a constant";
    case PCG_EINVAL: return "invalid argument";
    case PCG_EDOMAIN: return "density not positive and finite in a fluid cell, or non-finite source";
    case PCG_ESINGULAR: return "a fluid region touches no Dirichlet wall and is not the only one";
    case PCG_EBREAKDOWN: return "conjugate-gradient breakdown (p.Ap <= 0 or not finite)";
    case PCG_ENOMEM: return "workspace or arena too small";
    case PCG_EBUSY: return "admission refused: no free slot or not enough arena memory";
    case PCG_EHIP: return "HIP runtime error";
    case PCG_EUNSUPPORTED: return "unsupported: periodic z walls or grid too large";
    default: return "unknown status";
    }
}

const char *pcg_last_hip_error(void) { return g_hip_err.c_str(); }

int pcg_inject_failure(pcg_ctx_t *c, int32_t after_steps)
{
    if (!c || after_steps < 0) return PCG_EINVAL;
    c->eng.fail_after = after_steps;
    return PCG_OK;
}

int pcg_set_timing(pcg_ctx_t *c, int32_t on)
{
    if (!c) return PCG_EINVAL;
    c->eng.timing = on != 0;
    c->eng.table_dirty = true;   // the launch form depends on it
    return PCG_OK;
}

int pcg_last_timing(pcg_ctx_t *c, double *ms_k1, double *ms_k2, int32_t *n)
{
    if (!c || !c->have_timing) return PCG_EINVAL;
    if (ms_k1) *ms_k1 = c->last_k1;
    if (ms_k2) *ms_k2 = c->last_k2;
    if (n) *n = c->last_n;
    return PCG_OK;
}

int pcg_batch_create(pcg_batch_t **out, void *arena, size_t arena_bytes,
                     int32_t max_slots, const pcg_opts_t *opts, void *hip_stream)
{
    if (!out) return PCG_EINVAL;
    *out = nullptr;
    if (max_slots < 1) return PCG_EINVAL;
    if (opts && (opts->flags & PCG_FRACTIONS)) return PCG_EINVAL;   // contexts only
    pcg_batch *b = new (std::nothrow) pcg_batch();
    if (!b) return PCG_ENOMEM;
    b->eng.is_batch = true;
    int st = b->eng.init(arena, arena_bytes, max_slots, opts, hip_stream);
    if (st) { delete b; return st; }
    *out = b;
    return PCG_OK;
}

int pcg_batch_footprint(const pcg_batch_t *b, const pcg_grid_t *grid,
                        size_t *out_bytes)
{
    if (!b || !out_bytes) return PCG_EINVAL;
    int st = check_grid(grid);
    if (st) return st;
    *out_bytes = align_up(b->eng.footprint(*grid), kAlign);
    return PCG_OK;
}

int pcg_batch_admit(pcg_batch_t *b, const pcg_grid_t *grid, const double *rho,
                    const uint8_t *mask, const pcg_bc_t *bc, const double *rhs,
                    double *p, double tol, int32_t maxit, int32_t flags,
                    int32_t *slot)
{
    if (!b || !slot || !rhs || !p) return PCG_EINVAL;
    if (!(tol > 0.0) || !std::isfinite(tol) || maxit < 0) return PCG_EINVAL;
    if (flags & ~(PCG_WARM_START | PCG_SKIP_CONNECTIVITY_CHECK | PCG_NO_DENSITY_CLASSES |
                  PCG_FLAT_TILES | PCG_PLANE_TILES | PCG_TWO_SWEEPS | PCG_NARROW_TILES))
        return PCG_EINVAL;
    int id = -1;
    int st = b->eng.prepare(grid, rho, mask, bc, flags, &id);
    if (st) return st;
    st = b->eng.start(id, rhs, p, tol, maxit, flags);
    if (st) { b->eng.release(id); return st; }
    *slot = id;
    return PCG_OK;
}

int pcg_batch_step(pcg_batch_t *b, int32_t replays, int32_t *active_out)
{
    if (!b || replays < 1) return PCG_EINVAL;
    int st = b->eng.step(replays);
    if (st) return st;
    if (active_out) *active_out = b->eng.running_count();
    return PCG_OK;
}

int pcg_batch_poll(pcg_batch_t *b, int32_t slot, pcg_stats_t *stats)
{
    if (!b || slot < 0 || slot >= b->eng.max_slots || !b->eng.slots[slot].used)
        return PCG_EINVAL;
    const SlotHost &S = b->eng.slots[slot];
    if (S.running) {
        if (stats) { std::memset(stats, 0, sizeof(*stats)); stats->status = PCG_PENDING; }
        return PCG_PENDING;
    }
    pcg_stats_t s;
    b->eng.fill_stats(slot, &s);
    if (stats) *stats = s;
    return s.status;
}

int pcg_batch_release(pcg_batch_t *b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->eng.max_slots || !b->eng.slots[slot].used)
        return PCG_EINVAL;
    b->eng.release(slot);
    return PCG_OK;
}

int pcg_batch_destroy(pcg_batch_t *b)
{
    delete b;   // the engine waits for its stream first
    return PCG_OK;
}

int pcg_copy_probe(const double *src, double *dst, size_t n, int32_t reps,
                   void *hip_stream, double *ms_per_copy)
{
    if (!src || !dst || n < 2 || reps < 1 || !ms_per_copy) return PCG_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    return time_launches(s, reps, [&] { return launch_copy(src, dst, n, s); }, ms_per_copy);
}

int pcg_triad_probe(double *a, const double *b, const double *c, size_t n, double scalar,
                    int32_t reps, void *hip_stream, double *ms_per_triad)
{
    if (!a || !b || !c || n < 2 || reps < 1 || !ms_per_triad) return PCG_EINVAL;
    if (a == b || a == c) return PCG_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    return time_launches(s, reps, [&] { return launch_triad(a, b, c, scalar, n, s); },
                         ms_per_triad);
}

}  // extern "C"
