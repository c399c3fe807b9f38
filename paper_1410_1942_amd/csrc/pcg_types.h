// Internal layout shared by the host engine and the device kernels.
//
// A "slot" is one resident solve.  Every launch covers all tiles of all
// active slots; each slot carries its own scalars and a small state machine
// that the last-arriving workgroup of a launch advances.  A single solve is
// a batch of one slot.
#pragma once
#include <stdint.h>

namespace pcgmi {

constexpr int kBlock = 256;       // threads per workgroup = cells per plane tile
constexpr int kMaxPartials = 3;   // reduction values per tile

// 2-D plane tiles of the LDS-staged passes: kTileY rows of kTileX columns
// for FP64 (two cells per thread), of 2 kTileX columns for FP32 (four)
constexpr int kTileX = 128;
constexpr int kTileY = 4;

// Bytes of the device array behind the allocation-free entry point.
constexpr unsigned long long kStaticScratchBytes = 64ull << 20;

// Density classes: up to kMaxFluidClasses distinct fluid densities get a
// one-byte class; kClsWallD stands for a Dirichlet wall (density 0 in the
// face formula), kClsSolid for hull cells and Neumann walls (density +inf).
constexpr int kClasses = 16;
constexpr int kMaxFluidClasses = 14;
constexpr int kClsWallD = 14;
constexpr int kClsSolid = 15;

// Next action of a slot.  Launches alternate K1, K2, K1, K2, ...; a K1
// action is always followed by a K2 action and vice versa.
enum Phase : int32_t {
    PH_IDLE = 0,       // empty slot or finished solve: no work, no state change
    // K1 actions (first launch of an iteration)
    K1_INIT64 = 1,     // b = -h^2 Sigma, x = 0 (or r = b - A x0), z = D^-1 r
    K1_CG_A = 2,       // p = z + beta p ; p.Ap
    K1_CHECK64 = 3,    // true residual ||b - A x||
    K1_IR_INIT = 4,    // ||b||, x = 0 (or solids zeroed), d = 0
    K1_IR_RESID = 5,   // r = b - A (x + s d) in FP64, z32 = D32^-1 (scale r)
    K1_IR_A = 6,       // FP32 p = z + beta p ; p.Ap (FP64 sum)
    K1_MEAN_B = 7,     // singular problem: sum of b and count of fluid cells
    K1_MEAN_X = 8,     // singular problem: sum of x over fluid cells
    K1_FLUSH_X = 9,    // x += alpha p: the updates the last iterations left pending
    // K2 actions (second launch of an iteration)
    K2_NONE = 11,      // nothing; then the K1 action in `after`
    K2_CG_B = 12,      // q = A p, x += alpha p (three at a time), z -= alpha D^-1 q ; r.z, r.r
    K2_IR_B = 13,      // FP32 q = A p, d += alpha p (three at a time), z -= alpha D^-1 q ; r.z, r.r (FP64)
    K2_IR_UPDATE = 14, // x += s d, d = 0
    K2_ZERO_X = 15,    // x = 0 (zero source with a warm start)
    K2_SUB_X = 16,     // singular problem: x -= its fluid mean
    K2_CG_F = 17,      // one-sweep iteration: p = z + beta p, q = A p, x += alpha p
                       // (three at a time), z' = z - alpha D^-1 q ; r.z, r.r, z'.A z'
    K2_IR_F = 18,      // the same for the FP32 inner solve (d in place of x; FP64 sums)
    PH_DONE = 20
};

// Device-resident, mutated only by the last workgroup of each launch.
struct alignas(128) SlotState {
    double rz;        // r.z of the current iterate (preconditioned)
    double pap;       // p.A p
    double alpha, beta;
    double bb;        // ||b||^2
    double tol2;      // tol^2 * ||b||^2
    double rr;        // recursive ||r||^2 (FP64) or inner ||r||^2 (IR)
    double rr_true;   // last FP64 recomputed ||b - A x||^2
    double rr0_inner; // IR: ||r||^2 at the start of the inner solve
    double inner_tol2;// IR: (inner reduction)^2
    double scale;     // IR: power-of-two scale of the current inner system
    double upd_s;     // IR: multiplier of the pending update x += upd_s * d
    double tol;
    double inner_goal2; // IR: (reduction asked of the current inner solve)^2
    double bshift;    // singular problem: mean of b over fluid cells (else 0)
    double nfluid;    // singular problem: number of fluid cells
    double xshift;    // singular problem: mean of x over fluid cells
    // alphas of the directions whose x updates are pending, oldest first
    double alpha_p0, alpha_p1;
    int32_t phase;
    int32_t after;    // K1 action after a K2_NONE
    int32_t status;   // PCG_PENDING while running, else the final code
    int32_t iter;     // CG iterations (inner iterations for IR)
    int32_t outer;    // IR refinement trips
    int32_t inner_iter;
    int32_t maxit, inner_maxit;
    int32_t first;    // next pass A uses beta = 0
    int32_t pbuf;     // which of the three p buffers holds the current direction
    int32_t final_upd;// IR: the pending update is the last one
    uint32_t ticket;  // arrivals of the current launch
    int32_t warm;     // warm start requested
    int32_t singular; // no Dirichlet face: solve for the mean-free source
    int32_t xpend;    // earlier iterations whose x (FP64) or d (IR) update is pending: 0..2
    int32_t fused;    // iterations run as one sweep (K2_CG_F, K2_IR_F)
    int32_t zsel;     // one-sweep iterations: z is in Slot::z2 (1) or Slot::z (0)
};

// Read-only description of a slot (rewritten by the host between replays).
struct Slot {
    int32_t nx, ny, nz;
    int32_t bcmask;        // bit f set: wall f is Dirichlet (x-,x+,y-,y+,z-,z+)
    int32_t plane_tiles;   // ceil(nx*ny / (cpt kBlock)), or tiles_x * ceil(ny / ty)
    int32_t ztiles;        // ceil(nz / tz)
    int32_t tz;            // planes per tile
    int32_t permask;       // bit 0: periodic x walls, bit 1: periodic y walls
    int32_t cpt;           // cells per thread: 1, or 2/4 adjacent columns (nx divisible)
    // 0: a tile is cpt * kBlock consecutive cells of a plane; else a 2-D
    // plane tile of tx columns x ty rows (tx ty = cpt kBlock), tiles_x of
    // them across a row, served by the LDS-staged pass B
    int32_t tx, ty, tiles_x;
    int64_t tile_begin;    // first global tile of this slot
    int64_t ntiles;        // plane_tiles * ztiles
    double h2;             // h*h
    const double *rhs;     // caller's Sigma
    double *x;             // caller's p (the CG iterate)
    const double *rho64;   // density, +inf in solid cells
    const float *rho32;    // IR only
    void *z;               // D^-1 r   (double, or float for IR)
    // second z buffer of the one-sweep iteration, or null: a sweep reads z
    // in its neighbours' tiles while they write theirs, so it reads one
    // buffer and writes the other
    void *z2;
    // search directions, rotating: pass A reads buffer b and writes b + 1
    // (mod 3), so the two directions before the current one stay readable
    void *dir0, *dir1, *dir2;
    float *d32;            // IR inner correction
    double *partials;      // kMaxPartials * ntiles
    SlotState *st;
    const uint8_t *cls;    // density class per cell, or null (density path)
    const double *tab64;   // kClasses^2 face coefficients 2/(rho_a + rho_b)
    const float *tab32;    // the same in FP32 (FP32+IR only)
    // free-slip cut cells, or null: area fractions on the MAC faces
    // (ax [nz][ny][nx+1], ay [nz][ny+1][nx], az [nz+1][ny][nx]) and volume
    // fractions per cell
    const double *ax, *ay, *az, *vol;
};

struct BatchHeader {
    int64_t total_tiles;
    int32_t nslots;
    // 0: workgroups stride over the tiles (tiles running at the same time
    // are neighbours, sharing y-halo rows in L2; one solve); 1: each
    // workgroup takes a contiguous range of tiles, so it meets few slots
    // per launch (several solves)
    int32_t chunked;
    // 1: every resident solve runs one sweep per iteration and only
    // second-half launches are issued; they also serve the rare first-half
    // actions (set-up, the first pass A, residuals, flushes)
    int32_t k2only;
    int32_t pad_;
};

}  // namespace pcgmi
