/*
 * pcg.h -- C ABI of the MI355X pressure-projection solver.
 *
 * The library solves the variable-coefficient pressure equation of the
 * cartesian-grid ship-wave method (Section 2, Eq. pois):
 *
 *     d/dx_i ( (1/rho) dP/dx_i ) = Sigma
 *
 * on a uniform grid of nx*ny*nz cubic cells of edge h, by Jacobi-
 * preconditioned conjugate gradients (the Introduction names a
 * preconditioned conjugate-gradient solver for this equation).  The solution
 * is the pressure used to project the velocity onto a solenoidal field
 * (Section 2.1, first and second Runge-Kutta stages).
 *
 * Discretisation (cell-centred pressure and density):
 *   - face coefficient between fluid cells c, n: beta = 1/((rho_c+rho_n)/2);
 *   - a face touching a hull ("solid") cell carries beta = 0: the binary
 *     form of the finite-volume free-slip hull (Section 2.2.1); solid cells
 *     get p = 0 and their rhs is ignored;
 *   - a Neumann wall carries beta = 0; a Dirichlet wall imposes p = 0 on the
 *     face (the zero reduced pressure at the walls, Section 2.4.2) with
 *     beta = 1/rho_c and the mirrored ghost value -p_c;
 *   - (L p)_c = h^-2 [ sum_n beta_cn (p_n - p_c) - 2 sum_D beta_c p_c ].
 * A solve succeeds when ||Sigma - L p||_2 <= tol * ||Sigma||_2 over fluid
 * cells.  The solution is unique iff every connected fluid region touches a
 * Dirichlet wall.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller,
 * C-ordered [nz][ny][nx] (x fastest; cell (i,j,k) at (k*ny + j)*nx + i),
 * unless marked "host".  The library never allocates device memory: it
 * carves what it needs out of a caller-provided workspace or arena.  It does
 * allocate small pinned host buffers (status mirrors) and hipGraph objects.
 *
 * Streams: all device work of a context or batch is ordered on the HIP
 * stream passed at creation (NULL = the legacy default stream).  Calls on
 * one context or batch must not overlap in time (not thread-safe).
 *
 * Errors: every function returns an int status; no exception crosses the
 * ABI.  0 is success, positive values are non-fatal conditions, negative
 * values are errors.  pcg_strerror() gives a static description;
 * pcg_last_hip_error() gives the text of the last HIP runtime failure.
 */
#ifndef PCG_MI355X_H
#define PCG_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
enum {
    PCG_OK = 0,
    PCG_MAXIT = 1,        /* iteration cap reached; p holds the last iterate */
    PCG_PENDING = 2,      /* batched solve still running                     */
    PCG_SINGULAR = 3,     /* pcg_check_connectivity: one fluid region and no
                             Dirichlet wall; solvable up to a constant       */
    PCG_EINVAL = -1,      /* null pointer, n < 1, h <= 0, tol <= 0, ...      */
    PCG_EDOMAIN = -2,     /* rho <= 0 or non-finite in a fluid cell, or a
                             non-finite rhs                                  */
    PCG_ESINGULAR = -3,   /* a fluid region touches no Dirichlet wall while
                             another region exists                           */
    PCG_EBREAKDOWN = -4,  /* p.Ap <= 0 or non-finite during the iteration    */
    PCG_ENOMEM = -5,      /* workspace / arena too small                     */
    PCG_EBUSY = -6,       /* admission refused: over the memory budget or no
                             free slot; retry after a release                */
    PCG_EHIP = -7,        /* HIP runtime failure (see pcg_last_hip_error)     */
    PCG_EUNSUPPORTED = -8 /* periodic z walls, or a grid above the size
                             limits (n >= 2^31 cells, or nx*ny*24 bytes
                             above 2^32)                                     */
};

/* ---- problem description --------------------------------------------- */
typedef struct {
    int32_t nx, ny, nz; /* cells along x, y, z (each >= 1)                   */
    double h;           /* cell edge (> 0)                                   */
} pcg_grid_t;

/*
 * Wall kinds.  Neumann: no flux (beta = 0).  Dirichlet: p = 0 on the wall
 * face (mirrored ghost -p_c, coefficient 1/rho_c).  Periodic (the strut case
 * of Section 3 is periodic along x): both walls of the x or of the y axis,
 * joining the last and the first cell of every row by an ordinary face; an
 * axis of one cell carries no flux across it.  Periodic z is unsupported.
 *
 * With no Dirichlet wall reaching the fluid (no-flux and periodic walls
 * only) the operator is singular, its null vector the constant over the
 * fluid cells.  When all fluid cells form one region the library solves
 * for the source with its mean over fluid cells removed and returns the
 * solution of zero mean over fluid cells; the relative residual is measured
 * against that mean-free source.  Several regions without a Dirichlet wall
 * (or such a region beside an anchored one) are refused (PCG_ESINGULAR).
 */
enum { PCG_BC_NEUMANN = 0, PCG_BC_DIRICHLET = 1, PCG_BC_PERIODIC = 2 };

typedef struct {
    int32_t kind[6];    /* walls in the order x-, x+, y-, y+, z-, z+         */
} pcg_bc_t;

enum { PCG_PREC_FP64 = 0, PCG_PREC_FP32_IR = 1 };

enum {
    PCG_WARM_START = 1,              /* p holds an initial guess on entry    */
    PCG_SKIP_CONNECTIVITY_CHECK = 2, /* skip the host flood fill of the mask:
                                        the problem is taken as anchored when
                                        a Dirichlet wall exists, else as one
                                        singular region                      */
    PCG_NO_DENSITY_CLASSES = 4,      /* always read the FP64/FP32 density per
                                        cell; by default a field with at most
                                        14 distinct fluid densities is coded
                                        as one byte per cell plus a table of
                                        exact face coefficients (same
                                        operator, fewer bytes per iteration) */
    PCG_FRACTIONS = 8,               /* reserve workspace for free-slip cut-cell
                                        fractions (pcg_set_fractions; single
                                        contexts only)                       */
    PCG_FLAT_TILES = 16,             /* keep tiles of consecutive cells: by
                                        default a grid runs 128 x 4 (FP64)
                                        or 256 x 4 (FP32_IR) plane tiles
                                        with the operator's in-plane
                                        neighbours staged in LDS where its
                                        rows are of cell pairs (FP64) or
                                        quads (FP32_IR), a periodic y axis
                                        holds whole tile rows, and the rows
                                        hold whole tiles or, with walls on
                                        x, keep at least 70% (FP64) or 50%
                                        (FP32_IR) of the lanes of their
                                        tiles busy; same operator, another
                                        summation order                     */
    PCG_PLANE_TILES = 32,            /* plane tiles also where rows of pairs
                                        or quads keep fewer lanes busy (a
                                        periodic x or y axis still needs
                                        whole tiles); PCG_FLAT_TILES wins if
                                        both                                 */
    PCG_TWO_SWEEPS = 64,             /* on plane tiles, keep two sweeps per
                                        iteration.  By default a solve on
                                        plane tiles (FP64, and the FP32
                                        inner iterations of FP32_IR) runs
                                        one sweep per iteration (the
                                        Chronopoulos-Gear recurrences: the
                                        same iterates up to rounding, 33
                                        instead of 50 bytes per cell and
                                        FP64 iteration before the x
                                        updates) with a second z vector in
                                        the workspace (8 bytes per cell, 4
                                        for FP32_IR)                         */
    PCG_NARROW_TILES = 128           /* 64 x 4 plane tiles of one cell a
                                        thread with one sweep per iteration
                                        wherever the wide plane tiles are
                                        not taken.  By default they are
                                        taken in batches, on rows of an odd
                                        length, and for single solves of at
                                        most 2^18 cells; not with
                                        PCG_TWO_SWEEPS, PCG_FLAT_TILES or
                                        fractions.  A periodic x axis needs
                                        rows of whole 64-cell tiles         */
};

/*
 * Options.  Zero-initialised fields take the defaults in brackets.
 *   precision   PCG_PREC_FP64 [default] or PCG_PREC_FP32_IR: FP32 stencil
 *               and vectors inside, FP64 residual, dot products, alpha/beta
 *               and solution update (iterative refinement).
 *   check_every iterations per captured graph replay between host polls [32]
 *   flags       PCG_WARM_START | PCG_SKIP_CONNECTIVITY_CHECK |
 *               PCG_NO_DENSITY_CLASSES | PCG_FRACTIONS | PCG_FLAT_TILES |
 *               PCG_PLANE_TILES | PCG_TWO_SWEEPS
 *   inner_maxit FP32_IR: cap on inner iterations per refinement trip [none]
 *   inner_tol   FP32_IR: relative reduction asked of each inner solve, never
 *               more than the last refinement trip needs [1e-4]
 *   tz          cells per tile along z; 0 = chosen by the autotuner table
 *   grid_blocks workgroups per launch; 0 = chosen by the autotuner table
 */
typedef struct {
    int32_t precision;
    int32_t check_every;
    int32_t flags;
    int32_t inner_maxit;
    double inner_tol;
    int32_t tz;
    int32_t grid_blocks;
} pcg_opts_t;

/* Per-solve statistics (host structure). */
typedef struct {
    int32_t status;           /* PCG_* code of the solve                     */
    int32_t iters;            /* CG iterations (inner iterations for IR)     */
    int32_t outer_iters;      /* refinement trips (IR), 0 for FP64           */
    double rel_res_true;      /* ||b - A p|| / ||b|| recomputed in FP64      */
    double rel_res_recursive; /* last recursive residual of the iteration    */
    double ms;                /* wall time of the call (pcg_solve), or from
                                 admission to completion (batched)           */
} pcg_stats_t;

typedef struct pcg_ctx pcg_ctx_t;     /* opaque, owned by the library */
typedef struct pcg_batch pcg_batch_t; /* opaque, owned by the library */

/* ---- single solve ----------------------------------------------------- */

/*
 * Bytes of device workspace pcg_setup needs for this grid and options.
 * Returns PCG_EINVAL on bad arguments, PCG_EUNSUPPORTED when
 * nx*ny*nz >= 2^31.
 */
int pcg_workspace_bytes(const pcg_grid_t *grid, const pcg_opts_t *opts,
                        size_t *out_bytes);

/*
 * Prepare a solver for one density field (Eq. density gives rho from the
 * volume fraction; here rho is given directly).
 *   rho        device f64[n]: density per cell (> 0 and finite in fluid cells)
 *   solid_mask device u8[n]: 1 = hull cell, 0 = fluid; NULL = no hull
 *   bc         host: the six wall kinds
 *   opts       host, may be NULL (defaults)
 *   workspace  device buffer of at least pcg_workspace_bytes(), 256-byte
 *              aligned, owned by the caller and kept alive until pcg_destroy
 *   hip_stream hipStream_t the context works on (NULL = default stream)
 * rho and solid_mask are read during the call and not retained.  Errors:
 * EINVAL, EDOMAIN (checked on the device), ESINGULAR (host flood fill of the
 * mask unless PCG_SKIP_CONNECTIVITY_CHECK), ENOMEM, EUNSUPPORTED, EHIP.
 */
int pcg_setup(pcg_ctx_t **out, const pcg_grid_t *grid, const double *rho,
              const uint8_t *solid_mask, const pcg_bc_t *bc,
              const pcg_opts_t *opts, void *workspace, size_t ws_bytes,
              void *hip_stream);

/*
 * Solve L p = rhs to relative residual tol with at most maxit iterations.
 *   rhs   device f64[n]: the source Sigma (values in solid cells ignored);
 *         must stay unchanged during the call
 *   p     device f64[n]: output pressure (0 in solid cells); input guess
 *         when the context was set up with PCG_WARM_START
 *   stats host, may be NULL
 * Blocks until the solve is complete.  Returns PCG_OK, PCG_MAXIT (p holds
 * the last iterate, usable as a warm start), or an error (EINVAL, EDOMAIN
 * for a non-finite rhs, EBREAKDOWN, EHIP).  A zero rhs gives p = 0 after
 * zero iterations.
 */
int pcg_solve(pcg_ctx_t *ctx, const double *rhs, double *p, double tol,
              int32_t maxit, pcg_stats_t *stats);

/*
 * pcg_solve with the warm start chosen per call: flags 0 (x0 = 0) or
 * PCG_WARM_START (x0 = p on entry), whatever the setup flags said.  The
 * second stage of the Runge-Kutta step (Section 2.1) starts from the
 * first-stage pressure P*, which solves a nearby equation.  Other flag bits
 * give PCG_EINVAL.
 */
int pcg_solve_ex(pcg_ctx_t *ctx, const double *rhs, double *p, double tol,
                 int32_t maxit, int32_t flags, pcg_stats_t *stats);

/*
 * Host-side analysis of the connected regions of fluid cells (face
 * adjacency, periodic faces included, mask == 0).  host_mask is a HOST u8[n]
 * array (1 = hull; NULL = no hull).  Returns PCG_OK when every region
 * touches a Dirichlet wall (unique solution), PCG_SINGULAR for a single
 * region touching none (solved up to a constant, see the wall kinds),
 * PCG_ESINGULAR otherwise, or PCG_EINVAL / PCG_EUNSUPPORTED for a bad grid
 * or wall kinds.  pcg_setup and pcg_batch_admit run the same analysis unless
 * PCG_SKIP_CONNECTIVITY_CHECK.
 */
int pcg_check_connectivity(const uint8_t *host_mask, const pcg_grid_t *grid,
                           const pcg_bc_t *bc);

/*
 * Number of density classes the context codes its field with (1..14), or 0
 * when it reads a density per cell (more distinct densities than classes,
 * or PCG_NO_DENSITY_CLASSES).
 */
int pcg_density_classes(const pcg_ctx_t *ctx, int32_t *nclasses);

/*
 * Tile form of a context: *tx, *ty = columns and rows of its 2-D plane tiles
 * (128 x 4 FP64, 256 x 4 FP32, 64 x 4 narrow tiles), or 0, 0 when its tiles are runs of
 * consecutive cells; *sweeps = passes over the grid per iteration (1: the
 * one-sweep iteration on plane tiles, else 2).  PCG_EINVAL for null
 * arguments.
 */
int pcg_tile_form(const pcg_ctx_t *ctx, int32_t *tx, int32_t *ty, int32_t *sweeps);

/*
 * Velocity projection (Section 2.1: u* = u - dt (1/rho) grad P on the MAC
 * faces), in place, with the context's face coefficients, walls and hull:
 *   u_f -= dt * beta_f * (p_hi - p_lo) / h,
 * Dirichlet walls with the mirrored ghost -p_c, Neumann and hull faces
 * untouched.  With Sigma = (D u)/dt and p solved to tol, the projected field
 * has ||D u_new|| = dt ||Sigma - L p|| <= tol dt ||Sigma||.
 *   p  device f64[n] (pressure from pcg_solve)
 *   u  device f64[nz][ny][nx+1], v f64[nz][ny+1][nx], w f64[nz+1][ny][nx]
 * Stream-ordered on the context's stream; returns after the launch.
 */
int pcg_project(pcg_ctx_t *ctx, const double *p, double dt, double *u, double *v,
                double *w);

/*
 * Both velocity updates of the two-stage Runge-Kutta step (Section 2.1,
 * the first-stage prediction u* and the second-stage average u^{k+1}), with
 * the context's current face coefficients:
 *   out_f = weight * (a_f [+ b_f] - dt * beta_f * (p_hi - p_lo) / h)
 * on every MAC face, walls and hull as in pcg_project (which is this call
 * with b absent, weight 1 and out = a).  First stage: a = u^k, b absent,
 * weight 1, p = P*.  Second stage (after pcg_update_density to rho(phi*)):
 * a = u*, b = u^k, weight 1/2, p = P^{k+1}.
 *   a, b  device face triples (u f64[nz][ny][nx+1], v f64[nz][ny+1][nx],
 *         w f64[nz+1][ny][nx]); b all NULL or all set
 *   out   device face triple; may be the same arrays as a (or b), not
 *         partly overlapping them
 * PCG_EINVAL for a NULL array, a partial b, non-finite dt or weight, or a
 * context whose coefficients are not valid.  Stream-ordered; returns after
 * the launch.
 */
int pcg_project_ex(pcg_ctx_t *ctx, const double *p, double dt, const double *au,
                   const double *av, const double *aw, const double *bu,
                   const double *bv, const double *bw, double weight, double *u,
                   double *v, double *w);

/*
 * Source term of either stage's pressure equation (Section 2.1, the
 * right-hand sides of the two Poisson equations with the remaining terms R
 * set to zero): rhs_c = (D U)_c / dt with U = a [+ b], i.e.
 *   rhs_c = ((U_{i+1/2} - U_{i-1/2}) + (V_{j+1/2} - V_{j-1/2})
 *            + (W_{k+1/2} - W_{k-1/2})) / h / dt
 * in fluid cells and 0 in hull cells.  First stage a = u^k; second stage
 * a = u*, b = u^k.  Face triples as in pcg_project_ex; rhs device f64[n].
 * PCG_EINVAL for NULL arrays, a partial b, dt zero or non-finite.
 * Stream-ordered; returns after the launch.
 */
int pcg_rhs(pcg_ctx_t *ctx, double dt, const double *au, const double *av,
            const double *aw, const double *bu, const double *bv, const double *bw,
            double *rhs);

/*
 * Free-slip cut cells (Section 2.2.1: the hull's area fractions A and volume
 * fractions V enter the Poisson equation and the projection).  With
 * fractions every face coefficient, wall faces included, is weighted by the
 * face's open area and the equation holds in finite-volume form,
 *   (1/(V_c h^2)) sum_f A_f beta_f (p_n - p_c) = Sigma_c,
 * so the scaled system is sum_f A_f beta_f (p_c - p_n) = -h^2 V_c Sigma_c
 * and the reported relative residual is its (volume-weighted) one.  The
 * source and divergence entry points then weight every face velocity by its
 * area fraction and divide the cell sum by V_c; the projection keeps its
 * form.  The hull mask still marks the cells with no fluid; fractions
 * describe the rest.
 *   ax device f64[nz][ny][nx+1], ay f64[nz][ny+1][nx], az f64[nz+1][ny][nx]:
 *      area fractions in [0, 1] of the MAC faces (same layout as the face
 *      velocities; on a periodic axis face 0 is the shared face)
 *   vol device f64[n]: volume fractions, in (0, 1] on fluid cells
 * The arrays are copied into the workspace (set up with PCG_FRACTIONS, else
 * PCG_EINVAL) and validated on the device (PCG_EDOMAIN when out of range, and
 * the context then has no fractions).  All four NULL returns the context to
 * the binary hull.  While fractions are set the density is read per cell
 * (no density classes).  Blocks until done.
 */
int pcg_set_fractions(pcg_ctx_t *ctx, const double *ax, const double *ay, const double *az,
                      const double *vol);

/*
 * Rebuild the context's face coefficients in place for a new density field
 * (and hull mask) on the same grid and walls: the second stage solves with
 * rho(phi*) instead of rho(phi^k) (Section 2.1).  Same input rules and
 * checks as pcg_setup (flags: PCG_SKIP_CONNECTIVITY_CHECK,
 * PCG_NO_DENSITY_CLASSES; the setup flags no longer apply to the field).
 * The workspace and any previous solution array are untouched, so a
 * following pcg_solve may warm-start from the last pressure.  On error the
 * context keeps no valid coefficients and every call that needs them returns
 * PCG_EINVAL until a rebuild succeeds.  Blocks until done.
 */
int pcg_update_density(pcg_ctx_t *ctx, const double *rho, const uint8_t *solid_mask,
                       int32_t flags);

/*
 * Discrete divergence of MAC face velocities over the fluid cells (the form
 * of Eq. mass used by the projection): out[0] = ||D u||_2, out[1] =
 * max |D u|.  out is HOST double[2].  Blocks until done.
 */
int pcg_divergence(pcg_ctx_t *ctx, const double *u, const double *v,
                   const double *w, double *out);

/* Wait for the context's stream, then release the context (not the
 * workspace).  NULL is accepted. */
int pcg_destroy(pcg_ctx_t *ctx);

/* Static text for a status code. */
const char *pcg_strerror(int code);

/* Text of the last HIP runtime error seen by the library on this thread. */
const char *pcg_last_hip_error(void);

/* ---- batched and served solves ---------------------------------------- */

/*
 * A batch keeps several independent solves resident on the device and
 * advances all of them together: every launch covers the tiles of every
 * active solve, and each solve's iterations are captured once in a hipGraph
 * and replayed.  Solves may be admitted and released between steps
 * (continuous batching).  A solve's arithmetic depends only on its own
 * grid, tile shape and data, so its result is bitwise the same alone or in
 * any mix.
 *
 *   arena       device buffer owned by the caller; admission succeeds only
 *               while the sum of the resident solves' footprints fits in it
 *   arena_bytes its size
 *   max_slots   most solves resident at once (>= 1)
 *   opts        precision and tiling for every solve of the batch
 */
int pcg_batch_create(pcg_batch_t **out, void *arena, size_t arena_bytes,
                     int32_t max_slots, const pcg_opts_t *opts,
                     void *hip_stream);

/* Device bytes one solve of this grid occupies in a batch's arena. */
int pcg_batch_footprint(const pcg_batch_t *b, const pcg_grid_t *grid,
                        size_t *out_bytes);

/*
 * Admit one solve.  rho, mask (NULL = none) are read during the call;
 * rhs and p must stay valid until the solve is released.  flags: any of
 * PCG_WARM_START, PCG_SKIP_CONNECTIVITY_CHECK and PCG_NO_DENSITY_CLASSES,
 * with their pcg_setup / pcg_solve_ex meanings; others are PCG_EINVAL.
 * Returns PCG_EBUSY when the footprint does not fit in the free arena space
 * or no slot is free, and validation errors as pcg_setup.  On success *slot
 * names it.
 */
int pcg_batch_admit(pcg_batch_t *b, const pcg_grid_t *grid, const double *rho,
                    const uint8_t *mask, const pcg_bc_t *bc, const double *rhs,
                    double *p, double tol, int32_t maxit, int32_t flags,
                    int32_t *slot);

/*
 * Run `replays` captured graphs of check_every iterations each over every
 * active solve, then refresh the host mirror of every solve's status.
 * Blocks until the work is done.  *active_out (may be NULL) receives the
 * number of solves still running.
 */
int pcg_batch_step(pcg_batch_t *b, int32_t replays, int32_t *active_out);

/*
 * Status of one admitted solve, as of the last pcg_batch_step: returns
 * PCG_PENDING while it runs, else its final code (PCG_OK, PCG_MAXIT or an
 * error), and fills *stats (host; may be NULL) with its iterations, outer
 * trips, residuals and wall time (status PCG_PENDING and zeros while it
 * runs).  A finished solve's p holds its result.  PCG_EINVAL for a null
 * batch or a slot that is not admitted.
 */
int pcg_batch_poll(pcg_batch_t *b, int32_t slot, pcg_stats_t *stats);

/*
 * Free a slot and its arena space, finished or not (a running solve is
 * dropped: its p is left as the last step wrote it).  The slot number may
 * be reused by a later admission.  PCG_EINVAL for a null batch or a slot
 * that is not admitted.
 */
int pcg_batch_release(pcg_batch_t *b, int32_t slot);

/*
 * Wait for the batch's stream, then free the batch and its host and graph
 * resources; the arena belongs to the caller and is not freed.  NULL is
 * accepted.
 */
int pcg_batch_destroy(pcg_batch_t *b);

/* ---- tile shapes ------------------------------------------------------- */

/*
 * Tables consulted when opts.tz (or opts.grid_blocks) is 0: a solve of n
 * cells uses the first rule with n <= max_cells[i]: tile height tz[i] and,
 * for single-solve contexts, grid[i] workgroups (0 = library default).
 * Rules must be ordered by increasing max_cells, 1 <= n <= 64, tz >= 1.
 * There are four tables per precision: table = 0 for single-solve
 * contexts on tiles of consecutive cells, 1 for batches (any tile form),
 * where many resident solves already fill the device and longer tiles cost
 * less per-tile overhead, 2 for single-solve contexts on wide 2-D plane
 * tiles and 3 for single-solve contexts on narrow ones (64 x 4).  Contexts
 * and batches created afterwards use them.  A
 * solve's tile height depends only on its own cell count, so its result
 * does not depend on the other solves of a batch.  Host-only; not
 * thread-safe against concurrent setup.  pcg_get_tile_rules copies at most
 * cap rules out and sets *n_out to the table length.
 */
int pcg_set_tile_rules(int32_t precision, int32_t table, int32_t n,
                       const int64_t *max_cells, const int32_t *tz,
                       const int32_t *grid);
int pcg_get_tile_rules(int32_t precision, int32_t table, int32_t cap,
                       int64_t *max_cells, int32_t *tz, int32_t *grid,
                       int32_t *n_out);

/*
 * Test hook for the error path of pcg_solve / pcg_solve_ex: the
 * after_steps-th host polling step of the next solve on this context reports
 * PCG_EHIP (message "failure injected by pcg_inject_failure") without
 * touching the device; 0 disarms it.  A solve that ends in a host-side
 * error (this one, a runtime error, or a solve that stopped advancing)
 * waits for the context's stream and leaves the context usable: the next
 * pcg_solve starts normally.  PCG_EINVAL for a null context or
 * after_steps < 0.
 */
int pcg_inject_failure(pcg_ctx_t *ctx, int32_t after_steps);

/* ---- allocation-free solve ---------------------------------------------- */

/*
 * One solve that allocates nothing, for callers that cannot allocate device
 * or pinned memory (code that must not call hipMalloc, tight serving loops,
 * harnesses that forbid allocation).  Same problem, arguments and results
 * as pcg_setup + pcg_solve + pcg_destroy on the stream given (opts may be
 * NULL; flags as for pcg_setup except PCG_FRACTIONS, which is refused with
 * PCG_EINVAL, plus PCG_WARM_START to start from p), but the workspace is a
 * fixed 64 MiB device array inside the library (one per GPU, held until the
 * process ends; pcg_workspace_bytes gives a grid's need) and the iterations
 * are launched directly, without a captured graph.  No HIP allocation,
 * stream, event or graph routine is called; host bookkeeping uses a few
 * small ordinary heap blocks.  A grid whose workspace exceeds the array
 * returns PCG_ENOMEM (pcg_last_hip_error names both sizes).  All calls on
 * one GPU share the array, so calls that overlap on one GPU (from several
 * host threads, or on several streams) race and must be serialised by the
 * caller.  Returns after completion like pcg_solve, with its status codes.
 */
int pcg_solve_static(const pcg_grid_t *grid, const double *rho, const uint8_t *solid_mask,
                     const pcg_bc_t *bc, const pcg_opts_t *opts, const double *rhs, double *p,
                     double tol, int32_t maxit, pcg_stats_t *stats, void *hip_stream);

/* ---- measurement helpers ---------------------------------------------- */

/*
 * Kernel timing of pcg_solve.  After pcg_set_timing(ctx, 1) the solve
 * launches its two iteration kernels directly (not through the captured
 * graph) with a hipEvent recorded on the context's stream around each
 * launch; pcg_last_timing then gives the average duration (ms) of the first
 * (direction update + p.Ap) and second (operator apply + vector update +
 * dots) kernel over the launches that did work, and how many first-kernel
 * launches were averaged.  PCG_EINVAL when no timed solve has run.
 */
int pcg_set_timing(pcg_ctx_t *ctx, int32_t on);
int pcg_last_timing(pcg_ctx_t *ctx, double *ms_k1, double *ms_k2,
                    int32_t *launches);

/*
 * Copy-kernel bandwidth probe: copies n doubles src -> dst `reps` times on
 * the given stream and returns the average ms per copy.
 */
int pcg_copy_probe(const double *src, double *dst, size_t n, int32_t reps,
                   void *hip_stream, double *ms_per_copy);

/*
 * Triad bandwidth probe (the STREAM triad a = b + scalar * c, read 16 B and
 * write 8 B per element): runs it `reps` times on n doubles on the given
 * stream after one untimed launch and returns the average ms per triad.
 * All three are device arrays of n doubles owned by the caller; a must not
 * alias b or c.  PCG_EINVAL for null pointers, n < 2, reps < 1 or aliasing;
 * PCG_EHIP for a runtime error.
 */
int pcg_triad_probe(double *a, const double *b, const double *c, size_t n, double scalar,
                    int32_t reps, void *hip_stream, double *ms_per_triad);

#ifdef __cplusplus
}
#endif
#endif /* PCG_MI355X_H */
