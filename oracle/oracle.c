/*
 * oracle.c -- plain, slow, obviously correct FP64 reference for the pressure
 * projection of the cartesian-grid ship-wave method.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
 * only the test suite, the smoke check and the CPU-baseline leg of the bench
 * load it.  It shares no code, header or constant with the HIP library.
 *
 * What it computes
 * ----------------
 * The pressure equation of Section 2 (Eq. pois),
 *     d/dx_i ( (1/rho) dP/dx_i ) = Sigma,
 * discretised on a uniform grid of nx*ny*nz cells of spacing h with the
 * pressure and density at cell centres (flat index (k*ny + j)*nx + i):
 *   * between two face-adjacent fluid cells c, n the face coefficient is
 *     beta_cn = 1 / ((rho_c + rho_n)/2)   (1/rho at the face, rho averaged);
 *   * a face with a solid (hull) cell on either side carries beta = 0: the
 *     binary form of the free-slip hull of Section 2.2.1;
 *   * a Neumann wall face carries beta = 0; a Dirichlet wall face (p = 0 on
 *     the face, the zero reduced pressure of Section 2.4.2) uses
 *     beta = 1/rho_c with the mirrored ghost value -p_c;
 *   * (L p)_c = h^-2 [ sum_n beta_cn (p_n - p_c)
 *                      + sum_{Dirichlet faces} beta_c (-p_c - p_c) ].
 *   * periodic walls (the strut case of Section 3, periodic along x) come in
 *     opposite pairs on x or y: the face beyond the last cell of a row is the
 *     face before its first cell, an ordinary face between those two cells.
 *     An axis of one cell has no flux across its periodic face.
 * The solution is p = L^-1 Sigma on fluid cells and p = 0 on solid cells.
 * It exists and is unique iff every connected fluid region (periodic faces
 * included) touches a Dirichlet face.  When there is exactly one fluid
 * region and it touches none (no-flux and periodic walls only, as in the
 * strut case), L is singular with the constant as its null vector: the
 * oracle then solves for the source with its mean over fluid cells removed
 * and returns the solution of zero mean over fluid cells.
 *
 * The Introduction states that the equation is solved by a preconditioned
 * conjugate-gradient method.  The oracle runs textbook Jacobi-preconditioned
 * CG (Hestenes-Stiefel form) on the symmetric positive definite system
 * A x = b with A = -h^2 L and b = -h^2 Sigma; solid rows are identity rows
 * with b = 0.  The stop rule is ||b - A x||_2 <= tol ||b||_2, tested on the
 * recursive residual and confirmed on the recomputed one.
 *
 * Free-slip cut cells (Section 2.2.1): optional area fractions A on every
 * MAC face (arrays shaped like the face velocities) and volume fractions V
 * per cell enter the finite-volume form of the same equation,
 *     (1/(V_c h^2)) sum_f A_f beta_f (p_n - p_c) = Sigma_c,
 * i.e. every face coefficient (walls included) is weighted by its area
 * fraction and the scaled right-hand side is b_c = -h^2 V_c Sigma_c; the
 * divergence becomes (1/(V_c h)) sum_f A_f u_f n_f.  Without fractions
 * A = V = 1 and everything reduces to the binary form above.
 *
 * The velocity projection of Section 2.1 (u* = u - dt (1/rho) grad P on the
 * faces) and the face divergence are included so the divergence-free result
 * of the projection can be checked.
 *
 * Compiled with gcc -O2 -fopenmp, without fast-math.  Loops are plain; the
 * only parallelism is OpenMP over k.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* wall-clock seconds (used by the host bandwidth probe only) */
static double omp_now(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

enum { O_NEUMANN = 0, O_DIRICHLET = 1, O_PERIODIC = 2 };
enum {
    O_OK = 0, O_MAXIT = 1,
    O_EINVAL = -1, O_EDOMAIN = -2, O_ESINGULAR = -3, O_EBREAKDOWN = -4,
    O_ENOMEM = -5, O_EUNSUPPORTED = -8
};

typedef struct {
    int nx, ny, nz;
    double h;
    const double *rho;
    const uint8_t *solid;
    int bc[6]; /* x-, x+, y-, y+, z-, z+ */
    /* optional fractions (NULL: 1): faces u-, v-, w-shaped, cells */
    const double *ax, *ay, *az, *vol;
} problem;

/* area fraction of face f (order x-, x+, y-, y+, z-, z+) of cell (i,j,k);
 * on a periodic axis the face beyond the last cell is the row's face 0 */
static double area(const problem *P, int i, int j, int k, int f)
{
    int nx = P->nx, ny = P->ny;
    switch (f) {
    case 0: case 1: {
        if (!P->ax) return 1.0;
        int fi = i + (f == 1);
        if (fi == nx && P->bc[1] == O_PERIODIC) fi = 0;
        return P->ax[((size_t)k * ny + j) * (nx + 1) + fi];
    }
    case 2: case 3: {
        if (!P->ay) return 1.0;
        int fj = j + (f == 3);
        if (fj == ny && P->bc[3] == O_PERIODIC) fj = 0;
        return P->ay[((size_t)k * (ny + 1) + fj) * nx + i];
    }
    default:
        if (!P->az) return 1.0;
        return P->az[((size_t)(k + (f == 5)) * ny + j) * nx + i];
    }
}

static double volume(const problem *P, size_t c)
{
    return P->vol ? P->vol[c] : 1.0;
}

static size_t cell(const problem *P, int i, int j, int k)
{
    return ((size_t)k * P->ny + j) * P->nx + i;
}

/* beta on the face between cells a and b (both inside the grid). */
static double face_beta(const problem *P, size_t a, size_t b)
{
    if (P->solid[a] || P->solid[b]) return 0.0;
    return 1.0 / ((P->rho[a] + P->rho[b]) / 2.0);
}

/* beta on a wall face of cell a with boundary kind kind. */
static double wall_beta(const problem *P, size_t a, int kind)
{
    if (P->solid[a] || kind != O_DIRICHLET) return 0.0;
    return 1.0 / P->rho[a];
}

/*
 * Visit the six faces of cell (i,j,k).  For each face report the neighbour
 * index (or -1 for a wall) and beta.  Order: x-, x+, y-, y+, z-, z+.
 */
/*
 * Neighbour of (i,j,k) across face f (order x-, x+, y-, y+, z-, z+), with
 * periodic wrap-around.  Returns 1 and the neighbour's coordinates, or 0 for
 * a wall face.  The cell itself is never its own neighbour: on a periodic
 * axis of one cell the face carries no flux and is reported as a wall of
 * kind Neumann via *closed.
 */
static int neighbour(const problem *P, int i, int j, int k, int f, int *ni,
                     int *nj, int *nk, int *closed)
{
    int ii = i + (f == 0 ? -1 : f == 1 ? 1 : 0);
    int jj = j + (f == 2 ? -1 : f == 3 ? 1 : 0);
    int kk = k + (f == 4 ? -1 : f == 5 ? 1 : 0);
    *closed = 0;
    if (P->bc[f] == O_PERIODIC) {
        int len = f < 2 ? P->nx : P->ny;
        if (len == 1) { *closed = 1; return 0; }
        if (f < 2) ii = (ii + P->nx) % P->nx;
        else jj = (jj + P->ny) % P->ny;
    }
    if (ii < 0 || ii >= P->nx || jj < 0 || jj >= P->ny || kk < 0 || kk >= P->nz)
        return 0;
    *ni = ii; *nj = jj; *nk = kk;
    return 1;
}

static void faces_of(const problem *P, int i, int j, int k,
                     long long nb[6], double beta[6])
{
    size_t c = cell(P, i, j, k);
    for (int f = 0; f < 6; ++f) {
        int ni, nj, nk, closed;
        if (neighbour(P, i, j, k, f, &ni, &nj, &nk, &closed)) {
            size_t n = cell(P, ni, nj, nk);
            nb[f] = (long long)n;
            beta[f] = area(P, i, j, k, f) * face_beta(P, c, n);
        } else {
            nb[f] = -1;
            beta[f] = closed ? 0.0 : area(P, i, j, k, f) * wall_beta(P, c, P->bc[f]);
        }
    }
}

/* out = A p with A = -h^2 L on fluid rows and the identity on solid rows. */
static void apply_A(const problem *P, const double *p, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                size_t c = cell(P, i, j, k);
                if (P->solid[c]) { out[c] = p[c]; continue; }
                long long nb[6]; double beta[6];
                faces_of(P, i, j, k, nb, beta);
                double s = 0.0;
                for (int f = 0; f < 6; ++f) {
                    double pn = nb[f] >= 0 ? p[nb[f]] : -p[c]; /* ghost */
                    s += beta[f] * (p[c] - pn);
                }
                out[c] = s;
            }
}

/* diagonal of A (1 on solid rows). */
static void diag_A(const problem *P, double *d)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < P->nz; ++k)
        for (int j = 0; j < P->ny; ++j)
            for (int i = 0; i < P->nx; ++i) {
                size_t c = cell(P, i, j, k);
                if (P->solid[c]) { d[c] = 1.0; continue; }
                long long nb[6]; double beta[6];
                faces_of(P, i, j, k, nb, beta);
                double s = 0.0;
                for (int f = 0; f < 6; ++f)
                    s += nb[f] >= 0 ? beta[f] : 2.0 * beta[f];
                d[c] = s;
            }
}

static double dot(size_t n, const double *a, const double *b)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long long c = 0; c < (long long)n; ++c) s += a[c] * b[c];
    return s;
}

static int check_problem(const problem *P)
{
    if (P->nx < 1 || P->ny < 1 || P->nz < 1 || !(P->h > 0.0)) return O_EINVAL;
    for (int f = 0; f < 6; ++f)
        if (P->bc[f] != O_NEUMANN && P->bc[f] != O_DIRICHLET && P->bc[f] != O_PERIODIC)
            return O_EINVAL;
    /* periodic walls pair up; periodic z is not part of this reference */
    for (int a = 0; a < 3; ++a)
        if ((P->bc[2 * a] == O_PERIODIC) != (P->bc[2 * a + 1] == O_PERIODIC)) return O_EINVAL;
    if (P->bc[4] == O_PERIODIC) return O_EUNSUPPORTED;
    size_t n = (size_t)P->nx * P->ny * P->nz;
    for (size_t c = 0; c < n; ++c)
        if (!P->solid[c] && !(P->rho[c] > 0.0 && isfinite(P->rho[c])))
            return O_EDOMAIN;
    /* fractions come as a set: areas in [0, 1], fluid volumes in (0, 1] */
    int given = (P->ax != NULL) + (P->ay != NULL) + (P->az != NULL) + (P->vol != NULL);
    if (given != 0 && given != 4) return O_EINVAL;
    if (given) {
        size_t nfx = (size_t)P->nz * P->ny * (P->nx + 1), nfy = (size_t)P->nz * (P->ny + 1) * P->nx,
               nfz = (size_t)(P->nz + 1) * P->ny * P->nx;
        for (size_t f = 0; f < nfx; ++f) if (!(P->ax[f] >= 0.0 && P->ax[f] <= 1.0)) return O_EDOMAIN;
        for (size_t f = 0; f < nfy; ++f) if (!(P->ay[f] >= 0.0 && P->ay[f] <= 1.0)) return O_EDOMAIN;
        for (size_t f = 0; f < nfz; ++f) if (!(P->az[f] >= 0.0 && P->az[f] <= 1.0)) return O_EDOMAIN;
        for (size_t c = 0; c < n; ++c)
            if (!P->solid[c] && !(P->vol[c] > 0.0 && P->vol[c] <= 1.0)) return O_EDOMAIN;
    }
    return O_OK;
}

/*
 * Connected regions of fluid cells (face adjacency, periodic faces
 * included), by breadth-first search.  Returns the number of regions and
 * writes to *unanchored how many of them contain no cell with a Dirichlet
 * wall face; -1 when memory runs out.
 */
int oracle_components(int nx, int ny, int nz, const uint8_t *solid, const int *bc,
                      int *unanchored)
{
    problem P = { nx, ny, nz, 1.0, NULL, solid, { 0 } };
    for (int f = 0; f < 6; ++f) P.bc[f] = bc[f];
    size_t n = (size_t)nx * ny * nz;
    uint8_t *seen = calloc(n, 1);
    size_t *queue = malloc(n * sizeof(size_t));
    if (!seen || !queue) { free(seen); free(queue); return -1; }
    int regions = 0, loose = 0;
    for (size_t s0 = 0; s0 < n; ++s0) {
        if (solid[s0] || seen[s0]) continue;
        size_t head = 0, tail = 0;
        int anchored = 0;
        seen[s0] = 1;
        queue[tail++] = s0;
        while (head < tail) {
            size_t c = queue[head++];
            int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
            for (int f = 0; f < 6; ++f) {
                int ni, nj, nk, closed;
                if (neighbour(&P, i, j, k, f, &ni, &nj, &nk, &closed)) {
                    size_t m = cell(&P, ni, nj, nk);
                    if (!solid[m] && !seen[m]) { seen[m] = 1; queue[tail++] = m; }
                } else if (!closed && bc[f] == O_DIRICHLET) {
                    anchored = 1;
                }
            }
        }
        ++regions;
        if (!anchored) ++loose;
    }
    free(seen);
    free(queue);
    *unanchored = loose;
    return regions;
}

/* 1 if every fluid region touches a Dirichlet face, else 0 (-1: no memory). */
int oracle_connected(int nx, int ny, int nz, const uint8_t *solid, const int *bc)
{
    int loose = 0;
    int regions = oracle_components(nx, ny, nz, solid, bc, &loose);
    if (regions < 0) return -1;
    return loose == 0;
}

/* out = L p (the operator of Eq. pois as discretised above); 0 on solids. */
int oracle_apply(int nx, int ny, int nz, double h, const double *rho,
                 const uint8_t *solid, const int *bc, const double *p,
                 double *out, const double *ax, const double *ay, const double *az, const double *vol)
{
    problem P = { nx, ny, nz, h, rho, solid, { 0 }, ax, ay, az, vol };
    for (int f = 0; f < 6; ++f) P.bc[f] = bc[f];
    int st = check_problem(&P);
    if (st != O_OK) return st;
    size_t n = (size_t)nx * ny * nz;
    apply_A(&P, p, out);
    double s = -1.0 / (h * h);
#pragma omp parallel for schedule(static)
    for (long long c = 0; c < (long long)n; ++c)
        out[c] = solid[c] ? 0.0 : s * out[c] / volume(&P, (size_t)c);
    return O_OK;
}

/*
 * Relative residual of a pressure p for the source Sigma, measured as the
 * solver measures it: ||w - V L p||_2 / ||w||_2 over fluid cells, with
 * w = V Sigma the volume-weighted source (w = Sigma without fractions).
 * When the problem is singular (one fluid region, no Dirichlet face: the
 * constant is in the null space of L) w first loses its mean over fluid
 * cells, exactly the source oracle_pcg solves for; hull cells are skipped,
 * so whatever the caller holds there does not count.  NAN on invalid input.
 */
double oracle_relres(int nx, int ny, int nz, double h, const double *rho,
                     const uint8_t *solid, const int *bc, const double *rhs,
                     const double *p, const double *ax, const double *ay, const double *az, const double *vol)
{
    size_t n = (size_t)nx * ny * nz;
    int loose = 0;
    int regions = oracle_components(nx, ny, nz, solid, bc, &loose);
    if (regions < 0) return NAN;
    int singular = loose == 1 && regions == 1;
    double *Lp = malloc(n * sizeof(double));
    if (!Lp) return NAN;
    if (oracle_apply(nx, ny, nz, h, rho, solid, bc, p, Lp, ax, ay, az, vol) != O_OK) {
        free(Lp);
        return NAN;
    }
    double mean = 0.0;
    if (singular) {
        double sw = 0.0, nf = 0.0;
        for (size_t c = 0; c < n; ++c)
            if (!solid[c]) { sw += (vol ? vol[c] : 1.0) * rhs[c]; nf += 1.0; }
        mean = sw / nf;
    }
    double rr = 0.0, bb = 0.0;
#pragma omp parallel for reduction(+ : rr, bb) schedule(static)
    for (long long c = 0; c < (long long)n; ++c) {
        if (solid[c]) continue;
        double v = vol ? vol[c] : 1.0;
        double w = v * rhs[c] - mean;
        double r = w - v * Lp[c];
        rr += r * r;
        bb += w * w;
    }
    free(Lp);
    return bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
}

/*
 * Jacobi-preconditioned conjugate gradients on A x = b, A = -h^2 V L,
 * b = -h^2 V Sigma (fluid), 0 (solid).  Cold start x0 = 0.
 *   r = b, z = D^-1 r, p = z, rz = r.z
 *   repeat: q = A p; pq = p.q (breakdown if <= 0 or not finite);
 *           alpha = rz/pq; x += alpha p; r -= alpha q;
 *           if ||r|| <= tol ||b||: if ||b - A x|| <= tol ||b||: stop;
 *           z = D^-1 r; rz' = r.z; beta = rz'/rz; p = z + beta p.
 * Writes the solution (pressure, 0 on solids) to p_out, the iteration count,
 * the final true relative residual and, when hist != NULL, the recursive
 * relative residual after each iteration (hist[0] = 1).
 */
int oracle_pcg(int nx, int ny, int nz, double h, const double *rho,
               const uint8_t *solid, const int *bc, const double *rhs,
               double tol, int maxit, double *p_out, int *iters_out,
               double *relres_out, double *hist, const double *ax, const double *ay, const double *az, const double *vol)
{
    problem P = { nx, ny, nz, h, rho, solid, { 0 }, ax, ay, az, vol };
    for (int f = 0; f < 6; ++f) P.bc[f] = bc[f];
    *iters_out = 0;
    *relres_out = NAN;
    if (!(tol > 0.0) || maxit < 0) return O_EINVAL;
    int st = check_problem(&P);
    if (st != O_OK) return st;
    int loose = 0;
    int regions = oracle_components(nx, ny, nz, solid, bc, &loose);
    if (regions < 0) return O_ENOMEM;
    /* one region with no Dirichlet face: singular, solved for the mean-free
     * source; anything else unanchored has no unique answer here */
    int singular = loose == 1 && regions == 1;
    if (loose && !singular) return O_ESINGULAR;

    size_t n = (size_t)nx * ny * nz;
    double *x = calloc(n, sizeof(double));
    double *r = malloc(n * sizeof(double));
    double *z = malloc(n * sizeof(double));
    double *pp = malloc(n * sizeof(double));
    double *q = malloc(n * sizeof(double));
    double *d = malloc(n * sizeof(double));
    double *b = malloc(n * sizeof(double));
    if (!x || !r || !z || !pp || !q || !d || !b) {
        free(x); free(r); free(z); free(pp); free(q); free(d); free(b);
        return O_ENOMEM;
    }
    double h2 = h * h;
    for (size_t c = 0; c < n; ++c) {
        b[c] = solid[c] ? 0.0 : -h2 * volume(&P, c) * rhs[c];
        if (!isfinite(b[c])) st = O_EDOMAIN;
    }
    if (singular && st == O_OK) {
        /* remove the source's component along the null vector */
        double sb = 0.0, nf = 0.0;
        for (size_t c = 0; c < n; ++c)
            if (!solid[c]) { sb += b[c]; nf += 1.0; }
        double mean = sb / nf;
        for (size_t c = 0; c < n; ++c)
            if (!solid[c]) b[c] -= mean;
    }
    diag_A(&P, d);
    double nb = sqrt(dot(n, b, b));
    if (hist) hist[0] = 1.0;
    if (st != O_OK || nb == 0.0) {
        if (st == O_OK) { memset(p_out, 0, n * sizeof(double)); *relres_out = 0.0; }
        free(x); free(r); free(z); free(pp); free(q); free(d); free(b);
        return st;
    }
    for (size_t c = 0; c < n; ++c) {
        r[c] = b[c];
        z[c] = r[c] / d[c];
        pp[c] = z[c];
    }
    double rz = dot(n, r, z);
    int k = 0;
    int status = O_MAXIT;
    double relres = 1.0;
    while (k < maxit) {
        apply_A(&P, pp, q);
        double pq = dot(n, pp, q);
        if (!(pq > 0.0) || !isfinite(pq)) { status = O_EBREAKDOWN; break; }
        double alpha = rz / pq;
#pragma omp parallel for schedule(static)
        for (long long c = 0; c < (long long)n; ++c) {
            x[c] += alpha * pp[c];
            r[c] -= alpha * q[c];
        }
        ++k;
        double rn = sqrt(dot(n, r, r));
        if (hist) hist[k] = rn / nb;
        if (rn <= tol * nb) {
            apply_A(&P, x, q);
            double tt = 0.0;
#pragma omp parallel for reduction(+ : tt) schedule(static)
            for (long long c = 0; c < (long long)n; ++c) {
                double e = b[c] - q[c];
                tt += e * e;
            }
            relres = sqrt(tt) / nb;
            if (relres <= tol) { status = O_OK; break; }
        }
#pragma omp parallel for schedule(static)
        for (long long c = 0; c < (long long)n; ++c) z[c] = r[c] / d[c];
        double rz_new = dot(n, r, z);
        double beta = rz_new / rz;
#pragma omp parallel for schedule(static)
        for (long long c = 0; c < (long long)n; ++c) pp[c] = z[c] + beta * pp[c];
        rz = rz_new;
    }
    if (status != O_OK) {
        apply_A(&P, x, q);
        double tt = 0.0;
        for (size_t c = 0; c < n; ++c) {
            double e = b[c] - q[c];
            tt += e * e;
        }
        relres = sqrt(tt) / nb;
    }
    if (singular) {
        /* the solution of zero mean over fluid cells */
        double sx = 0.0, nf = 0.0;
        for (size_t c = 0; c < n; ++c)
            if (!solid[c]) { sx += x[c]; nf += 1.0; }
        double mean = sx / nf;
        for (size_t c = 0; c < n; ++c)
            if (!solid[c]) x[c] -= mean;
    }
    for (size_t c = 0; c < n; ++c) p_out[c] = solid[c] ? 0.0 : x[c];
    *iters_out = k;
    *relres_out = relres;
    free(x); free(r); free(z); free(pp); free(q); free(d); free(b);
    return status;
}

/*
 * Velocity projection of Section 2.1 on MAC faces, in place:
 *   u_f <- u_f - dt * beta_f * (p_right - p_left) / h,
 * with beta_f as in the operator (0 on Neumann and hull faces, 1/rho_c with
 * the ghost -p_c on Dirichlet faces).  Face arrays are u[nz][ny][nx+1],
 * v[nz][ny+1][nx], w[nz+1][ny][nx].  With periodic x (y) walls face 0 is the
 * face between the last and the first cell of the row, and face nx (ny) is
 * written as a copy of it.
 */
int oracle_project(int nx, int ny, int nz, double h, const double *rho,
                   const uint8_t *solid, const int *bc, double dt,
                   const double *p, double *u, double *v, double *w)
{
    problem P = { nx, ny, nz, h, rho, solid, { 0 } };
    for (int f = 0; f < 6; ++f) P.bc[f] = bc[f];
    int st = check_problem(&P);
    if (st != O_OK) return st;
    double s = dt / h;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int f = 0; f <= nx; ++f) {
                double *uf = &u[((size_t)k * ny + j) * (nx + 1) + f];
                if (bc[0] == O_PERIODIC && (f == 0 || f == nx)) {
                    /* face 0 is shared by cells nx-1 and 0; face nx repeats it */
                    if (f == nx) { *uf = uf[-nx]; continue; }
                    size_t a = cell(&P, nx - 1, j, k), b = cell(&P, 0, j, k);
                    if (nx > 1) *uf -= s * face_beta(&P, a, b) * (p[b] - p[a]);
                } else if (f == 0) {
                    size_t c = cell(&P, 0, j, k);
                    *uf -= s * wall_beta(&P, c, bc[0]) * (p[c] - (-p[c]));
                } else if (f == nx) {
                    size_t c = cell(&P, nx - 1, j, k);
                    *uf -= s * wall_beta(&P, c, bc[1]) * ((-p[c]) - p[c]);
                } else {
                    size_t a = cell(&P, f - 1, j, k), b = cell(&P, f, j, k);
                    *uf -= s * face_beta(&P, a, b) * (p[b] - p[a]);
                }
            }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int f = 0; f <= ny; ++f)
            for (int i = 0; i < nx; ++i) {
                double *vf = &v[((size_t)k * (ny + 1) + f) * nx + i];
                if (bc[2] == O_PERIODIC && (f == 0 || f == ny)) {
                    if (f == ny) { *vf = v[((size_t)k * (ny + 1)) * nx + i]; continue; }
                    size_t a = cell(&P, i, ny - 1, k), b = cell(&P, i, 0, k);
                    if (ny > 1) *vf -= s * face_beta(&P, a, b) * (p[b] - p[a]);
                } else if (f == 0) {
                    size_t c = cell(&P, i, 0, k);
                    *vf -= s * wall_beta(&P, c, bc[2]) * (p[c] - (-p[c]));
                } else if (f == ny) {
                    size_t c = cell(&P, i, ny - 1, k);
                    *vf -= s * wall_beta(&P, c, bc[3]) * ((-p[c]) - p[c]);
                } else {
                    size_t a = cell(&P, i, f - 1, k), b = cell(&P, i, f, k);
                    *vf -= s * face_beta(&P, a, b) * (p[b] - p[a]);
                }
            }
#pragma omp parallel for schedule(static)
    for (int f = 0; f <= nz; ++f)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double *wf = &w[((size_t)f * ny + j) * nx + i];
                if (f == 0) {
                    size_t c = cell(&P, i, j, 0);
                    *wf -= s * wall_beta(&P, c, bc[4]) * (p[c] - (-p[c]));
                } else if (f == nz) {
                    size_t c = cell(&P, i, j, nz - 1);
                    *wf -= s * wall_beta(&P, c, bc[5]) * ((-p[c]) - p[c]);
                } else {
                    size_t a = cell(&P, i, j, f - 1), b = cell(&P, i, j, f);
                    *wf -= s * face_beta(&P, a, b) * (p[b] - p[a]);
                }
            }
    return O_OK;
}

/* (D u)_c = (u_{i+1/2} - u_{i-1/2} + v_{j+1/2} - v_{j-1/2}
 *           + w_{k+1/2} - w_{k-1/2}) / h  -- the discrete form of Eq. (mass);
 * with fractions every face velocity is weighted by its area fraction and
 * the sum divided by V_c.  Arrays are used as given (on a periodic axis the
 * last face must repeat face 0). */
void oracle_divergence(int nx, int ny, int nz, double h, const double *u,
                       const double *v, const double *w, double *out, const double *ax, const double *ay, const double *az, const double *vol)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t u0 = ((size_t)k * ny + j) * (nx + 1) + i;
                size_t v0 = ((size_t)k * (ny + 1) + j) * nx + i;
                size_t w0 = ((size_t)k * ny + j) * nx + i;
                size_t v1 = v0 + nx, w1 = w0 + (size_t)nx * ny;
                double du, dv, dw, vc = 1.0;
                if (ax) {
                    du = ax[u0 + 1] * u[u0 + 1] - ax[u0] * u[u0];
                    dv = ay[v1] * v[v1] - ay[v0] * v[v0];
                    dw = az[w1] * w[w1] - az[w0] * w[w0];
                    vc = vol[w0];
                } else {
                    du = u[u0 + 1] - u[u0];
                    dv = v[v1] - v[v0];
                    dw = w[w1] - w[w0];
                }
                out[w0] = ax ? (du + dv + dw) / (vc * h) : (du + dv + dw) / h;
            }
}

/*
 * Host memory bandwidth of the threads the oracle runs on: the STREAM triad
 * a = b + 3 c over n doubles (24 B per element), best of `reps` passes after
 * a first-touch initialisation by the same threads.  Context for the
 * oracle's timing only; no part of the method.  GB/s, or -1 if the arrays
 * cannot be allocated.
 */
double oracle_host_triad(long n, int reps)
{
    double *a = malloc(sizeof(double) * (size_t)n);
    double *b = malloc(sizeof(double) * (size_t)n);
    double *c = malloc(sizeof(double) * (size_t)n);
    if (!a || !b || !c) { free(a); free(b); free(c); return -1.0; }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) { a[i] = 0.0; b[i] = 1.0; c[i] = 2.0; }
    double best = 1e300;
    for (int r = 0; r < reps; ++r) {
        const double t0 = omp_now();
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) a[i] = b[i] + 3.0 * c[i];
        const double t = omp_now() - t0;
        if (t < best) best = t;
    }
    const double check = a[n / 2];
    free(a); free(b); free(c);
    if (check != 7.0) return -1.0;
    return 24.0 * (double)n / best / 1e9;
}

/* Threads of the oracle's parallel loops started from the calling thread
 * (each host thread that calls the oracle keeps its own setting). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
