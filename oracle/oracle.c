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
 * The solution is p = L^-1 Sigma on fluid cells and p = 0 on solid cells.
 * It exists and is unique iff every connected fluid region touches a
 * Dirichlet face.
 *
 * The Introduction states that the equation is solved by a preconditioned
 * conjugate-gradient method.  The oracle runs textbook Jacobi-preconditioned
 * CG (Hestenes-Stiefel form) on the symmetric positive definite system
 * A x = b with A = -h^2 L and b = -h^2 Sigma; solid rows are identity rows
 * with b = 0.  The stop rule is ||b - A x||_2 <= tol ||b||_2, tested on the
 * recursive residual and confirmed on the recomputed one.
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
#ifdef _OPENMP
#include <omp.h>
#endif

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
} problem;

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
static void faces_of(const problem *P, int i, int j, int k,
                     long long nb[6], double beta[6])
{
    size_t c = cell(P, i, j, k);
    int ii[6] = { i - 1, i + 1, i, i, i, i };
    int jj[6] = { j, j, j - 1, j + 1, j, j };
    int kk[6] = { k, k, k, k, k - 1, k + 1 };
    for (int f = 0; f < 6; ++f) {
        int inside = ii[f] >= 0 && ii[f] < P->nx && jj[f] >= 0 &&
                     jj[f] < P->ny && kk[f] >= 0 && kk[f] < P->nz;
        if (inside) {
            size_t n = cell(P, ii[f], jj[f], kk[f]);
            nb[f] = (long long)n;
            beta[f] = face_beta(P, c, n);
        } else {
            nb[f] = -1;
            beta[f] = wall_beta(P, c, P->bc[f]);
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
    for (int f = 0; f < 6; ++f) {
        if (P->bc[f] == O_PERIODIC) return O_EUNSUPPORTED;
        if (P->bc[f] != O_NEUMANN && P->bc[f] != O_DIRICHLET) return O_EINVAL;
    }
    size_t n = (size_t)P->nx * P->ny * P->nz;
    for (size_t c = 0; c < n; ++c)
        if (!P->solid[c] && !(P->rho[c] > 0.0 && isfinite(P->rho[c])))
            return O_EDOMAIN;
    return O_OK;
}

/*
 * 1 if every connected region of fluid cells (face adjacency) contains a cell
 * with a Dirichlet wall face, else 0.  Breadth-first search from all such
 * cells, then a scan for unreached fluid.
 */
int oracle_connected(int nx, int ny, int nz, const uint8_t *solid,
                     const int *bc)
{
    problem P = { nx, ny, nz, 1.0, NULL, solid, { 0 } };
    for (int f = 0; f < 6; ++f) P.bc[f] = bc[f];
    size_t n = (size_t)nx * ny * nz;
    uint8_t *seen = calloc(n, 1);
    size_t *queue = malloc(n * sizeof(size_t));
    if (!seen || !queue) { free(seen); free(queue); return -1; }
    size_t head = 0, tail = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = cell(&P, i, j, k);
                if (solid[c]) continue;
                int touches = (i == 0 && bc[0] == O_DIRICHLET) ||
                              (i == nx - 1 && bc[1] == O_DIRICHLET) ||
                              (j == 0 && bc[2] == O_DIRICHLET) ||
                              (j == ny - 1 && bc[3] == O_DIRICHLET) ||
                              (k == 0 && bc[4] == O_DIRICHLET) ||
                              (k == nz - 1 && bc[5] == O_DIRICHLET);
                if (touches) { seen[c] = 1; queue[tail++] = c; }
            }
    while (head < tail) {
        size_t c = queue[head++];
        int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
        int ii[6] = { i - 1, i + 1, i, i, i, i };
        int jj[6] = { j, j, j - 1, j + 1, j, j };
        int kk[6] = { k, k, k, k, k - 1, k + 1 };
        for (int f = 0; f < 6; ++f) {
            if (ii[f] < 0 || ii[f] >= nx || jj[f] < 0 || jj[f] >= ny ||
                kk[f] < 0 || kk[f] >= nz) continue;
            size_t m = cell(&P, ii[f], jj[f], kk[f]);
            if (!solid[m] && !seen[m]) { seen[m] = 1; queue[tail++] = m; }
        }
    }
    int ok = 1;
    for (size_t c = 0; c < n && ok; ++c)
        if (!solid[c] && !seen[c]) ok = 0;
    free(seen);
    free(queue);
    return ok;
}

/* out = L p (the operator of Eq. pois as discretised above); 0 on solids. */
int oracle_apply(int nx, int ny, int nz, double h, const double *rho,
                 const uint8_t *solid, const int *bc, const double *p,
                 double *out)
{
    problem P = { nx, ny, nz, h, rho, solid, { 0 } };
    for (int f = 0; f < 6; ++f) P.bc[f] = bc[f];
    int st = check_problem(&P);
    if (st != O_OK) return st;
    size_t n = (size_t)nx * ny * nz;
    apply_A(&P, p, out);
    double s = -1.0 / (h * h);
#pragma omp parallel for schedule(static)
    for (long long c = 0; c < (long long)n; ++c)
        out[c] = solid[c] ? 0.0 : s * out[c];
    return O_OK;
}

/*
 * Relative residual ||Sigma - L p||_2 / ||Sigma||_2 over fluid cells (the
 * same number as ||b - A p|| / ||b|| for the scaled SPD system).
 */
double oracle_relres(int nx, int ny, int nz, double h, const double *rho,
                     const uint8_t *solid, const int *bc, const double *rhs,
                     const double *p)
{
    size_t n = (size_t)nx * ny * nz;
    double *Lp = malloc(n * sizeof(double));
    if (!Lp) return NAN;
    if (oracle_apply(nx, ny, nz, h, rho, solid, bc, p, Lp) != O_OK) {
        free(Lp);
        return NAN;
    }
    double rr = 0.0, bb = 0.0;
#pragma omp parallel for reduction(+ : rr, bb) schedule(static)
    for (long long c = 0; c < (long long)n; ++c) {
        if (solid[c]) continue;
        double r = rhs[c] - Lp[c];
        rr += r * r;
        bb += rhs[c] * rhs[c];
    }
    free(Lp);
    return bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
}

/*
 * Jacobi-preconditioned conjugate gradients on A x = b, A = -h^2 L,
 * b = -h^2 Sigma (fluid), 0 (solid).  Cold start x0 = 0.
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
               double *relres_out, double *hist)
{
    problem P = { nx, ny, nz, h, rho, solid, { 0 } };
    for (int f = 0; f < 6; ++f) P.bc[f] = bc[f];
    *iters_out = 0;
    *relres_out = NAN;
    if (!(tol > 0.0) || maxit < 0) return O_EINVAL;
    int st = check_problem(&P);
    if (st != O_OK) return st;
    if (!oracle_connected(nx, ny, nz, solid, bc)) return O_ESINGULAR;

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
        b[c] = solid[c] ? 0.0 : -h2 * rhs[c];
        if (!isfinite(b[c])) st = O_EDOMAIN;
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
 * v[nz][ny+1][nx], w[nz+1][ny][nx].
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
                if (f == 0) {
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
                if (f == 0) {
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
 *           + w_{k+1/2} - w_{k-1/2}) / h  -- the discrete form of Eq. (mass). */
void oracle_divergence(int nx, int ny, int nz, double h, const double *u,
                       const double *v, const double *w, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double du = u[((size_t)k * ny + j) * (nx + 1) + i + 1] -
                            u[((size_t)k * ny + j) * (nx + 1) + i];
                double dv = v[((size_t)k * (ny + 1) + j + 1) * nx + i] -
                            v[((size_t)k * (ny + 1) + j) * nx + i];
                double dw = w[((size_t)(k + 1) * ny + j) * nx + i] -
                            w[((size_t)k * ny + j) * nx + i];
                out[((size_t)k * ny + j) * nx + i] = (du + dv + dw) / h;
            }
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
