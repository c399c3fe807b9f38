// Device kernels of the MI355X pressure solver (gfx950, wave64).
//
// The operator is the 7-point discretisation of div((1/rho) grad p) of the
// pressure equation (Section 2, Eq. pois) in its symmetric positive definite
// form A = -h^2 L: for fluid cell c
//     (A v)_c = sum_faces beta_f (v_c - v_n) + sum_Dirichlet (2/rho_c) v_c,
//     beta_f  = 2/(rho_c + rho_n)   (1 over the mean density on the face).
// Face coefficients are not stored: they are recomputed from one density
// array in which hull cells hold +inf, so every face touching the hull gets
// beta = 2/(rho + inf) = 0 (binary free-slip hull, Section 2.2.1) and the
// diagonal of a hull row is 0.  Walls are described by a 6-bit Dirichlet mask.
//
// The Krylov method is Jacobi-preconditioned CG (the Introduction names a
// preconditioned conjugate-gradient solver) written in "z form": the
// vector kept between iterations is z = D^-1 r instead of r, so
//   pass A:  p = z + beta p                 and  p.Ap = sum_f beta_f (dp_f)^2
//   pass B:  q = A p (recomputed), x += alpha p, z -= alpha q / diag
//            r.z = sum diag z^2,  r.r = sum (diag z)^2
// Each pass is one HBM sweep; the two global reductions per iteration are
// per-tile partial sums written to memory and added in tile order by the
// last workgroup to arrive, which also advances the solve's state machine.
//
// Work decomposition: a tile is kBlock consecutive cells of an x-y plane
// (x fastest) times tz planes; each thread owns one (i,j) column of the tile
// and marches up in z keeping the k-1, k, k+1 values in registers.  A launch
// grid-strides over the tiles of all active solves; workgroup ids are
// remapped so each of the 8 XCDs walks a contiguous range of tiles, keeping
// the y-neighbour rows of concurrently running tiles in that XCD's L2.
#include <hip/hip_runtime.h>
#include <math.h>
#include <type_traits>
#include <stdint.h>

#include "pcg_types.h"
#include "pcg.h"

namespace pcgmi {

constexpr int kMaxOuter = 40;   // cap on refinement trips

// ------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------

__device__ __forceinline__ int xcd_major(int b, int G)
{
    // hardware dispatches workgroup b to XCD b % 8; give XCD x the ids
    // x*G/8 .. (x+1)*G/8-1 (G is a multiple of 8)
    return (b & 7) * (G >> 3) + (b >> 3);
}

__device__ __forceinline__ int find_slot(const Slot *__restrict__ slots, int n,
                                         int64_t t)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (slots[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum NV values over the workgroup; the total lands in thread 0 in an order
// fixed by the tile alone.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds)
{
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m] = wave_sum(v[m]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int m = 0; m < NV; ++m) lds[m * 4 + w] = v[m];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int m = 0; m < NV; ++m)
            v[m] = (lds[m * 4 + 0] + lds[m * 4 + 1]) + (lds[m * 4 + 2] + lds[m * 4 + 3]);
    }
    __syncthreads();
}

__device__ __forceinline__ void store_agent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double load_agent(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

struct TileCtx {
    int q;       // index of this thread's column in the x-y plane
    int i, j;
    int k0, k1;  // planes [k0, k1)
    int P;       // nx*ny
    bool active;
};

__device__ __forceinline__ TileCtx tile_ctx(const Slot &S, int64_t lt)
{
    TileCtx t;
    const int pt = (int)(lt % S.plane_tiles);
    const int zt = (int)(lt / S.plane_tiles);
    t.P = S.nx * S.ny;
    t.q = pt * kBlock + (int)threadIdx.x;
    t.active = t.q < t.P;
    t.i = t.q % S.nx;
    t.j = t.q / S.nx;
    t.k0 = zt * S.tz;
    t.k1 = min(S.nz, t.k0 + S.tz);
    return t;
}

// One interior face: beta = 2/(rho_c + rho_n).
template <typename T>
__device__ __forceinline__ void face(T vc, T rc, T vn, T rn, T &q, T &dg)
{
    const T b = T(2) / (rc + rn);
    q += b * (vc - vn);
    dg += b;
}

// One wall face: Dirichlet contributes (2/rho_c) to the diagonal.
template <typename T>
__device__ __forceinline__ void wall(T vc, T rc, bool dirichlet, T &q, T &dg)
{
    if (dirichlet) {
        const T b = T(2) / rc;
        q += b * vc;
        dg += b;
    }
}

// q = (A v)_c and dg = A_cc for cell c.  x and y neighbours are loaded; the
// z neighbours are passed in by the z march.  MASK: read v as 0 in hull
// cells (for vectors whose hull entries are not yet cleared).
template <typename T, bool MASK = false>
__device__ __forceinline__ void stencil(const T *__restrict__ v,
                                        const T *__restrict__ rho, int64_t c,
                                        const TileCtx &t, int k, const Slot &S,
                                        T vc, T rc, T vzm, T rzm, T vzp, T rzp,
                                        T &q, T &dg)
{
    q = T(0);
    dg = T(0);
    const int bm = S.bcmask;
    auto val = [&](int64_t n, T rn) -> T {
        T vn = v[n];
        if (MASK) vn = isinf(rn) ? T(0) : vn;
        return vn;
    };
    if (t.i > 0) { T rn = rho[c - 1]; face(vc, rc, val(c - 1, rn), rn, q, dg); }
    else wall(vc, rc, bm & 1, q, dg);
    if (t.i < S.nx - 1) { T rn = rho[c + 1]; face(vc, rc, val(c + 1, rn), rn, q, dg); }
    else wall(vc, rc, bm & 2, q, dg);
    if (t.j > 0) { T rn = rho[c - S.nx]; face(vc, rc, val(c - S.nx, rn), rn, q, dg); }
    else wall(vc, rc, bm & 4, q, dg);
    if (t.j < S.ny - 1) { T rn = rho[c + S.nx]; face(vc, rc, val(c + S.nx, rn), rn, q, dg); }
    else wall(vc, rc, bm & 8, q, dg);
    if (k > 0) face(vc, rc, vzm, rzm, q, dg);
    else wall(vc, rc, bm & 16, q, dg);
    if (k < S.nz - 1) face(vc, rc, vzp, rzp, q, dg);
    else wall(vc, rc, bm & 32, q, dg);
}

// Diagonal only (no vector).
template <typename T>
__device__ __forceinline__ T diag_at(const T *__restrict__ rho, int64_t c,
                                     const TileCtx &t, int k, const Slot &S,
                                     T rc, T rzm, T rzp)
{
    T q = T(0), dg = T(0);
    const int bm = S.bcmask;
    const T z0 = T(0);
    if (t.i > 0) face(z0, rc, z0, rho[c - 1], q, dg); else wall(z0, rc, bm & 1, q, dg);
    if (t.i < S.nx - 1) face(z0, rc, z0, rho[c + 1], q, dg); else wall(z0, rc, bm & 2, q, dg);
    if (t.j > 0) face(z0, rc, z0, rho[c - S.nx], q, dg); else wall(z0, rc, bm & 4, q, dg);
    if (t.j < S.ny - 1) face(z0, rc, z0, rho[c + S.nx], q, dg); else wall(z0, rc, bm & 8, q, dg);
    if (k > 0) face(z0, rc, z0, rzm, q, dg); else wall(z0, rc, bm & 16, q, dg);
    if (k < S.nz - 1) face(z0, rc, z0, rzp, q, dg); else wall(z0, rc, bm & 32, q, dg);
    return dg;
}

// x + s d, evaluated identically wherever the refined iterate is needed.
__device__ __forceinline__ double refined(double x, double s, float d)
{
    return fma(s, (double)d, x);
}

// ------------------------------------------------------------------------
// phase bodies (one tile each); acc[] receives this thread's partial sums
// ------------------------------------------------------------------------

// K1_INIT64: b = -h^2 Sigma (0 on hull), r = b (cold) or b - A x0 (warm),
// z = r / diag.  acc = [b.b, r.z, r.r].
__device__ void body_init64(const Slot &S, const SlotState &st, int64_t lt,
                            double (&acc)[3])
{
    const TileCtx t = tile_ctx(S, lt);
    if (!t.active) return;
    const double *rho = S.rho64;
    double *x = S.x;
    double *z = (double *)S.z;
    const bool warm = st.warm != 0;
    int64_t c = (int64_t)t.k0 * t.P + t.q;
    double rzm = 1.0, xzm = 0.0;
    double rc = rho[c];
    double xc = 0.0;
    if (warm) {
        xc = isinf(rc) ? 0.0 : x[c];
        if (t.k0 > 0) {
            rzm = rho[c - t.P];
            xzm = isinf(rzm) ? 0.0 : x[c - t.P];
        }
    } else if (t.k0 > 0) {
        rzm = rho[c - t.P];
    }
    for (int k = t.k0; k < t.k1; ++k, c += t.P) {
        double rzp = 1.0, xzp = 0.0;
        if (k + 1 < S.nz) {
            rzp = rho[c + t.P];
            if (warm) xzp = isinf(rzp) ? 0.0 : x[c + t.P];
        }
        const bool solid = isinf(rc);
        const double b = solid ? 0.0 : -S.h2 * S.rhs[c];
        double r, dg;
        if (warm) {
            double q;
            stencil<double, true>(x, rho, c, t, k, S, xc, rc, xzm, rzm, xzp, rzp, q, dg);
            r = solid ? 0.0 : b - q;
            if (solid) x[c] = 0.0;
        } else {
            dg = diag_at(rho, c, t, k, S, rc, rzm, rzp);
            r = b;
            x[c] = 0.0;
        }
        const double zc = dg > 0.0 ? r / dg : 0.0;
        z[c] = zc;
        acc[0] += b * b;
        acc[1] += r * zc;
        acc[2] += r * r;
        rzm = rc; xzm = xc;
        rc = rzp; xc = xzp;
    }
}

// K1_CG_A / K1_IR_A: p_new = z + beta p_old (z when first), stored; the
// quadratic form p.Ap summed over the low faces of each cell.
template <typename T>
__device__ void body_passA(const Slot &S, const SlotState &st, int64_t lt,
                           double (&acc)[3])
{
    const TileCtx t = tile_ctx(S, lt);
    if (!t.active) return;
    const T *ps = (const T *)(st.pbuf ? S.pb : S.pa);
    T *pd = (T *)(st.pbuf ? S.pa : S.pb);
    const T *z = (const T *)S.z;
    const T *rho = std::is_same<T, double>::value ? (const T *)S.rho64
                                                   : (const T *)S.rho32;
    const bool first = st.first != 0;
    const T beta = (T)st.beta;
    auto pnew = [&](int64_t n) -> T {
        const T zz = z[n];
        return first ? zz : zz + beta * ps[n];
    };
    const int bm = S.bcmask;
    int64_t c = (int64_t)t.k0 * t.P + t.q;
    T pzm = T(0), rzm = T(1);
    if (t.k0 > 0) { pzm = pnew(c - t.P); rzm = rho[c - t.P]; }
    double a = 0.0;
    for (int k = t.k0; k < t.k1; ++k, c += t.P) {
        const T pc = pnew(c);
        const T rc = rho[c];
        pd[c] = pc;
        T s = T(0);
        const T bd = T(2) / rc;          // Dirichlet wall weight (0 on hull)
        const T pc2 = pc * pc;
        if (t.i > 0) {
            const T d = pc - pnew(c - 1);
            s += (T(2) / (rc + rho[c - 1])) * d * d;
        } else if (bm & 1) s += bd * pc2;
        if (t.i == S.nx - 1 && (bm & 2)) s += bd * pc2;
        if (t.j > 0) {
            const T d = pc - pnew(c - S.nx);
            s += (T(2) / (rc + rho[c - S.nx])) * d * d;
        } else if (bm & 4) s += bd * pc2;
        if (t.j == S.ny - 1 && (bm & 8)) s += bd * pc2;
        if (k > 0) {
            const T d = pc - pzm;
            s += (T(2) / (rc + rzm)) * d * d;
        } else if (bm & 16) s += bd * pc2;
        if (k == S.nz - 1 && (bm & 32)) s += bd * pc2;
        a += (double)s;
        pzm = pc;
        rzm = rc;
    }
    acc[0] += a;
}

// K2_CG_B (T = double, X = double: x) / K2_IR_B (T = float, X = float: d):
// q = A p, x += alpha p, z -= alpha q / diag; acc = [r.z, r.r].
template <typename T, typename X>
__device__ void body_passB(const Slot &S, const SlotState &st, int64_t lt,
                           double (&acc)[3])
{
    const TileCtx t = tile_ctx(S, lt);
    if (!t.active) return;
    const T *p = (const T *)(st.pbuf ? S.pb : S.pa);
    const T *rho = std::is_same<T, double>::value ? (const T *)S.rho64
                                                   : (const T *)S.rho32;
    T *z = (T *)S.z;
    X *x = std::is_same<X, double>::value ? (X *)S.x : (X *)S.d32;
    const T alpha = (T)st.alpha;
    int64_t c = (int64_t)t.k0 * t.P + t.q;
    T vzm = T(0), rzm = T(1);
    T vc = p[c], rc = rho[c];
    if (t.k0 > 0) { vzm = p[c - t.P]; rzm = rho[c - t.P]; }
    double a0 = 0.0, a1 = 0.0;
    for (int k = t.k0; k < t.k1; ++k, c += t.P) {
        T vzp = T(0), rzp = T(1);
        if (k + 1 < S.nz) { vzp = p[c + t.P]; rzp = rho[c + t.P]; }
        T q, dg;
        stencil<T>(p, rho, c, t, k, S, vc, rc, vzm, rzm, vzp, rzp, q, dg);
        x[c] += (X)(alpha * vc);
        T zc = z[c];
        if (dg > T(0)) zc -= alpha * q / dg;
        z[c] = zc;
        const double dd = (double)dg, dz = (double)zc;
        const double r = dd * dz;
        a0 += r * dz;
        a1 += r * r;
        vzm = vc; rzm = rc;
        vc = vzp; rc = rzp;
    }
    acc[0] += a0;
    acc[1] += a1;
}

// K1_CHECK64: ||b - A x||^2 with the FP64 operator.
__device__ void body_check64(const Slot &S, const SlotState &st, int64_t lt,
                             double (&acc)[3])
{
    const TileCtx t = tile_ctx(S, lt);
    if (!t.active) return;
    const double *rho = S.rho64;
    const double *x = S.x;
    int64_t c = (int64_t)t.k0 * t.P + t.q;
    double vzm = 0.0, rzm = 1.0, vc = x[c], rc = rho[c];
    if (t.k0 > 0) { vzm = x[c - t.P]; rzm = rho[c - t.P]; }
    double a = 0.0;
    for (int k = t.k0; k < t.k1; ++k, c += t.P) {
        double vzp = 0.0, rzp = 1.0;
        if (k + 1 < S.nz) { vzp = x[c + t.P]; rzp = rho[c + t.P]; }
        double q, dg;
        stencil<double>(x, rho, c, t, k, S, vc, rc, vzm, rzm, vzp, rzp, q, dg);
        if (!isinf(rc)) {
            const double r = -S.h2 * S.rhs[c] - q;
            a += r * r;
        }
        vzm = vc; rzm = rc;
        vc = vzp; rc = rzp;
    }
    acc[0] += a;
}

// K1_IR_INIT: x = 0 (cold) or hull entries cleared (warm), d = 0; acc = [b.b].
__device__ void body_ir_init(const Slot &S, const SlotState &st, int64_t lt,
                             double (&acc)[3])
{
    const TileCtx t = tile_ctx(S, lt);
    if (!t.active) return;
    int64_t c = (int64_t)t.k0 * t.P + t.q;
    const bool warm = st.warm != 0;
    double a = 0.0;
    for (int k = t.k0; k < t.k1; ++k, c += t.P) {
        const bool solid = isinf(S.rho64[c]);
        if (!warm || solid) S.x[c] = 0.0;
        S.d32[c] = 0.0f;
        const double b = solid ? 0.0 : -S.h2 * S.rhs[c];
        a += b * b;
    }
    acc[0] += a;
}

// K1_IR_RESID: r = b - A64 (x + s d) in FP64, and the scaled inner right-hand
// side in z form, z32 = (scale r) / diag32.  acc = [r.r, r32.z32, r32.r32].
__device__ void body_ir_resid(const Slot &S, const SlotState &st, int64_t lt,
                              double (&acc)[3])
{
    const TileCtx t = tile_ctx(S, lt);
    if (!t.active) return;
    const double *rho = S.rho64;
    const float *rho32 = S.rho32;
    const double *x = S.x;
    const float *d = S.d32;
    float *z = (float *)S.z;
    const double s = st.upd_s;
    const double scale = st.scale;
    const int64_t P = t.P;
    int64_t c = (int64_t)t.k0 * P + t.q;
    auto xe = [&](int64_t n) { return refined(x[n], s, d[n]); };
    double vzm = 0.0, rzm = 1.0;
    float fzm = 1.0f;
    double vc = xe(c), rc = rho[c];
    float fc = rho32[c];
    if (t.k0 > 0) { vzm = xe(c - P); rzm = rho[c - P]; fzm = rho32[c - P]; }
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const int bm = S.bcmask;
    for (int k = t.k0; k < t.k1; ++k, c += P) {
        double vzp = 0.0, rzp = 1.0;
        float fzp = 1.0f;
        if (k + 1 < S.nz) { vzp = xe(c + P); rzp = rho[c + P]; fzp = rho32[c + P]; }
        // FP64 residual of the refined iterate
        double q = 0.0, dg = 0.0;
        if (t.i > 0) face(vc, rc, xe(c - 1), rho[c - 1], q, dg); else wall(vc, rc, bm & 1, q, dg);
        if (t.i < S.nx - 1) face(vc, rc, xe(c + 1), rho[c + 1], q, dg); else wall(vc, rc, bm & 2, q, dg);
        if (t.j > 0) face(vc, rc, xe(c - S.nx), rho[c - S.nx], q, dg); else wall(vc, rc, bm & 4, q, dg);
        if (t.j < S.ny - 1) face(vc, rc, xe(c + S.nx), rho[c + S.nx], q, dg); else wall(vc, rc, bm & 8, q, dg);
        if (k > 0) face(vc, rc, vzm, rzm, q, dg); else wall(vc, rc, bm & 16, q, dg);
        if (k < S.nz - 1) face(vc, rc, vzp, rzp, q, dg); else wall(vc, rc, bm & 32, q, dg);
        const bool solid = isinf(rc);
        const double r = solid ? 0.0 : (-S.h2 * S.rhs[c] - q);
        // inner diagonal from the FP32 densities, as the inner passes see it
        const float dg32 = diag_at<float>(rho32, c, t, k, S, fc, fzm, fzp);
        const float z32 = dg32 > 0.0f ? (float)((scale * r) / (double)dg32) : 0.0f;
        z[c] = z32;
        const double rz = (double)dg32 * (double)z32;
        a0 += r * r;
        a1 += rz * (double)z32;
        a2 += rz * rz;
        vzm = vc; rzm = rc; fzm = fc;
        vc = vzp; rc = rzp; fc = fzp;
    }
    acc[0] += a0;
    acc[1] += a1;
    acc[2] += a2;
}

// K2_IR_UPDATE: x += s d, d = 0.
__device__ void body_ir_update(const Slot &S, const SlotState &st, int64_t lt,
                               double (&acc)[3])
{
    const TileCtx t = tile_ctx(S, lt);
    if (!t.active) return;
    const double s = st.upd_s;
    int64_t c = (int64_t)t.k0 * t.P + t.q;
    for (int k = t.k0; k < t.k1; ++k, c += t.P) {
        S.x[c] = refined(S.x[c], s, S.d32[c]);
        S.d32[c] = 0.0f;
    }
}

// K2_ZERO_X: x = 0 (zero source with a warm start).
__device__ void body_zero_x(const Slot &S, const SlotState &st, int64_t lt,
                            double (&acc)[3])
{
    const TileCtx t = tile_ctx(S, lt);
    if (!t.active) return;
    int64_t c = (int64_t)t.k0 * t.P + t.q;
    for (int k = t.k0; k < t.k1; ++k, c += t.P) S.x[c] = 0.0;
}

// ------------------------------------------------------------------------
// state machine, run by one thread of the last workgroup of a launch
// ------------------------------------------------------------------------

__device__ void finish(SlotState &st, int code)
{
    st.status = code;
    st.phase = PH_DONE;
}

__device__ double pow2_scale(double norm)
{
    // power of two near 1/norm, so scaling is exact
    if (!(norm > 0.0) || !isfinite(norm)) return 1.0;
    return ldexp(1.0, -ilogb(norm));
}

__device__ void advance(SlotState &st, int phase, const double (&tot)[3])
{
    switch (phase) {
    case K1_INIT64: {
        st.bb = tot[0];
        if (!isfinite(tot[0])) { finish(st, PCG_EDOMAIN); break; }
        if (tot[0] == 0.0) {
            st.rr = st.rr_true = 0.0;
            if (st.warm) { st.phase = K2_ZERO_X; st.after = PH_DONE; }
            else finish(st, PCG_OK);
            break;
        }
        st.tol2 = st.tol * st.tol * tot[0];
        st.rz = tot[1];
        st.rr = tot[2];
        st.first = 1;
        st.phase = K2_NONE;
        st.after = (st.rr <= st.tol2 || st.maxit == 0) ? K1_CHECK64 : K1_CG_A;
        break;
    }
    case K1_CG_A: {
        const double pap = tot[0];
        if (!(pap > 0.0) || !isfinite(pap)) { finish(st, PCG_EBREAKDOWN); break; }
        st.pap = pap;
        st.alpha = st.rz / pap;
        st.pbuf ^= 1;
        st.first = 0;
        st.phase = K2_CG_B;
        break;
    }
    case K2_CG_B: {
        st.iter += 1;
        st.rr = tot[1];
        st.beta = tot[0] / st.rz;
        st.rz = tot[0];
        if (!isfinite(st.rr) || !isfinite(st.rz)) { finish(st, PCG_EBREAKDOWN); break; }
        st.phase = (st.rr <= st.tol2 || st.iter >= st.maxit) ? K1_CHECK64 : K1_CG_A;
        break;
    }
    case K1_CHECK64: {
        st.rr_true = tot[0];
        if (tot[0] <= st.tol2) { st.phase = K2_NONE; st.after = PH_DONE; st.status = PCG_OK; }
        else if (st.iter >= st.maxit) { st.phase = K2_NONE; st.after = PH_DONE; st.status = PCG_MAXIT; }
        else { st.phase = K2_NONE; st.after = K1_CG_A; }
        break;
    }
    case K2_NONE:
    case K2_ZERO_X:
        if (st.after == PH_DONE) {
            st.phase = PH_DONE;
            if (st.status == PCG_PENDING) st.status = PCG_OK;
        } else {
            st.phase = st.after;
        }
        break;
    case K1_IR_INIT: {
        st.bb = tot[0];
        if (!isfinite(tot[0])) { finish(st, PCG_EDOMAIN); break; }
        if (tot[0] == 0.0) {
            st.rr = st.rr_true = 0.0;
            if (st.warm) { st.phase = K2_ZERO_X; st.after = PH_DONE; }
            else finish(st, PCG_OK);
            break;
        }
        st.tol2 = st.tol * st.tol * tot[0];
        st.rr_true = tot[0];
        st.upd_s = 0.0;
        st.scale = pow2_scale(sqrt(tot[0]));
        st.phase = K2_NONE;
        st.after = K1_IR_RESID;
        break;
    }
    case K1_IR_RESID: {
        const double rr = tot[0];
        st.rr_true = rr;
        st.outer += 1;
        if (!isfinite(rr)) { finish(st, PCG_EBREAKDOWN); break; }
        st.phase = K2_IR_UPDATE;
        if (rr <= st.tol2) { st.final_upd = 1; st.status = PCG_OK; }
        else if (st.iter >= st.maxit || st.outer > kMaxOuter) { st.final_upd = 1; st.status = PCG_MAXIT; }
        else {
            st.final_upd = 0;
            st.rz = tot[1];
            st.rr0_inner = tot[2];
            st.rr = tot[2];
        }
        break;
    }
    case K2_IR_UPDATE: {
        if (st.final_upd) { st.phase = PH_DONE; break; }
        st.upd_s = 1.0 / st.scale;
        st.first = 1;
        st.inner_iter = 0;
        st.phase = K1_IR_A;
        break;
    }
    case K1_IR_A: {
        const double pap = tot[0];
        if (!isfinite(pap)) { finish(st, PCG_EBREAKDOWN); break; }
        if (!(pap > 0.0)) {  // the inner direction vanished: refine now
            st.scale = pow2_scale(sqrt(st.rr_true * st.inner_tol2));
            st.phase = K2_NONE;
            st.after = K1_IR_RESID;
            break;
        }
        st.pap = pap;
        st.alpha = st.rz / pap;
        st.pbuf ^= 1;
        st.first = 0;
        st.phase = K2_IR_B;
        break;
    }
    case K2_IR_B: {
        st.iter += 1;
        st.inner_iter += 1;
        st.rr = tot[1];
        st.beta = tot[0] / st.rz;
        st.rz = tot[0];
        if (!isfinite(st.rr)) { finish(st, PCG_EBREAKDOWN); break; }
        const bool inner_done = st.rr <= st.inner_tol2 * st.rr0_inner ||
                                st.inner_iter >= st.inner_maxit ||
                                st.iter >= st.maxit;
        if (inner_done) {
            st.scale = pow2_scale(sqrt(st.rr_true * st.inner_tol2));
            st.phase = K1_IR_RESID;
        } else {
            st.phase = K1_IR_A;
        }
        break;
    }
    default:
        break;
    }
}

// ------------------------------------------------------------------------
// launch skeleton
// ------------------------------------------------------------------------

template <int FAMILY>
__device__ __forceinline__ void run_body(int ph, const Slot &S,
                                         const SlotState &st, int64_t lt,
                                         double (&acc)[3])
{
    if (FAMILY == PCG_PREC_FP64) {
        switch (ph) {
        case K1_INIT64: body_init64(S, st, lt, acc); break;
        case K1_CG_A: body_passA<double>(S, st, lt, acc); break;
        case K1_CHECK64: body_check64(S, st, lt, acc); break;
        case K2_CG_B: body_passB<double, double>(S, st, lt, acc); break;
        case K2_ZERO_X: body_zero_x(S, st, lt, acc); break;
        default: break;
        }
    } else {
        switch (ph) {
        case K1_IR_INIT: body_ir_init(S, st, lt, acc); break;
        case K1_IR_RESID: body_ir_resid(S, st, lt, acc); break;
        case K1_IR_A: body_passA<float>(S, st, lt, acc); break;
        case K2_IR_B: body_passB<float, float>(S, st, lt, acc); break;
        case K2_IR_UPDATE: body_ir_update(S, st, lt, acc); break;
        case K2_ZERO_X: body_zero_x(S, st, lt, acc); break;
        default: break;
        }
    }
}

__device__ __forceinline__ bool is_k1(int ph) { return ph >= 1 && ph <= 10; }
__device__ __forceinline__ bool is_k2(int ph) { return ph >= 11 && ph <= 19; }

// Account `run` finished tiles of slot S; the last arrival sums the slot's
// per-tile partials in tile order and advances its state machine.
__device__ __forceinline__ void arrive(const Slot &S, int ph, uint32_t run,
                                       double *lds, int *s_last)
{
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t old = __hip_atomic_fetch_add(
            &S.st->ticket, run, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        *s_last = (int64_t)(old + run) == S.ntiles;
    }
    __syncthreads();
    if (*s_last) {
        __threadfence();
        double tot[3] = { 0.0, 0.0, 0.0 };
        for (int64_t t = threadIdx.x; t < S.ntiles; t += kBlock) {
            tot[0] += load_agent(S.partials + kMaxPartials * t + 0);
            tot[1] += load_agent(S.partials + kMaxPartials * t + 1);
            tot[2] += load_agent(S.partials + kMaxPartials * t + 2);
        }
        block_sum<3>(tot, lds);
        if (threadIdx.x == 0) {
            advance(*S.st, ph, tot);
            __hip_atomic_store(&S.st->ticket, 0u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
        }
    }
    __syncthreads();
}

template <int FAMILY>
__global__ void __launch_bounds__(kBlock)
k_iter(const BatchHeader *__restrict__ hdr, const Slot *__restrict__ slots,
       int which)
{
    __shared__ double lds[kMaxPartials * 4];
    __shared__ int s_last;
    const int64_t T = hdr->total_tiles;
    const int ns = hdr->nslots;
    const int G = (int)gridDim.x;
    const int g = xcd_major((int)blockIdx.x, G);
    int cur = -1, cur_ph = 0;
    uint32_t run = 0;
    for (int64_t t = g; t < T; t += G) {
        const int s = find_slot(slots, ns, t);
        const Slot &S = slots[s];
        if (s != cur) {
            if (run) arrive(slots[cur], cur_ph, run, lds, &s_last);
            cur = s;
            run = 0;
            cur_ph = S.st->phase;
        }
        const int ph = cur_ph;
        if (which == 1 ? !is_k1(ph) : !is_k2(ph)) continue;
        double acc[3] = { 0.0, 0.0, 0.0 };
        run_body<FAMILY>(ph, S, *S.st, t - S.tile_begin, acc);
        block_sum<3>(acc, lds);
        if (threadIdx.x == 0) {
            double *dst = S.partials + kMaxPartials * (t - S.tile_begin);
            store_agent(dst + 0, acc[0]);
            store_agent(dst + 1, acc[1]);
            store_agent(dst + 2, acc[2]);
        }
        ++run;
    }
    if (run) arrive(slots[cur], cur_ph, run, lds, &s_last);
}

// Density encoding: fluid keeps rho (checked > 0 and finite), hull -> +inf.
__global__ void __launch_bounds__(256)
k_encode(const double *__restrict__ rho, const uint8_t *__restrict__ mask,
         double *__restrict__ r64, float *__restrict__ r32, int64_t n,
         int *__restrict__ bad)
{
    int local_bad = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const bool solid = mask != nullptr && mask[c] != 0;
        double v = rho[c];
        if (solid) v = INFINITY;
        else if (!(v > 0.0) || !isfinite(v) || v > 1.0e37) local_bad = 1;
        r64[c] = v;
        if (r32) r32[c] = (float)v;
    }
    if (local_bad) atomicOr(bad, 1);
}

__global__ void __launch_bounds__(256)
k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, int64_t n2)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n2;
         c += (int64_t)gridDim.x * blockDim.x)
        dst[c] = src[c];
}

// ------------------------------------------------------------------------
// host-callable launchers
// ------------------------------------------------------------------------

hipError_t launch_iter(int family, int which, int grid,
                       const BatchHeader *hdr, const Slot *slots,
                       hipStream_t s)
{
    if (family == PCG_PREC_FP64)
        hipLaunchKernelGGL(k_iter<PCG_PREC_FP64>, dim3(grid), dim3(kBlock), 0, s,
                           hdr, slots, which);
    else
        hipLaunchKernelGGL(k_iter<PCG_PREC_FP32_IR>, dim3(grid), dim3(kBlock), 0,
                           s, hdr, slots, which);
    return hipGetLastError();
}

hipError_t launch_encode(const double *rho, const uint8_t *mask, double *r64,
                         float *r32, int64_t n, int *bad, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_encode, dim3((unsigned)blocks), dim3(256), 0, s, rho,
                       mask, r64, r32, n, bad);
    return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, size_t n, hipStream_t s)
{
    const int64_t n2 = (int64_t)(n / 2);
    int64_t blocks = (n2 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const double2 *)src, (double2 *)dst, n2);
    return hipGetLastError();
}

}  // namespace pcgmi
