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
// where x += alpha p is applied every third pass B, the two deferred
// updates first and in order (the directions rotate through three buffers).
// Each pass is one HBM sweep; the two global reductions per iteration are
// per-tile partial sums written to memory and added in tile order by the
// last workgroup to arrive, which also advances the solve's state machine.
//
// Work decomposition: a tile is cpt * kBlock consecutive cells of an x-y
// plane (x fastest) times tz planes, cpt = 1, or 2 / 4 when the row length
// allows; in passes A and B each thread owns cpt adjacent (i,j) columns of a
// row and marches up in z keeping the k-1, k, k+1 values in registers, so
// its loads are cpt elements wide.  With one resident solve a launch
// grid-strides over the tiles (workgroup ids remapped so each of the 8 XCDs
// walks a contiguous range, keeping the y-neighbour rows of concurrently
// running tiles in that XCD's L2); with several, each workgroup takes a
// contiguous range of tiles.
#include <hip/hip_runtime.h>
#include <math.h>
#include <type_traits>
#include <stdint.h>

#include <mutex>

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

struct TileCtx {
    int q;       // index of this thread's column in the x-y plane
    int i, j;
    int k0, k1;  // planes [k0, k1)
    int P;       // nx*ny
    bool active;
};

// Column of this thread in tile lt.  A tile holds S.cpt kBlock cells of a
// plane (S.cpt = 1, 2 or 4 cells per thread; 2 and 4 need a row length
// divisible by them): consecutive cells, or with S.tx > 0 a 2-D block of
// S.tx = S.cpt kBlock / S.ty columns x S.ty rows numbered row by row.  Phases that treat cells
// one by one take them in S.cpt coalesced runs (r: cells r kBlock + l of
// the tile); passes A and B give thread l the adjacent cells S.cpt l ..
// S.cpt l + S.cpt - 1 of one row (group_ctx).  On a 2-D tile i and j are
// set for every lane, also past the grid's edge (active false there).
__device__ __forceinline__ TileCtx tile_at(const Slot &S, int64_t lt, int q_in_tile)
{
    TileCtx t;
    const int pt = (int)(lt % S.plane_tiles);
    const int zt = (int)(lt / S.plane_tiles);
    t.P = S.nx * S.ny;
    if (S.tx > 0) {
        t.i = (pt % S.tiles_x) * S.tx + q_in_tile % S.tx;
        t.j = (pt / S.tiles_x) * S.ty + q_in_tile / S.tx;
        t.active = t.i < S.nx && t.j < S.ny;
        t.q = t.j * S.nx + t.i;
    } else {
        t.q = pt * (S.cpt * kBlock) + q_in_tile;
        t.active = t.q < t.P;
        t.i = t.q % S.nx;
        t.j = t.q / S.nx;
    }
    t.k0 = zt * S.tz;
    t.k1 = min(S.nz, t.k0 + S.tz);
    return t;
}

__device__ __forceinline__ TileCtx tile_ctx(const Slot &S, int64_t lt, int r = 0)
{
    return tile_at(S, lt, r * kBlock + (int)threadIdx.x);
}

// The first of this thread's adjacent cells (S.cpt > 1).
__device__ __forceinline__ TileCtx group_ctx(const Slot &S, int64_t lt)
{
    return tile_at(S, lt, S.cpt * (int)threadIdx.x);
}

// f(t) for each column of the thread in tile lt (S.cpt of them).
template <class F>
__device__ __forceinline__ void for_rows(const Slot &S, int64_t lt, F &&f)
{
    for (int r = 0; r < S.cpt; ++r) f(tile_ctx(S, lt, r));
}

// Global-address-space views: pointers read from the slot table are
// generic; casting them lets the compiler emit global (not flat) accesses.
#define GLB __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLB T *gp(T *p) { return (GLB T *)p; }
template <typename T>
__device__ __forceinline__ const GLB T *gp(const T *p) { return (const GLB T *)p; }

// The three direction buffers rotate: pass A reads buffer b (p_old) and
// writes b + 1 mod 3, so the two directions before the current one are
// still there when their x updates are applied.
__device__ __forceinline__ int dir_next(int b) { return b == 2 ? 0 : b + 1; }
__device__ __forceinline__ int dir_prev(int b) { return b == 0 ? 2 : b - 1; }
__device__ __forceinline__ void *dir_buf(const Slot &S, int b)
{
    return b == 0 ? S.dir0 : (b == 1 ? S.dir1 : S.dir2);
}

// Reciprocal of a positive finite value: hardware estimate refined by two
// Newton-Raphson steps (quadratic convergence from the ~2^-23 estimate).
__device__ __forceinline__ double recip(double d)
{
    double y = __builtin_amdgcn_rcp(d);
    double e = fma(-d, y, 1.0);
    y = fma(y, e, y);
    e = fma(-d, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ float recip(float d) { return __builtin_amdgcn_rcpf(d); }

// Face coefficient from the sum of the two densities on either side:
// beta = 1/((rho_c + rho_n)/2) = 2/(rho_c + rho_n).  A hull cell holds +inf,
// so the sum is +inf and beta = 0.  Walls use rho_n = 0 for Dirichlet
// (beta = 2/rho_c: the mirrored ghost -p_c) and +inf for Neumann (beta = 0).
template <typename T>
__device__ __forceinline__ T fb(T den)
{
    const T inf = (T)INFINITY;
    return den < inf ? T(2) * recip(den) : T(0);
}

// ------------------------------------------------------------------------
// coefficient sources
// ------------------------------------------------------------------------
// A body reads a "key" per cell and turns two keys into a face coefficient.
//  * RhoCoef: the key is the density (hull cells +inf); beta = 2/(a + b).
//    A wall stands in as a neighbour of density 0 (Dirichlet: beta = 2/rho_c,
//    the mirrored ghost) or +inf (Neumann: beta = 0).
//  * ClsCoef: the key is a one-byte density class; beta comes from a 16x16
//    table of exact 2/(rho_a + rho_b) held in LDS.  Class kClsWallD stands
//    for a Dirichlet wall, kClsSolid for the hull and Neumann walls.
// Both give the same operator; classes move 1 byte per cell instead of 8
// and need no reciprocal per face.

// Area fractions of the six faces of a cell (x-, x+, y-, y+, z-, z+): the
// weights of the face coefficients (and of the Dirichlet wall terms) in the
// finite-volume form with free-slip cut cells.  Without cut cells they are 1
// at compile time and the multiplications vanish.
template <typename T>
struct Areas6 {
    T xm, xp, ym, yp, zm, zp;
};

// Two consecutive values of T in one load.
// N consecutive values of T in one load.
template <typename T, int N> struct VecN {
    typedef T type __attribute__((ext_vector_type(N)));
};

template <typename T>
struct RhoCoef {
    using Key = T;
    const GLB T *__restrict__ rho;
    __device__ __forceinline__ Key load(int64_t c) const { return rho[c]; }
    template <int N>
    __device__ __forceinline__ void loadN(int64_t c, Key (&k)[N]) const
    {
        using V = typename VecN<T, N>::type;
        const V v = ((const GLB V *)rho)[c / N];
#pragma unroll
        for (int n = 0; n < N; ++n) k[n] = v[n];
    }
    __device__ __forceinline__ Key dirichlet() const { return T(0); }
    __device__ __forceinline__ Key neumann() const { return (T)INFINITY; }
    __device__ __forceinline__ bool solid(Key k) const { return isinf(k); }
    __device__ __forceinline__ T beta(Key a, Key b) const { return fb(a + b); }
    __device__ __forceinline__ Areas6<T> areas(int, int, int, int64_t) const
    {
        return { T(1), T(1), T(1), T(1), T(1), T(1) };
    }
};

template <typename T>
struct ClsCoef {
    using Key = int;
    const GLB uint8_t *__restrict__ cls;
    const T *tab;   // LDS, kClasses x kClasses
    __device__ __forceinline__ Key load(int64_t c) const { return cls[c]; }
    // the keys of cells c .. c + N - 1, c a multiple of N (one load)
    template <int N>
    __device__ __forceinline__ void loadN(int64_t c, Key (&k)[N]) const
    {
        static_assert(N == 2 || N == 4, "two or four cells");
        using W = typename std::conditional<
        N == 1, uint8_t, typename std::conditional<N == 2, uint16_t, uint32_t>::type>::type;
        const unsigned h = ((const GLB W *)cls)[c / N];
#pragma unroll
        for (int n = 0; n < N; ++n) k[n] = (int)((h >> (8 * n)) & 0xffu);
    }
    __device__ __forceinline__ Key dirichlet() const { return kClsWallD; }
    __device__ __forceinline__ Key neumann() const { return kClsSolid; }
    __device__ __forceinline__ bool solid(Key k) const { return k == kClsSolid; }
    __device__ __forceinline__ T beta(Key a, Key b) const { return tab[a * kClasses + b]; }
    __device__ __forceinline__ Areas6<T> areas(int, int, int, int64_t) const
    {
        return { T(1), T(1), T(1), T(1), T(1), T(1) };
    }
};

// Per-cell density with free-slip cut cells: the density key of RhoCoef and
// the area fractions of the MAC faces (FP64, converted for FP32 passes).  On
// a periodic axis the face beyond the last cell is the row's face 0.
template <typename T>
struct FracCoef {
    using Key = T;
    const GLB T *__restrict__ rho;
    const GLB double *__restrict__ ax;
    const GLB double *__restrict__ ay;
    const GLB double *__restrict__ az;
    int nx, ny;
    int64_t P;
    bool perx, pery;
    __device__ __forceinline__ Key load(int64_t c) const { return rho[c]; }
    template <int N>
    __device__ __forceinline__ void loadN(int64_t c, Key (&k)[N]) const
    {
        using V = typename VecN<T, N>::type;
        const V v = ((const GLB V *)rho)[c / N];
#pragma unroll
        for (int n = 0; n < N; ++n) k[n] = v[n];
    }
    __device__ __forceinline__ Key dirichlet() const { return T(0); }
    __device__ __forceinline__ Key neumann() const { return (T)INFINITY; }
    __device__ __forceinline__ bool solid(Key k) const { return isinf(k); }
    __device__ __forceinline__ T beta(Key a, Key b) const { return fb(a + b); }
    __device__ __forceinline__ Areas6<T> areas(int i, int j, int k, int64_t c) const
    {
        const int64_t fu = ((int64_t)k * ny + j) * (nx + 1) + i;
        const int64_t fv = ((int64_t)k * (ny + 1) + j) * nx + i;
        Areas6<T> a;
        a.xm = (T)ax[fu];
        a.xp = (T)ax[(perx && i == nx - 1) ? fu - i : fu + 1];
        a.ym = (T)ay[fv];
        a.yp = (T)ay[(pery && j == ny - 1) ? fv - (int64_t)j * nx : fv + nx];
        a.zm = (T)az[c];
        a.zp = (T)az[c + P];
        return a;
    }
};

template <typename T>
__device__ __forceinline__ FracCoef<T> frac_coef(const Slot &S, const T *rho)
{
    return { gp(rho), gp(S.ax), gp(S.ay), gp(S.az), S.nx, S.ny, (int64_t)S.nx * S.ny,
             (S.permask & 1) != 0, (S.permask & 2) != 0 };
}

// Volume fraction of cell c (1 without cut cells): weights the source.
__device__ __forceinline__ double vol_at(const Slot &S, int64_t c)
{
    return S.vol ? gp(S.vol)[c] : 1.0;
}

// Per-thread neighbour description for the x/y faces of a column: offset to
// the neighbour (across a periodic wall, the cell at the other end; 0 at
// any other wall, so the load stays in bounds) and the key standing in for
// a missing neighbour.
template <typename Key>
struct Nbr {
    int oxm, oxp, oym, oyp;
    bool hxm, hxp, hym, hyp;
    Key wxm, wxp, wym, wyp, wzm, wzp;
};

template <class C>
__device__ __forceinline__ Nbr<typename C::Key> make_nbr(const TileCtx &t,
                                                         const Slot &S, const C &cf)
{
    Nbr<typename C::Key> n;
    const int bm = S.bcmask;
    // periodic axes wrap to the other end of the row (x) or plane (y); an
    // axis of one cell keeps the wall form with no flux (the wall key of a
    // periodic wall is the Neumann one)
    const bool px = (S.permask & 1) && S.nx > 1, py = (S.permask & 2) && S.ny > 1;
    n.hxm = t.i > 0 || px;
    n.hxp = t.i < S.nx - 1 || px;
    n.hym = t.j > 0 || py;
    n.hyp = t.j < S.ny - 1 || py;
    n.oxm = t.i > 0 ? -1 : (px ? S.nx - 1 : 0);
    n.oxp = t.i < S.nx - 1 ? 1 : (px ? -(S.nx - 1) : 0);
    n.oym = t.j > 0 ? -S.nx : (py ? (S.ny - 1) * S.nx : 0);
    n.oyp = t.j < S.ny - 1 ? S.nx : (py ? -(S.ny - 1) * S.nx : 0);
    n.wxm = (bm & 1) ? cf.dirichlet() : cf.neumann();
    n.wxp = (bm & 2) ? cf.dirichlet() : cf.neumann();
    n.wym = (bm & 4) ? cf.dirichlet() : cf.neumann();
    n.wyp = (bm & 8) ? cf.dirichlet() : cf.neumann();
    n.wzm = (bm & 16) ? cf.dirichlet() : cf.neumann();
    n.wzp = (bm & 32) ? cf.dirichlet() : cf.neumann();
    return n;
}

// Full operator at one cell: q = (A v)_c, dg = A_cc, given the cell's value
// and key, the z neighbours (already substituted at walls: value 0 and wall
// key) and a fetch of v for the x/y neighbours.
template <typename T, class C, class Fetch>
__device__ __forceinline__ void apply_cell(Fetch v, const C &cf, int64_t c,
                                           const Nbr<typename C::Key> &n, T vc,
                                           typename C::Key kc, T vzm,
                                           typename C::Key kzm, T vzp,
                                           typename C::Key kzp, const Areas6<T> &ar,
                                           T &q, T &dg)
{
    using K = typename C::Key;
    // loads are unconditional (wall offsets are 0); walls substituted after
    const K lkxm = cf.load(c + n.oxm), lkxp = cf.load(c + n.oxp);
    const K lkym = cf.load(c + n.oym), lkyp = cf.load(c + n.oyp);
    const T lvxm = v(c + n.oxm), lvxp = v(c + n.oxp);
    const T lvym = v(c + n.oym), lvyp = v(c + n.oyp);
    const K kxm = n.hxm ? lkxm : n.wxm, kxp = n.hxp ? lkxp : n.wxp;
    const K kym = n.hym ? lkym : n.wym, kyp = n.hyp ? lkyp : n.wyp;
    const T vxm = n.hxm ? lvxm : T(0), vxp = n.hxp ? lvxp : T(0);
    const T vym = n.hym ? lvym : T(0), vyp = n.hyp ? lvyp : T(0);
    const T bxm = cf.beta(kc, kxm) * ar.xm, bxp = cf.beta(kc, kxp) * ar.xp;
    const T bym = cf.beta(kc, kym) * ar.ym, byp = cf.beta(kc, kyp) * ar.yp;
    const T bzm = cf.beta(kc, kzm) * ar.zm, bzp = cf.beta(kc, kzp) * ar.zp;
    dg = ((bxm + bxp) + (bym + byp)) + (bzm + bzp);
    q = ((bxm * (vc - vxm) + bxp * (vc - vxp)) + (bym * (vc - vym) + byp * (vc - vyp))) +
        (bzm * (vc - vzm) + bzp * (vc - vzp));
}

// Diagonal only.
template <typename T, class C>
__device__ __forceinline__ T diag_cell(const C &cf, int64_t c,
                                       const Nbr<typename C::Key> &n,
                                       typename C::Key kc, typename C::Key kzm,
                                       typename C::Key kzp, const Areas6<T> &ar)
{
    using K = typename C::Key;
    const K lkxm = cf.load(c + n.oxm), lkxp = cf.load(c + n.oxp);
    const K lkym = cf.load(c + n.oym), lkyp = cf.load(c + n.oyp);
    const K kxm = n.hxm ? lkxm : n.wxm, kxp = n.hxp ? lkxp : n.wxp;
    const K kym = n.hym ? lkym : n.wym, kyp = n.hyp ? lkyp : n.wyp;
    return ((cf.beta(kc, kxm) * ar.xm + cf.beta(kc, kxp) * ar.xp) +
            (cf.beta(kc, kym) * ar.ym + cf.beta(kc, kyp) * ar.yp)) +
           (cf.beta(kc, kzm) * ar.zm + cf.beta(kc, kzp) * ar.zp);
}

// x + s d, evaluated identically wherever the refined iterate is needed.
__device__ __forceinline__ double refined(double x, double s, float d)
{
    return fma(s, (double)d, x);
}

// ------------------------------------------------------------------------
// phase bodies (one tile each); acc[] receives this thread's partial sums.
// Every body marches its column up through planes k0..k1-1 carrying the
// k-1 and k values; z neighbours beyond the domain are replaced by the wall
// (value 0 and the wall's key).
// ------------------------------------------------------------------------

// K1_INIT64: b = -h^2 Sigma (0 on hull), r = b (cold) or b - A x0 (warm),
// z = r / diag, the direction buffers zeroed.  acc = [b.b, r.z, r.r].
template <class C>
__device__ void body_init64(const Slot &S, const SlotState &st, int64_t lt,
                            const C &cf, double (&acc)[3])
{
    using K = typename C::Key;
    for_rows(S, lt, [&](const TileCtx &t) {
        if (!t.active) return;
        GLB double *__restrict__ x = gp(S.x);
        GLB double *__restrict__ z = gp((double *)S.z);
        const GLB double *__restrict__ rhs = gp(S.rhs);
        GLB double *__restrict__ pa = gp((double *)S.dir0);
        GLB double *__restrict__ pb = gp((double *)S.dir1);
        GLB double *__restrict__ pc = gp((double *)S.dir2);
        const Nbr<K> n = make_nbr(t, S, cf);
        const bool warm = st.warm != 0;
        const int64_t P = t.P;
        // warm start: hull entries of x0 are read as 0 (they are cleared here)
        auto xv = [&](int64_t m) -> double {
            const K k = cf.load(m);
            const double v = x[m];
            return cf.solid(k) ? 0.0 : v;
        };
        int64_t c = (int64_t)t.k0 * P + t.q;
        K kc = cf.load(c);
        double xc = warm ? xv(c) : 0.0;
        K kzm = n.wzm;
        double xzm = 0.0;
        if (t.k0 > 0) { kzm = cf.load(c - P); if (warm) xzm = xv(c - P); }
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int k = t.k0; k < t.k1; ++k, c += P) {
            const bool top = k == S.nz - 1;
            K kzp = n.wzp;
            double xzp = 0.0;
            if (!top) { kzp = cf.load(c + P); if (warm) xzp = xv(c + P); }
            const bool solid = cf.solid(kc);
            const double b = solid ? 0.0 : -S.h2 * vol_at(S, c) * rhs[c] - st.bshift;
            double r, dg;
            if (warm) {
                double q;
                apply_cell<double>(xv, cf, c, n, xc, kc, xzm, kzm, xzp, kzp,
                                   cf.areas(t.i, t.j, k, c), q, dg);
                r = solid ? 0.0 : b - q;
                if (solid) x[c] = 0.0;
            } else {
                dg = diag_cell<double>(cf, c, n, kc, kzm, kzp, cf.areas(t.i, t.j, k, c));
                r = b;
                x[c] = 0.0;
            }
            const double zc = dg > 0.0 ? r / dg : 0.0;
            z[c] = zc;
            pa[c] = 0.0;
            pb[c] = 0.0;
            pc[c] = 0.0;
            a0 += b * b;
            a1 += r * zc;
            a2 += r * r;
            kzm = kc; xzm = xc;
            kc = kzp; xc = xzp;
        }
        acc[0] += a0;
        acc[1] += a1;
        acc[2] += a2;
    });
}

// ------------------------------------------------------------------------
// buffer addressing for pass A
// ------------------------------------------------------------------------
// Each array pass A streams is reached through a buffer resource (four
// scalar registers) based at the plane below the tile, a per-plane scalar
// byte offset, and a per-lane 32-bit byte offset fixed for the whole tile
// (the lane's column, or its x/y neighbour's).  Addresses then cost one
// vector register per neighbour direction instead of a 64-bit pointer per
// load, and the resource's record count bounds every access.  A tile spans
// at most tz + 2 planes, which set-up keeps under 2^32 bytes of 8-byte
// values.

// Dword 3 of a raw buffer resource on this architecture: 32-bit data format,
// no swizzle, no index stride.
constexpr int kRawBufferWord3 = 0x00020000;
// Cache-policy bit for streaming (non-temporal) accesses.
constexpr int kBufNT = 2;

struct Buf {
    __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ Buf make_buf(const void *base, uint32_t bytes)
{
    return { __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes,
                                               kRawBufferWord3) };
}

template <int AUX = 0>
__device__ __forceinline__ double bld(double *, Buf b, uint32_t v, uint32_t s)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.r, v, s, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ float bld(float *, Buf b, uint32_t v, uint32_t s)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, v, s, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ int bld(uint8_t *, Buf b, uint32_t v, uint32_t s)
{
    return (int)__builtin_amdgcn_raw_buffer_load_b8(b.r, v, s, AUX);
}
template <typename T, int AUX = 0>
__device__ __forceinline__ T bload(Buf b, uint32_t v, uint32_t s)
{
    return bld<AUX>((T *)nullptr, b, v, s);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void bstore_nt(Buf b, uint32_t v, uint32_t s, double x)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), b.r, v, s, kBufNT);
}
__device__ __forceinline__ void bstore_nt(Buf b, uint32_t v, uint32_t s, float x)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), b.r, v, s, kBufNT);
}

// N consecutive elements at byte offset v + s (a multiple of their total
// size): 8 or 16 B of floats or doubles, 2 or 4 class bytes.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int BYTES, int AUX>
__device__ __forceinline__ auto braw(Buf b, uint32_t v, uint32_t s)
{
    if constexpr (BYTES == 16) return __builtin_amdgcn_raw_buffer_load_b128(b.r, v, s, AUX);
    else if constexpr (BYTES == 8) return __builtin_amdgcn_raw_buffer_load_b64(b.r, v, s, AUX);
    else if constexpr (BYTES == 4) return __builtin_amdgcn_raw_buffer_load_b32(b.r, v, s, AUX);
    else return (unsigned)__builtin_amdgcn_raw_buffer_load_b16(b.r, v, s, AUX);
}
template <typename E, int N, int AUX = 0, typename K>
__device__ __forceinline__ void bloadN(Buf b, uint32_t v, uint32_t s, K (&out)[N])
{
    if constexpr (std::is_same<E, uint8_t>::value) {
        const unsigned h = braw<N, AUX>(b, v, s);
#pragma unroll
        for (int n = 0; n < N; ++n) out[n] = (K)((h >> (8 * n)) & 0xffu);
    } else {
        using V = typename VecN<E, N>::type;
        const V x = __builtin_bit_cast(V, braw<N * (int)sizeof(E), AUX>(b, v, s));
#pragma unroll
        for (int n = 0; n < N; ++n) out[n] = x[n];
    }
}
template <typename T, int N>
__device__ __forceinline__ void bstoreN_nt(Buf b, uint32_t v, uint32_t s, const T (&in)[N])
{
    using V = typename VecN<T, N>::type;
    V x;
#pragma unroll
    for (int n = 0; n < N; ++n) x[n] = in[n];
    if constexpr (sizeof(V) == 16)
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, x), b.r, v, s, kBufNT);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), b.r, v, s, kBufNT);
}

// Byte offsets of a lane's cell and its x/y neighbours within a plane
// (wall neighbours point at the cell itself), for elements of ES bytes.
struct LaneOff {
    uint32_t c, xm, xp, ym, yp;
};
template <typename Key>
__device__ __forceinline__ LaneOff lane_off(const TileCtx &t, const Nbr<Key> &n, int es)
{
    return { (uint32_t)t.q * es, (uint32_t)(t.q + n.oxm) * es, (uint32_t)(t.q + n.oxp) * es,
             (uint32_t)(t.q + n.oym) * es, (uint32_t)(t.q + n.oyp) * es };
}

// The tile's window of an array: planes [b0, e0) with b0 the plane below
// the tile (if any) and e0 the plane above it (if any).
struct Window {
    int b0, e0;
    int64_t P;
    template <typename T>
    __device__ __forceinline__ Buf buf(const T *a) const
    {
        return make_buf(a + (int64_t)b0 * P, (uint32_t)((int64_t)(e0 - b0) * P * sizeof(T)));
    }
    // byte offset of plane kk for elements of ES bytes
    __device__ __forceinline__ uint32_t so(int kk, int es) const
    {
        return (uint32_t)((int64_t)(kk - b0) * P * es);
    }
};

__device__ __forceinline__ Window tile_window(const TileCtx &t, const Slot &S)
{
    return { t.k0 > 0 ? t.k0 - 1 : 0, t.k1 < S.nz ? t.k1 + 1 : S.nz, (int64_t)t.P };
}

// Key source of a coefficient policy through a buffer.
template <typename T>
__device__ __forceinline__ const void *key_array(const RhoCoef<T> &cf) { return (const void *)cf.rho; }
template <typename T>
__device__ __forceinline__ const void *key_array(const ClsCoef<T> &cf) { return (const void *)cf.cls; }
template <typename T>
__device__ __forceinline__ const void *key_array(const FracCoef<T> &cf) { return (const void *)cf.rho; }
template <class C> struct KeyElem;
template <typename T> struct KeyElem<RhoCoef<T>> { using type = T; };
template <typename T> struct KeyElem<ClsCoef<T>> { using type = uint8_t; };
template <typename T> struct KeyElem<FracCoef<T>> { using type = T; };

// K1_CG_A / K1_IR_A: p_new = z + beta p_old, stored; the quadratic form
// p.Ap = sum over faces of beta_f (p_c - p_n)^2, each face counted once
// from the cell above it (x, y, z low faces), plus the wall terms
// (2/rho_c) p_c^2 of the Dirichlet walls.  Two load sets alternate, each
// refilled for the plane after next before the other's plane is computed,
// so a wave waits only for loads issued a plane earlier.
template <typename T, typename K>
struct PlaneA {
    T zc, qc, zxm, qxm, zym, qym;
    K kc, kxm, kym;
};

template <typename T, class C>
__device__ void body_passA(const Slot &S, const SlotState &st, int64_t lt,
                           const C &cf, double (&acc)[3])
{
    using K = typename C::Key;
    using KE = typename KeyElem<C>::type;
    const TileCtx t = tile_ctx(S, lt);
    if (!t.active) return;
    const Window W = tile_window(t, S);
    // the buffer index is the same in every lane (state written by the
    // previous launch); reading it from one lane keeps the resources scalar
    const int pbuf = __builtin_amdgcn_readfirstlane(st.pbuf);
    const Buf bps = W.buf((const T *)dir_buf(S, pbuf));
    const Buf bpd = W.buf((const T *)dir_buf(S, dir_next(pbuf)));
    const Buf bz = W.buf((const T *)S.z);
    const Buf bk = W.buf((const KE *)key_array(cf));
    // first direction: beta = 0.  p_old is then still read (it holds zeros
    // from the set-up phase or a finite earlier direction), which keeps the
    // loads unconditional.
    const T beta = st.first ? T(0) : (T)st.beta;
    const Nbr<K> n = make_nbr(t, S, cf);
    const LaneOff ov = lane_off(t, n, (int)sizeof(T));
    const LaneOff ok = lane_off(t, n, (int)sizeof(KE));
    const int bm = S.bcmask;
    // Dirichlet high walls of this column (x+, y+); z+ is added on the top plane
    const bool hwx = !n.hxp && (bm & 2), hwy = !n.hyp && (bm & 8);
    const int nz = S.nz;
    auto load = [&](int kk) {
        kk = kk < t.k1 ? kk : t.k1 - 1;    // past the tile's end: re-read its last plane
        const uint32_t sv = W.so(kk, sizeof(T)), sk = W.so(kk, sizeof(KE));
        PlaneA<T, K> L;
        L.zxm = bload<T>(bz, ov.xm, sv); L.qxm = bload<T>(bps, ov.xm, sv);
        L.zym = bload<T>(bz, ov.ym, sv); L.qym = bload<T>(bps, ov.ym, sv);
        L.kxm = bload<KE>(bk, ok.xm, sk); L.kym = bload<KE>(bk, ok.ym, sk);
        L.zc = bload<T>(bz, ov.c, sv); L.qc = bload<T>(bps, ov.c, sv);
        L.kc = bload<KE>(bk, ok.c, sk);
        return L;
    };
    T pzm = T(0);
    K kzm = n.wzm;
    if (t.k0 > 0) {
        const uint32_t sv = W.so(t.k0 - 1, sizeof(T)), sk = W.so(t.k0 - 1, sizeof(KE));
        pzm = bload<T>(bz, ov.c, sv) + beta * bload<T>(bps, ov.c, sv);
        kzm = bload<KE>(bk, ok.c, sk);
    }
    double a = 0.0;
    auto step = [&](const PlaneA<T, K> &L, int kk) {
        const T pc = L.zc + beta * L.qc;
        const K kxm = n.hxm ? L.kxm : n.wxm, kym = n.hym ? L.kym : n.wym;
        const T pxm = n.hxm ? L.zxm + beta * L.qxm : T(0);
        const T pym = n.hym ? L.zym + beta * L.qym : T(0);
        const T dx = pc - pxm, dy = pc - pym, dz = pc - pzm;
        const Areas6<T> ar = cf.areas(t.i, t.j, kk, (int64_t)kk * t.P + t.q);
        T s = (cf.beta(L.kc, kxm) * ar.xm * dx * dx + cf.beta(L.kc, kym) * ar.ym * dy * dy) +
              cf.beta(L.kc, kzm) * ar.zm * dz * dz;
        // Dirichlet high walls (x+, y+ of this column, z+ on the top plane),
        // each weighted by its area
        const T w = (hwx ? ar.xp : T(0)) + (hwy ? ar.yp : T(0)) +
                    ((kk == nz - 1 && (bm & 32)) ? ar.zp : T(0));
        s += w * cf.beta(L.kc, cf.dirichlet()) * (pc * pc);   // + 0 without walls
        a += (double)s;
        bstore_nt(bpd, ov.c, W.so(kk, sizeof(T)), pc);
        pzm = pc;
        kzm = L.kc;
    };
    PlaneA<T, K> A = load(t.k0), B;
    int k = t.k0;
    for (; k + 1 < t.k1; k += 2) {
        B = load(k + 1);
        step(A, k);
        A = load(k + 2);
        step(B, k + 1);
    }
    if (k < t.k1) step(A, k);
    acc[0] += a;
}

// K2_CG_B (T = double, X = double: x) / K2_IR_B (T = float, X = float: d):
// q = A p, z -= alpha q / diag; acc = [r.z, r.r] with r = diag z.  The low z
// face coefficient is carried from the plane below.  XM says what happens to
// x: 0 nothing (the update is left pending); 3 the two pending updates, then
// this one: x += alpha_p0 p_p0, += alpha_p1 p_p1,
// += alpha p, with p_p0 and p_p1 still in the other two direction buffers.
// Solves run 0, 0, 3, reading and writing x every third iteration only; the
// fused multiply-adds are those of one update per iteration, in order.
template <typename T, typename X, class C, int XM>
__device__ void body_passB(const Slot &S, const SlotState &st, int64_t lt,
                           const C &cf, double (&acc)[3])
{
    static_assert(XM == 0 || XM == 3, "x left pending, or caught up");
    using K = typename C::Key;
    const TileCtx t = tile_ctx(S, lt);
    if (!t.active) return;
    const int pbuf = st.pbuf;
    const GLB T *__restrict__ p = gp((const T *)dir_buf(S, pbuf));
    // the directions one and two iterations back
    const GLB T *__restrict__ pp1 = gp((const T *)dir_buf(S, dir_prev(pbuf)));
    const GLB T *__restrict__ pp0 = gp((const T *)dir_buf(S, dir_next(pbuf)));
    GLB T *__restrict__ z = gp((T *)S.z);
    GLB X *__restrict__ x = gp(std::is_same<X, double>::value ? (X *)S.x : (X *)S.d32);
    const T alpha = (T)st.alpha;
    const T alpha_p0 = (T)st.alpha_p0, alpha_p1 = (T)st.alpha_p1;
    const Nbr<K> n = make_nbr(t, S, cf);
    const int64_t P = t.P;
    int64_t c = (int64_t)t.k0 * P + t.q;
    T vc = p[c];
    K kc = cf.load(c);
    T vzm = T(0);
    K kzm = n.wzm;
    if (t.k0 > 0) { vzm = p[c - P]; kzm = cf.load(c - P); }
    T bzm = cf.beta(kc, kzm) * cf.areas(t.i, t.j, t.k0, c).zm;
    double a0 = 0.0, a1 = 0.0;
    for (int k = t.k0; k < t.k1; ++k, c += P) {
        const bool top = k == S.nz - 1;
        const int64_t cz = top ? c : c + P;
        const T vzp_l = p[cz];
        const K kzp_l = cf.load(cz);
        const K lkxm = cf.load(c + n.oxm), lkxp = cf.load(c + n.oxp);
        const K lkym = cf.load(c + n.oym), lkyp = cf.load(c + n.oyp);
        const T lvxm = p[c + n.oxm], lvxp = p[c + n.oxp];
        const T lvym = p[c + n.oym], lvyp = p[c + n.oyp];
        const X xc = XM ? __builtin_nontemporal_load(&x[c]) : X(0);
        const T po0 = XM == 3 ? __builtin_nontemporal_load(&pp0[c]) : T(0);
        const T po1 = XM == 3 ? __builtin_nontemporal_load(&pp1[c]) : T(0);
        T zc = __builtin_nontemporal_load(&z[c]);
        const T vzp = top ? T(0) : vzp_l;
        const K kzp = top ? n.wzp : kzp_l;
        const K kxm = n.hxm ? lkxm : n.wxm, kxp = n.hxp ? lkxp : n.wxp;
        const K kym = n.hym ? lkym : n.wym, kyp = n.hyp ? lkyp : n.wyp;
        const T vxm = n.hxm ? lvxm : T(0), vxp = n.hxp ? lvxp : T(0);
        const T vym = n.hym ? lvym : T(0), vyp = n.hyp ? lvyp : T(0);
        const Areas6<T> ar = cf.areas(t.i, t.j, k, c);
        const T bxm = cf.beta(kc, kxm) * ar.xm, bxp = cf.beta(kc, kxp) * ar.xp;
        const T bym = cf.beta(kc, kym) * ar.ym, byp = cf.beta(kc, kyp) * ar.yp;
        const T bzp = cf.beta(kc, kzp) * ar.zp;
        const T dg = ((bxm + bxp) + (bym + byp)) + (bzm + bzp);
        const T q = ((bxm * (vc - vxm) + bxp * (vc - vxp)) +
                     (bym * (vc - vym) + byp * (vc - vyp))) +
                    (bzm * (vc - vzm) + bzp * (vc - vzp));
        if (XM == 3)
            __builtin_nontemporal_store(
                fma((X)alpha, (X)vc, fma((X)alpha_p1, (X)po1, fma((X)alpha_p0, (X)po0, xc))), &x[c]);
        const T inv = dg > T(0) ? recip(dg) : T(0);   // hull rows keep z = 0
        zc -= alpha * q * inv;
        __builtin_nontemporal_store(zc, &z[c]);
        const double dd = (double)dg, dz = (double)zc;
        const double r = dd * dz;
        a0 += r * dz;
        a1 += r * r;
        vzm = vc;
        bzm = bzp;
        vc = vzp;
        kc = kzp;
    }
    acc[0] += a0;
    acc[1] += a1;
}

// One cell of pass B: the operator row from the cell's value and key and
// those of its six neighbours (walls already substituted), the low z face
// coefficient carried from the plane below (bzm, replaced by the high one),
// z -= alpha q / diag and the two dot terms; in the catch-up form (XM 3)
// also the three pending x updates.  Shared by the grouped and the
// LDS-staged pass so both evaluate a cell the same way.
template <typename T, typename X, class C, int XM>
__device__ __forceinline__ void passB_cell(const C &cf, const Areas6<T> &ar,
                                           typename C::Key kc, T vc, T vxm,
                                           typename C::Key kxm, T vxp, typename C::Key kxp,
                                           T vym, typename C::Key kym, T vyp,
                                           typename C::Key kyp, T vzm, T vzp,
                                           typename C::Key kz, T &bzm, T zc, T alpha,
                                           T alpha_p0, T alpha_p1, X xo, T po0, T po1,
                                           X &xn, T &zn, double &a0, double &a1)
{
    const T bxm = cf.beta(kc, kxm) * ar.xm, bxp = cf.beta(kc, kxp) * ar.xp;
    const T bym = cf.beta(kc, kym) * ar.ym;
    const T byp = cf.beta(kc, kyp) * ar.yp;
    const T bzp = cf.beta(kc, kz) * ar.zp;
    const T dg = ((bxm + bxp) + (bym + byp)) + (bzm + bzp);
    const T q = ((bxm * (vc - vxm) + bxp * (vc - vxp)) + (bym * (vc - vym) + byp * (vc - vyp))) +
                (bzm * (vc - vzm) + bzp * (vc - vzp));
    if (XM == 3) xn = fma((X)alpha, (X)vc, fma((X)alpha_p1, (X)po1, fma((X)alpha_p0, (X)po0, xo)));
    const T inv = dg > T(0) ? recip(dg) : T(0);   // hull rows keep z = 0
    zn = zc - alpha * q * inv;
    const double r = (double)dg * (double)zn;
    a0 += r * (double)zn;
    a1 += r * r;
    bzm = bzp;
}

// ------------------------------------------------------------------------
// grouped tiles: passes A and B on N adjacent columns per thread
// ------------------------------------------------------------------------
// With the row length divisible by N (2, or 4 for floats), a thread owns
// cells c .. c + N - 1 of a row: the group, its y and z neighbour groups
// and their class bytes come in one load each (16 B of doubles or 8/16 B of
// floats, 2/4 B of classes); inside the group the cells are each other's x
// neighbours, so only the column before the group (pass A) and the one after
// it (pass B) are element loads.  That divides the vector memory
// instructions per cell by about N.

template <typename T, typename K, int N>
struct GroupA {
    T z[N], q[N], zy[N], qy[N], zx, qx;
    K k[N], ky[N], kx;
};

template <typename T, class C, int N>
__device__ void group_passA(const Slot &S, const SlotState &st, int64_t lt,
                            const C &cf, double (&acc)[3])
{
    using K = typename C::Key;
    using KE = typename KeyElem<C>::type;
    const TileCtx t = group_ctx(S, lt);     // the group's first cell
    if (!t.active) return;                  // planes hold whole groups
    const Window W = tile_window(t, S);
    const int pbuf = __builtin_amdgcn_readfirstlane(st.pbuf);
    const Buf bps = W.buf((const T *)dir_buf(S, pbuf));
    const Buf bpd = W.buf((const T *)dir_buf(S, dir_next(pbuf)));
    const Buf bz = W.buf((const T *)S.z);
    const Buf bk = W.buf((const KE *)key_array(cf));
    const T beta = st.first ? T(0) : (T)st.beta;
    const int nx = S.nx, ny = S.ny, nz = S.nz, bm = S.bcmask;
    const bool px = (S.permask & 1) && nx > 1, py = (S.permask & 2) && ny > 1;
    const int i0 = t.i, j = t.j;
    // the column before the group (across a periodic x wall: the row's last)
    const bool hxm = i0 > 0 || px;
    const int oxm = i0 > 0 ? -1 : (px ? nx - 1 : 0);
    const bool hym = j > 0 || py;
    const int oym = j > 0 ? -nx : (py ? (ny - 1) * nx : 0);
    // Dirichlet high walls: x+ of the last cell, y+ of all
    const bool hwx = !(i0 + N - 1 < nx - 1 || px) && (bm & 2);
    const bool hwy = !(j < ny - 1 || py) && (bm & 8);
    const K wxm = (bm & 1) ? cf.dirichlet() : cf.neumann();
    const K wym = (bm & 4) ? cf.dirichlet() : cf.neumann();
    const K wzm = (bm & 16) ? cf.dirichlet() : cf.neumann();
    const uint32_t vc = (uint32_t)t.q * sizeof(T), vy = (uint32_t)(t.q + oym) * sizeof(T);
    const uint32_t vx = (uint32_t)(t.q + oxm) * sizeof(T);
    const uint32_t kc = (uint32_t)t.q * sizeof(KE), ky = (uint32_t)(t.q + oym) * sizeof(KE);
    const uint32_t kx = (uint32_t)(t.q + oxm) * sizeof(KE);
    auto load = [&](int kk) {
        kk = kk < t.k1 ? kk : t.k1 - 1;    // past the tile's end: re-read its last plane
        const uint32_t sv = W.so(kk, sizeof(T)), sk = W.so(kk, sizeof(KE));
        GroupA<T, K, N> L;
        bloadN<T>(bz, vc, sv, L.z);
        bloadN<T>(bps, vc, sv, L.q);
        bloadN<KE>(bk, kc, sk, L.k);
        bloadN<T>(bz, vy, sv, L.zy);
        bloadN<T>(bps, vy, sv, L.qy);
        bloadN<KE>(bk, ky, sk, L.ky);
        L.zx = bload<T>(bz, vx, sv);
        L.qx = bload<T>(bps, vx, sv);
        L.kx = bload<KE>(bk, kx, sk);
        return L;
    };
    T pzm[N];
    K kzm[N];
#pragma unroll
    for (int n = 0; n < N; ++n) { pzm[n] = T(0); kzm[n] = wzm; }
    if (t.k0 > 0) {
        const uint32_t sv = W.so(t.k0 - 1, sizeof(T)), sk = W.so(t.k0 - 1, sizeof(KE));
        T z[N], q[N];
        bloadN<T>(bz, vc, sv, z);
        bloadN<T>(bps, vc, sv, q);
        bloadN<KE>(bk, kc, sk, kzm);
#pragma unroll
        for (int n = 0; n < N; ++n) pzm[n] = z[n] + beta * q[n];
    }
    double a = 0.0;
    auto step = [&](const GroupA<T, K, N> &L, int kk) {
        const int64_t c0 = (int64_t)kk * t.P + t.q;
        const bool top = kk == nz - 1 && (bm & 32);
        T pl = hxm ? L.zx + beta * L.qx : T(0);   // x- value of the next cell
        K kl = hxm ? L.kx : wxm;
        T p[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            p[n] = L.z[n] + beta * L.q[n];
            const T pym = hym ? L.zy[n] + beta * L.qy[n] : T(0);
            const K kym = hym ? L.ky[n] : wym;
            const Areas6<T> ar = cf.areas(i0 + n, j, kk, c0 + n);
            const T dx = p[n] - pl, dy = p[n] - pym, dz = p[n] - pzm[n];
            T sn = (cf.beta(L.k[n], kl) * ar.xm * dx * dx + cf.beta(L.k[n], kym) * ar.ym * dy * dy) +
                   cf.beta(L.k[n], kzm[n]) * ar.zm * dz * dz;
            const T w = ((n == N - 1 && hwx) ? ar.xp : T(0)) + (hwy ? ar.yp : T(0)) +
                        (top ? ar.zp : T(0));
            sn += w * cf.beta(L.k[n], cf.dirichlet()) * (p[n] * p[n]);
            a += (double)sn;
            pzm[n] = p[n];
            kzm[n] = L.k[n];
            pl = p[n];
            kl = L.k[n];
        }
        bstoreN_nt<T, N>(bpd, vc, W.so(kk, sizeof(T)), p);
    };
    GroupA<T, K, N> A = load(t.k0), B;
    int k = t.k0;
    for (; k + 1 < t.k1; k += 2) {
        B = load(k + 1);
        step(A, k);
        A = load(k + 2);
        step(B, k + 1);
    }
    if (k < t.k1) step(A, k);
    acc[0] += a;
}

template <typename T, typename X, class C, int XM, int N>
__device__ void group_passB(const Slot &S, const SlotState &st, int64_t lt,
                            const C &cf, double (&acc)[3])
{
    using K = typename C::Key;
    using V = typename VecN<T, N>::type;
    const TileCtx t = group_ctx(S, lt);
    if (!t.active) return;
    const int pbuf = st.pbuf;
    const GLB T *__restrict__ p = gp((const T *)dir_buf(S, pbuf));
    // the directions one and two iterations back
    const GLB T *__restrict__ pp1 = gp((const T *)dir_buf(S, dir_prev(pbuf)));
    const GLB T *__restrict__ pp0 = gp((const T *)dir_buf(S, dir_next(pbuf)));
    GLB T *__restrict__ z = gp((T *)S.z);
    // x is the caller's array (FP64), read and written element by element;
    // the FP32 correction d is ours (aligned), in groups
    GLB X *__restrict__ x = gp(std::is_same<X, double>::value ? (X *)S.x : (X *)S.d32);
    constexpr bool kXGroup = std::is_same<X, float>::value;
    using XV = typename VecN<X, N>::type;
    const GLB V *__restrict__ pv = (const GLB V *)p;
    const GLB V *__restrict__ pv0 = (const GLB V *)pp0;
    const GLB V *__restrict__ pv1 = (const GLB V *)pp1;
    GLB V *__restrict__ zv = (GLB V *)z;
    const T alpha = (T)st.alpha;
    const T alpha_p0 = (T)st.alpha_p0, alpha_p1 = (T)st.alpha_p1;
    const int nx = S.nx, ny = S.ny, bm = S.bcmask;
    const bool px = (S.permask & 1) && nx > 1, py = (S.permask & 2) && ny > 1;
    const int i0 = t.i, j = t.j;
    const bool hxm = i0 > 0 || px, hxp = i0 + N - 1 < nx - 1 || px;
    const int oxm = i0 > 0 ? -1 : (px ? nx - 1 : 0);
    const int oxp = i0 + N - 1 < nx - 1 ? 1 : (px ? -(nx - 1) : 0);   // from the last cell
    const bool hym = j > 0 || py, hyp = j < ny - 1 || py;
    const int oym = j > 0 ? -nx : (py ? (ny - 1) * nx : 0);
    const int oyp = j < ny - 1 ? nx : (py ? -(ny - 1) * nx : 0);
    const K wxm = (bm & 1) ? cf.dirichlet() : cf.neumann();
    const K wxp = (bm & 2) ? cf.dirichlet() : cf.neumann();
    const K wym = (bm & 4) ? cf.dirichlet() : cf.neumann();
    const K wyp = (bm & 8) ? cf.dirichlet() : cf.neumann();
    const K wzm = (bm & 16) ? cf.dirichlet() : cf.neumann();
    const K wzp = (bm & 32) ? cf.dirichlet() : cf.neumann();
    const int64_t P = t.P;
    int64_t c = (int64_t)t.k0 * P + t.q;   // a multiple of N
    T vc[N], vzm[N], bzm[N];
    K kc[N];
    {
        const V v = pv[c / N];
#pragma unroll
        for (int n = 0; n < N; ++n) { vc[n] = v[n]; vzm[n] = T(0); }
    }
    cf.template loadN<N>(c, kc);
    K kzm[N];
#pragma unroll
    for (int n = 0; n < N; ++n) kzm[n] = wzm;
    if (t.k0 > 0) {
        const V v = pv[(c - P) / N];
#pragma unroll
        for (int n = 0; n < N; ++n) vzm[n] = v[n];
        cf.template loadN<N>(c - P, kzm);
    }
#pragma unroll
    for (int n = 0; n < N; ++n)
        bzm[n] = cf.beta(kc[n], kzm[n]) * cf.areas(i0 + n, j, t.k0, c + n).zm;
    double a0 = 0.0, a1 = 0.0;
    for (int k = t.k0; k < t.k1; ++k, c += P) {
        const bool top = k == S.nz - 1;
        const int64_t cz = top ? c : c + P;
        const V vzp_v = pv[cz / N];
        K kzp[N], kym[N], kyp[N];
        cf.template loadN<N>(cz, kzp);
        const V vym_v = pv[(c + oym) / N], vyp_v = pv[(c + oyp) / N];
        cf.template loadN<N>(c + oym, kym);
        cf.template loadN<N>(c + oyp, kyp);
        const T lvxm = p[c + oxm], lvxp = p[c + N - 1 + oxp];
        const K lkxm = cf.load(c + oxm), lkxp = cf.load(c + N - 1 + oxp);
        const V zc = __builtin_nontemporal_load(&zv[c / N]);
        X xo[N];
#pragma unroll
        for (int n = 0; n < N; ++n) xo[n] = X(0);
        if (XM) {
            if constexpr (kXGroup) {
                const XV xv = __builtin_nontemporal_load(&((GLB XV *)x)[c / N]);
#pragma unroll
                for (int n = 0; n < N; ++n) xo[n] = xv[n];
            } else {
#pragma unroll
                for (int n = 0; n < N; ++n) xo[n] = __builtin_nontemporal_load(&x[c + n]);
            }
        }
        T po0[N], po1[N];
#pragma unroll
        for (int n = 0; n < N; ++n) po0[n] = po1[n] = T(0);
        if (XM == 3) {
            const V v0 = __builtin_nontemporal_load(&pv0[c / N]);
            const V v1 = __builtin_nontemporal_load(&pv1[c / N]);
#pragma unroll
            for (int n = 0; n < N; ++n) { po0[n] = v0[n]; po1[n] = v1[n]; }
        }
        T zn[N];
        X xn[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const T vzp = top ? T(0) : vzp_v[n];
            const K kz = top ? wzp : kzp[n];
            const Areas6<T> ar = cf.areas(i0 + n, j, k, c + n);
            // x neighbours: inside the group, or the columns around it
            const T vxm = n > 0 ? vc[n - 1] : (hxm ? lvxm : T(0));
            const K kxm = n > 0 ? kc[n - 1] : (hxm ? lkxm : wxm);
            const T vxp = n < N - 1 ? vc[n + 1] : (hxp ? lvxp : T(0));
            const K kxp = n < N - 1 ? kc[n + 1] : (hxp ? lkxp : wxp);
            const T vym = hym ? vym_v[n] : T(0), vyp = hyp ? vyp_v[n] : T(0);
            passB_cell<T, X, C, XM>(cf, ar, kc[n], vc[n], vxm, kxm, vxp, kxp, vym,
                                    hym ? kym[n] : wym, vyp, hyp ? kyp[n] : wyp, vzm[n], vzp,
                                    kz, bzm[n], zc[n], alpha, alpha_p0, alpha_p1, xo[n],
                                    po0[n], po1[n], xn[n], zn[n], a0, a1);
        }
        if (XM) {
            if constexpr (kXGroup) {
                XV xv;
#pragma unroll
                for (int n = 0; n < N; ++n) xv[n] = xn[n];
                __builtin_nontemporal_store(xv, &((GLB XV *)x)[c / N]);
            } else {
#pragma unroll
                for (int n = 0; n < N; ++n) __builtin_nontemporal_store(xn[n], &x[c + n]);
            }
        }
        {
            V zv_n;
#pragma unroll
            for (int n = 0; n < N; ++n) zv_n[n] = zn[n];
            __builtin_nontemporal_store(zv_n, &zv[c / N]);
        }
#pragma unroll
        for (int n = 0; n < N; ++n) {
            vzm[n] = vc[n];
            vc[n] = top ? T(0) : vzp_v[n];
            kc[n] = top ? wzp : kzp[n];
        }
    }
    acc[0] += a0;
    acc[1] += a1;
}

// ------------------------------------------------------------------------
// LDS-staged passes on 2-D plane tiles (N = 2 FP64 or 4 FP32 cells per
// thread; the one-sweep iteration also N = 1, narrow tiles)
// ------------------------------------------------------------------------
// A tile is TX = N kBlock / kTileY columns x kTileY rows x tz planes (128 x 4
// for FP64, 256 x 4 for FP32, 64 x 4 narrow); thread l owns the group of N cells
// (N l mod TX, N l / TX) of the tile.  Per plane the tile's
// direction values and coefficient keys, with a one-cell x-y halo, are
// written to LDS (two plane buffers, one barrier per plane) and every cell
// reads its four in-plane neighbours from there; z neighbours are carried in
// registers.  Global traffic per pair and plane is then the pair's values
// and keys one plane up and its z (plus x and the two earlier directions in
// the catch-up form), instead of also loading the y rows above and below
// and the columns beside it: the y-halo rows (TX cells each) are loaded by
// threads 0 .. 2 TX / N - 1, the x-halo columns (kTileY cells each) by the
// next 2 kTileY threads.  Lanes past the grid's edge load clamped cells,
// take part in the barriers and store nothing.  The set-up keeps this form
// to grids whose periodic axes hold whole tiles, so a wrapped neighbour is
// always a halo cell.
template <int N> constexpr int tile_x() { return N * kBlock / kTileY; }
// LDS row: N - 1 pad cells, the left halo, TX cells, the right halo, N - 1
// pad cells, so every group of N cells is aligned to its size
template <int N> constexpr int lds_w() { return tile_x<N>() + 2 * N; }
constexpr int kLdsR = kTileY + 2;   // LDS rows: lower halo, kTileY rows, upper halo
static_assert(tile_x<2>() == kTileX && 2 * tile_x<2>() / 2 + 2 * kTileY <= kBlock &&
              2 * tile_x<4>() / 4 + 2 * kTileY <= kBlock,
              "the halo loads fit the workgroup");

template <typename T, typename KE, int N>
struct LdsPlanes {
    T v[2][kLdsR * lds_w<N>()];
    KE k[2][kLdsR * lds_w<N>()];
};

// One LDS buffer set per value type, key type and group width, shared by
// the forms of the passes in one kernel.
template <typename T, typename KE, int N>
__device__ __forceinline__ LdsPlanes<T, KE, N> &lds_planes()
{
    __shared__ __attribute__((aligned(16))) LdsPlanes<T, KE, N> s;
    return s;
}

// A group of N keys as one load returns it (N class bytes, or N
// densities), split into keys only where they are used: splitting right
// after the load would make the wave wait for it before the plane's barrier.
template <class C, int N> struct KeyGroup;
template <typename T, int N> struct KeyGroup<ClsCoef<T>, N> {
    using W = typename std::conditional<
        N == 1, uint8_t, typename std::conditional<N == 2, uint16_t, uint32_t>::type>::type;
    using raw = unsigned;
    static __device__ __forceinline__ raw load(const ClsCoef<T> &cf, int64_t c)
    {
        return ((const GLB W *)cf.cls)[c / N];
    }
    static __device__ __forceinline__ void split(raw r, int (&k)[N])
    {
#pragma unroll
        for (int n = 0; n < N; ++n) k[n] = (int)((r >> (8 * n)) & 0xffu);
    }
    static __device__ __forceinline__ void put(uint8_t *a, raw r) { *(W *)a = (W)r; }
    static __device__ __forceinline__ raw get(const uint8_t *a) { return *(const W *)a; }
    // key `sel` of a group by shifts: a select over split keys is turned
    // back into an indexed (scratch) array
    static __device__ __forceinline__ uint8_t elem(raw r, int sel)
    {
        return (uint8_t)((r >> (8 * sel)) & 0xffu);
    }
};
template <typename T, int N> struct KeyGroup<RhoCoef<T>, N> {
    using raw = typename VecN<T, N>::type;
    static __device__ __forceinline__ raw load(const RhoCoef<T> &cf, int64_t c)
    {
        return ((const GLB raw *)cf.rho)[c / N];
    }
    static __device__ __forceinline__ void split(raw r, T (&k)[N])
    {
#pragma unroll
        for (int n = 0; n < N; ++n) k[n] = r[n];
    }
    static __device__ __forceinline__ void put(T *a, raw r) { *(raw *)a = r; }
    static __device__ __forceinline__ raw get(const T *a) { return *(const raw *)a; }
    static __device__ __forceinline__ T elem(raw r, int sel)
    {
        T e = r[0];
#pragma unroll
        for (int n = 1; n < N; ++n) e = sel == n ? r[n] : e;
        return e;
    }
};

// Element `sel` of a group (a select chain, no indexed register access).
template <typename E, int N, typename G>
__device__ __forceinline__ E pick(const G &g, int sel)
{
    E e = g[0];
#pragma unroll
    for (int n = 1; n < N; ++n) e = sel == n ? g[n] : e;
    return e;
}

template <typename T, typename X, class C, int XM, int N>
__device__ void lds_passB(const Slot &S, const SlotState &st, int64_t lt, const C &cf,
                          double (&acc)[3])
{
    constexpr int TX = tile_x<N>(), W = lds_w<N>();
    using K = typename C::Key;
    using KE = typename KeyElem<C>::type;
    using KP = KeyGroup<C, N>;
    using KR = typename KP::raw;
    using V = typename VecN<T, N>::type;
    using XV = typename VecN<X, N>::type;
    constexpr bool kXGroup = std::is_same<X, float>::value;   // d: ours, aligned
    LdsPlanes<T, KE, N> &L = lds_planes<T, KE, N>();
    const int l = (int)threadIdx.x;
    const TileCtx t = group_ctx(S, lt);
    const int ii = (N * l) % TX, jj = (N * l) / TX;
    const int ti0 = t.i - ii, tj0 = t.j - jj;       // the tile's first column and row
    const int nx = S.nx, ny = S.ny, nz = S.nz, bm = S.bcmask;
    const bool px = (S.permask & 1) && nx > 1, py = (S.permask & 2) && ny > 1;
    const int64_t P = t.P;
    const int pbuf = st.pbuf;
    const GLB T *__restrict__ p = gp((const T *)dir_buf(S, pbuf));
    const GLB T *__restrict__ pp1 = gp((const T *)dir_buf(S, dir_prev(pbuf)));
    const GLB T *__restrict__ pp0 = gp((const T *)dir_buf(S, dir_next(pbuf)));
    GLB X *__restrict__ x = gp(std::is_same<X, double>::value ? (X *)S.x : (X *)S.d32);
    const GLB V *__restrict__ pv = (const GLB V *)p;
    const GLB V *__restrict__ pv0 = (const GLB V *)pp0;
    const GLB V *__restrict__ pv1 = (const GLB V *)pp1;
    GLB V *__restrict__ zv = (GLB V *)gp((T *)S.z);
    const T alpha = (T)st.alpha;
    const T alpha_p0 = (T)st.alpha_p0, alpha_p1 = (T)st.alpha_p1;
    // this lane's group, clamped into the grid for lanes past its edge
    const int64_t qo = (int64_t)min(t.j, ny - 1) * nx + min(t.i, nx - N);
    const int own = (jj + 1) * W + ii + N;
    // halo role: a group of the row below or above the tile, or one cell of
    // the column left or right of it (wrapped on periodic axes, clamped at
    // walls, where the cells that would use it substitute the wall); an
    // x-halo cell comes with the other cells of its aligned group
    const bool yh = l < 2 * TX / N;
    const bool xh = !yh && l < 2 * TX / N + 2 * kTileY;
    int64_t qh = qo;       // group-aligned source; lanes without a role reload their own
    int hsel = 0, hslot = 0;
    if (yh) {
        const int up = l / (TX / N), hi = N * (l % (TX / N));
        int jy = up ? tj0 + kTileY : tj0 - 1;
        jy = py ? (jy + ny) % ny : max(0, min(ny - 1, jy));
        qh = (int64_t)jy * nx + min(ti0 + hi, nx - N);
        hslot = (up ? kTileY + 1 : 0) * W + hi + N;
    } else if (xh) {
        const int c = l - 2 * TX / N, right = c / kTileY, hj = c % kTileY;
        int ix = right ? ti0 + TX : ti0 - 1;
        ix = px ? (ix + nx) % nx : max(0, min(nx - 1, ix));
        const int64_t q1 = (int64_t)min(tj0 + hj, ny - 1) * nx + ix;
        qh = q1 & ~(int64_t)(N - 1);
        hsel = (int)(q1 & (N - 1));
        hslot = (hj + 1) * W + (right ? TX + N : N - 1);
    }
    // the waves holding halo lanes load in every lane (no divergent branch
    // around loads whose results must stay in flight); the others skip
    const bool hwave = __builtin_amdgcn_readfirstlane(l) < 2 * TX / N + 2 * kTileY;
    const int i0 = t.i, j = t.j;
    const bool hxm = i0 > 0 || px, hxp = i0 + N - 1 < nx - 1 || px;
    const bool hym = j > 0 || py, hyp = j < ny - 1 || py;
    const K wxm = (bm & 1) ? cf.dirichlet() : cf.neumann();
    const K wxp = (bm & 2) ? cf.dirichlet() : cf.neumann();
    const K wym = (bm & 4) ? cf.dirichlet() : cf.neumann();
    const K wyp = (bm & 8) ? cf.dirichlet() : cf.neumann();
    const K wzm = (bm & 16) ? cf.dirichlet() : cf.neumann();
    const K wzp = (bm & 32) ? cf.dirichlet() : cf.neumann();
    // halo values of a plane as loaded (a group)
    struct Halo {
        V v;
        KR kp;
    };
    auto load_halo = [&](int64_t base) {
        Halo h{};
        if (hwave) {
            h.v = pv[(base + qh) / N];
            h.kp = KP::load(cf, base + qh);
        }
        return h;
    };
    int64_t c = (int64_t)t.k0 * P;   // plane base
    T vc[N], vzm[N], bzm[N];
    K kc[N], kzm[N];
    V vcv = pv[(c + qo) / N];
    KR kcr = KP::load(cf, c + qo);
#pragma unroll
    for (int n = 0; n < N; ++n) {
        vc[n] = vcv[n];
        vzm[n] = T(0);
        kzm[n] = wzm;
    }
    KP::split(kcr, kc);
    if (t.k0 > 0) {
        const V v = pv[(c - P + qo) / N];
#pragma unroll
        for (int n = 0; n < N; ++n) vzm[n] = v[n];
        KP::split(KP::load(cf, c - P + qo), kzm);
    }
    Halo h = load_halo(c);
#pragma unroll
    for (int n = 0; n < N; ++n)
        bzm[n] = cf.beta(kc[n], kzm[n]) * cf.areas(i0 + n, j, t.k0, c + qo + n).zm;
    double a0 = 0.0, a1 = 0.0;
    for (int k = t.k0; k < t.k1; ++k, c += P) {
        const int b = (k - t.k0) & 1;
        T *Lv = L.v[b];
        KE *Lk = L.k[b];
        // stage plane k: this lane's group and its halo cells, as loaded
        *(V *)(Lv + own) = vcv;
        KP::put(Lk + own, kcr);
        if (yh) {
            *(V *)(Lv + hslot) = h.v;
            KP::put(Lk + hslot, h.kp);
        } else if (xh) {
            Lv[hslot] = pick<T, N>(h.v, hsel);
            Lk[hslot] = KP::elem(h.kp, hsel);
        }
        // loads for the next plane and this plane's vectors, left unsplit
        // and unused until after the barrier so they stay in flight across it
        const bool top = k == nz - 1;
        const int64_t cn = top ? c : c + P;
        const V vzp_v = pv[(cn + qo) / N];
        const KR kzpr = KP::load(cf, cn + qo);
        const Halo hn = load_halo(cn);
        const V zc = __builtin_nontemporal_load(&zv[(c + qo) / N]);
        X xo[N];
        V v0, v1;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            xo[n] = X(0);
            v0[n] = v1[n] = T(0);
        }
        if (XM == 3) {
            if constexpr (kXGroup) {
                const XV xv = __builtin_nontemporal_load(&((GLB XV *)x)[(c + qo) / N]);
#pragma unroll
                for (int n = 0; n < N; ++n) xo[n] = xv[n];
            } else {
#pragma unroll
                for (int n = 0; n < N; ++n) xo[n] = __builtin_nontemporal_load(&x[c + qo + n]);
            }
            v0 = __builtin_nontemporal_load(&pv0[(c + qo) / N]);
            v1 = __builtin_nontemporal_load(&pv1[(c + qo) / N]);
        }
        __syncthreads();
        const V vym = *(const V *)(Lv + own - W), vyp = *(const V *)(Lv + own + W);
        K kym[N], kyp[N], kzp[N];
        KP::split(KP::get(Lk + own - W), kym);
        KP::split(KP::get(Lk + own + W), kyp);
        KP::split(kzpr, kzp);
        const T lvxm = Lv[own - 1], lvxp = Lv[own + N];
        const K lkxm = (K)Lk[own - 1], lkxp = (K)Lk[own + N];
        T zn[N];
        X xn[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const T vzp = top ? T(0) : vzp_v[n];
            const K kz = top ? wzp : kzp[n];
            const Areas6<T> ar = cf.areas(i0 + n, j, k, c + qo + n);
            const T vxm = n > 0 ? vc[n - 1] : (hxm ? lvxm : T(0));
            const K kxm = n > 0 ? kc[n - 1] : (hxm ? lkxm : wxm);
            const T vxp = n < N - 1 ? vc[n + 1] : (hxp ? lvxp : T(0));
            const K kxp = n < N - 1 ? kc[n + 1] : (hxp ? lkxp : wxp);
            passB_cell<T, X, C, XM>(cf, ar, kc[n], vc[n], vxm, kxm, vxp, kxp,
                                    hym ? vym[n] : T(0), hym ? kym[n] : wym,
                                    hyp ? vyp[n] : T(0), hyp ? kyp[n] : wyp, vzm[n], vzp, kz,
                                    bzm[n], zc[n], alpha, alpha_p0, alpha_p1, xo[n], v0[n],
                                    v1[n], xn[n], zn[n], a0, a1);
        }
        if (t.active) {
            if (XM == 3) {
                if constexpr (kXGroup) {
                    XV xv;
#pragma unroll
                    for (int n = 0; n < N; ++n) xv[n] = xn[n];
                    __builtin_nontemporal_store(xv, &((GLB XV *)x)[(c + qo) / N]);
                } else {
#pragma unroll
                    for (int n = 0; n < N; ++n) __builtin_nontemporal_store(xn[n], &x[c + qo + n]);
                }
            }
            V zv_n;
#pragma unroll
            for (int n = 0; n < N; ++n) zv_n[n] = zn[n];
            __builtin_nontemporal_store(zv_n, &zv[(c + qo) / N]);
        }
        // the top plane's neighbour above is the wall: its staged copy is
        // never read, so the plane simply repeats
#pragma unroll
        for (int n = 0; n < N; ++n) {
            vzm[n] = vc[n];
            vc[n] = top ? T(0) : vzp_v[n];
            kc[n] = top ? wzp : kzp[n];
        }
        vcv = vzp_v;
        kcr = kzpr;
        h = hn;
    }
    if (t.active) {
        acc[0] += a0;
        acc[1] += a1;
    }
}

// Pass A on 2-D plane tiles with LDS staging: p = z + beta p_old for the
// tile's groups, stored, and written to LDS together with the keys; the
// row below the tile (threads 0 .. TX/N - 1, groups) and the column left of
// it (the next kTileY threads, one cell each) compute their p the same way
// into the halo.  After the plane's barrier every cell reads its x- and y-
// neighbours from LDS (pass A counts each face once, from its upper cell);
// the z- neighbour is carried in registers.  The next plane's loads are
// issued before the barrier and used after it.
template <typename T, class C, int N>
__device__ void lds_passA(const Slot &S, const SlotState &st, int64_t lt, const C &cf,
                          double (&acc)[3])
{
    constexpr int TX = tile_x<N>(), W = lds_w<N>();
    using K = typename C::Key;
    using KE = typename KeyElem<C>::type;
    using KP = KeyGroup<C, N>;
    using KR = typename KP::raw;
    using V = typename VecN<T, N>::type;
    LdsPlanes<T, KE, N> &L = lds_planes<T, KE, N>();
    const int l = (int)threadIdx.x;
    const TileCtx t = group_ctx(S, lt);
    const int ii = (N * l) % TX, jj = (N * l) / TX;
    const int ti0 = t.i - ii, tj0 = t.j - jj;
    const int nx = S.nx, ny = S.ny, nz = S.nz, bm = S.bcmask;
    const bool px = (S.permask & 1) && nx > 1, py = (S.permask & 2) && ny > 1;
    const int64_t P = t.P;
    const int pbuf = __builtin_amdgcn_readfirstlane(st.pbuf);
    const GLB V *__restrict__ zv = (const GLB V *)gp((const T *)S.z);
    const GLB V *__restrict__ qv = (const GLB V *)gp((const T *)dir_buf(S, pbuf));
    GLB V *__restrict__ pdv = (GLB V *)gp((T *)dir_buf(S, dir_next(pbuf)));
    // first direction: beta = 0 (p_old holds zeros from the set-up, or a
    // finite earlier direction, so the loads stay unconditional)
    const T beta = st.first ? T(0) : (T)st.beta;
    const int64_t qo = (int64_t)min(t.j, ny - 1) * nx + min(t.i, nx - N);
    const int own = (jj + 1) * W + ii + N;
    const bool yh = l < TX / N;
    const bool xh = !yh && l < TX / N + kTileY;
    int64_t qh = qo;
    int hsel = 0, hslot = 0;
    if (yh) {
        const int hi = N * l;
        int jy = tj0 - 1;
        jy = py ? (jy + ny) % ny : max(0, jy);
        qh = (int64_t)jy * nx + min(ti0 + hi, nx - N);
        hslot = hi + N;
    } else if (xh) {
        const int hj = l - TX / N;
        int ix = ti0 - 1;
        ix = px ? (ix + nx) % nx : max(0, ix);
        const int64_t q1 = (int64_t)min(tj0 + hj, ny - 1) * nx + ix;
        qh = q1 & ~(int64_t)(N - 1);
        hsel = (int)(q1 & (N - 1));
        hslot = (hj + 1) * W + N - 1;
    }
    const bool hwave = __builtin_amdgcn_readfirstlane(l) < TX / N + kTileY;
    const int i0 = t.i, j = t.j;
    const bool hxm = i0 > 0 || px, hym = j > 0 || py;
    // Dirichlet high walls: x+ of the group's last cell, y+ of all
    const bool hwx = !(i0 + N - 1 < nx - 1 || px) && (bm & 2);
    const bool hwy = !(j < ny - 1 || py) && (bm & 8);
    const K wxm = (bm & 1) ? cf.dirichlet() : cf.neumann();
    const K wym = (bm & 4) ? cf.dirichlet() : cf.neumann();
    const K wzm = (bm & 16) ? cf.dirichlet() : cf.neumann();
    struct Plane {
        V z, q, hz, hq;
        KR k, hk;
    };
    auto load = [&](int kk) {
        kk = kk < t.k1 ? kk : t.k1 - 1;    // past the tile's end: re-read its last plane
        const int64_t base = (int64_t)kk * P;
        Plane A;
        A.z = zv[(base + qo) / N];
        A.q = qv[(base + qo) / N];
        A.k = KP::load(cf, base + qo);
        if (hwave) {
            A.hz = zv[(base + qh) / N];
            A.hq = qv[(base + qh) / N];
            A.hk = KP::load(cf, base + qh);
        }
        return A;
    };
    T pzm[N];
    K kzm[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        pzm[n] = T(0);
        kzm[n] = wzm;
    }
    if (t.k0 > 0) {
        const int64_t base = (int64_t)(t.k0 - 1) * P;
        const V z = zv[(base + qo) / N], q = qv[(base + qo) / N];
#pragma unroll
        for (int n = 0; n < N; ++n) pzm[n] = z[n] + beta * q[n];
        KP::split(KP::load(cf, base + qo), kzm);
    }
    double a = 0.0;
    Plane A = load(t.k0);
    for (int k = t.k0; k < t.k1; ++k) {
        const int b = (k - t.k0) & 1;
        T *Lv = L.v[b];
        KE *Lk = L.k[b];
        V pn;
#pragma unroll
        for (int n = 0; n < N; ++n) pn[n] = A.z[n] + beta * A.q[n];
        K kc[N];
        KP::split(A.k, kc);
        *(V *)(Lv + own) = pn;
        KP::put(Lk + own, A.k);
        if (yh) {
            V hp;
#pragma unroll
            for (int n = 0; n < N; ++n) hp[n] = A.hz[n] + beta * A.hq[n];
            *(V *)(Lv + hslot) = hp;
            KP::put(Lk + hslot, A.hk);
        } else if (xh) {
            Lv[hslot] = pick<T, N>(A.hz, hsel) + beta * pick<T, N>(A.hq, hsel);
            Lk[hslot] = KP::elem(A.hk, hsel);
        }
        if (t.active) __builtin_nontemporal_store(pn, &pdv[((int64_t)k * P + qo) / N]);
        const Plane B = load(k + 1);
        __syncthreads();
        const bool top = k == nz - 1 && (bm & 32);
        const V pym_v = *(const V *)(Lv + own - W);
        K kym[N];
        KP::split(KP::get(Lk + own - W), kym);
        T pl = hxm ? Lv[own - 1] : T(0);          // x- value of the next cell
        K kl = hxm ? (K)Lk[own - 1] : wxm;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const T pym = hym ? pym_v[n] : T(0);
            const K kyn = hym ? kym[n] : wym;
            const Areas6<T> ar = cf.areas(i0 + n, j, k, (int64_t)k * P + qo + n);
            const T dx = pn[n] - pl, dy = pn[n] - pym, dz = pn[n] - pzm[n];
            T sn = (cf.beta(kc[n], kl) * ar.xm * dx * dx + cf.beta(kc[n], kyn) * ar.ym * dy * dy) +
                   cf.beta(kc[n], kzm[n]) * ar.zm * dz * dz;
            const T w = ((n == N - 1 && hwx) ? ar.xp : T(0)) + (hwy ? ar.yp : T(0)) +
                        (top ? ar.zp : T(0));
            sn += w * cf.beta(kc[n], cf.dirichlet()) * (pn[n] * pn[n]);
            a += (double)sn;
            pzm[n] = pn[n];
            kzm[n] = kc[n];
            pl = pn[n];
            kl = kc[n];
        }
        A = B;
    }
    if (t.active) acc[0] += a;
}

// ------------------------------------------------------------------------
// One-sweep iteration on plane tiles
// ------------------------------------------------------------------------
// The Chronopoulos-Gear form of the iteration: with alpha and beta known at
// the start of a sweep (both from the previous sweep's sums), one pass over
// the grid forms p = z + beta p_old, q = A p, z' = z - alpha D^-1 q and x +=
// alpha p (three directions at a time, as in pass B), and sums r.z = z'.D z',
// r.r and delta = z'.A z'.  The next step length is alpha' = (r.z)' / (delta
// - beta' (r.z)' / alpha), equal to (r.z)' / p'.A p' in exact arithmetic, so
// the iterates are those of the two-sweep iteration up to rounding, for 17
// bytes read and 16 written per cell instead of 34 and 16.  delta is summed
// over faces, each from its upper cell as in pass A, which needs z' in the
// column left of the tile and the row below it, and those cells' q needs p
// one cell further out: per plane the tile's groups and a halo two cells
// deep on the low sides and one deep on the high sides stage p and the keys
// in LDS, the row below the tile (threads 0 .. TX/N - 1) and the column left
// of it (groups of N cells ending there, kTileY threads) compute z' as the
// tile's own groups do, and z' is staged in a second LDS plane; one barrier
// per plane.  z is read from one buffer and written to the other, since a
// sweep reads z in the tiles beside its own while they are written.  A tile
// above the bottom of the grid starts one plane low: that plane's z' serves
// the faces below the tile and nothing is stored or summed for it.
constexpr int kLdsS = kTileY + 3;   // LDS rows: y0 - 2 .. y0 + kTileY
// LDS row of the sweep: the left halo two cells deep (a group of N cells
// ending at the tile, or for N = 1 two cells: the z' of the column left of
// the tile needs p one cell further out), the TX cells, the right halo (a
// group), so every group of N cells is aligned to its size
template <int N> constexpr int sweep_left() { return N > 1 ? N : 2; }
template <int N> constexpr int sweep_w() { return tile_x<N>() + sweep_left<N>() + N; }

template <typename T, typename KE, int N>
struct LdsSweep {
    T p[2][kLdsS * sweep_w<N>()];
    T z[2][kLdsS * sweep_w<N>()];
    KE k[2][kLdsS * sweep_w<N>()];
};

// One LDS block per value and key type, sized for the widest groups of that
// type (two FP64 or four FP32 cells a thread); one-cell-a-thread tiles use
// a smaller view of the same block.  A workgroup's tiles are separated by
// the barrier of their block sum, so the views never overlap in time.
template <typename T, typename KE>
__device__ __forceinline__ void *lds_sweep_block()
{
    constexpr int NW = sizeof(T) == 8 ? 2 : 4;
    __shared__ __attribute__((aligned(16))) LdsSweep<T, KE, NW> s;
    return &s;
}

template <typename T, typename KE, int N>
__device__ __forceinline__ LdsSweep<T, KE, N> &lds_sweep()
{
    static_assert(sizeof(LdsSweep<T, KE, N>) <= sizeof(LdsSweep<T, KE, sizeof(T) == 8 ? 2 : 4>),
                  "the view fits the block");
    return *static_cast<LdsSweep<T, KE, N> *>(lds_sweep_block<T, KE>());
}

template <typename T, typename X, class C, int XM, int N>
__device__ void lds_sweep_cg(const Slot &S, const SlotState &st, int64_t lt, const C &cf,
                             double (&acc)[3])
{
    constexpr int TX = tile_x<N>(), W = sweep_w<N>(), G = TX / N, XL = sweep_left<N>();
    // halo lanes: three rows of groups, the left column (z'), two corners,
    // the right column, and for N = 1 the second left column (p only)
    constexpr int kHalo = 3 * G + 2 * kTileY + 3 + (N == 1 ? kTileY : 0);
    static_assert(kHalo <= kBlock, "the halo roles fit the workgroup");
    using K = typename C::Key;
    using KE = typename KeyElem<C>::type;
    using KP = KeyGroup<C, N>;
    using KR = typename KP::raw;
    using V = typename VecN<T, N>::type;
    using XV = typename VecN<X, N>::type;
    constexpr bool kXGroup = std::is_same<X, float>::value;   // d: ours, aligned
    LdsSweep<T, KE, N> &L = lds_sweep<T, KE, N>();
    const int l = (int)threadIdx.x;
    const TileCtx t = group_ctx(S, lt);
    const int ii = (N * l) % TX, jj = (N * l) / TX;
    const int ti0 = t.i - ii, tj0 = t.j - jj;
    const int nx = S.nx, ny = S.ny, nz = S.nz, bm = S.bcmask;
    const bool px = (S.permask & 1) && nx > 1, py = (S.permask & 2) && ny > 1;
    const int64_t P = t.P;
    const int pbuf = __builtin_amdgcn_readfirstlane(st.pbuf);
    const int zsel = __builtin_amdgcn_readfirstlane(st.zsel);
    const GLB V *__restrict__ zin = (const GLB V *)gp((const T *)(zsel ? S.z2 : S.z));
    GLB V *__restrict__ zout = (GLB V *)gp((T *)(zsel ? S.z : S.z2));
    const GLB V *__restrict__ qv = (const GLB V *)gp((const T *)dir_buf(S, pbuf));
    GLB V *__restrict__ pdv = (GLB V *)gp((T *)dir_buf(S, dir_next(pbuf)));
    const GLB V *__restrict__ pv0 = (const GLB V *)gp((const T *)dir_buf(S, dir_prev(pbuf)));
    GLB X *__restrict__ x = gp(std::is_same<X, double>::value ? (X *)S.x : (X *)S.d32);
    const T beta = (T)st.beta, alpha = (T)st.alpha;
    const T alpha_p0 = (T)st.alpha_p0, alpha_p1 = (T)st.alpha_p1;
    const int64_t qo = (int64_t)min(t.j, ny - 1) * nx + min(t.i, nx - N);
    const int own = (jj + 2) * W + ii + XL;
    // halo role of this lane: a group of the rows below (two) or above the
    // tile, of the column left of it (with z'; for N = 1 also the cell left
    // of that, p only), of the corners left of the rows below and above, or
    // of the column right of it; wrapped on periodic axes, clamped at walls,
    // where the cells that would use it substitute the wall.  role 2: p and
    // z', role 1: p only.
    int dx = 0, dy = 0, role = 0;
    if (l < G) { dx = N * l; dy = -1; role = 2; }
    else if (l < 2 * G) { dx = N * (l - G); dy = -2; role = 1; }
    else if (l < 3 * G) { dx = N * (l - 2 * G); dy = kTileY; role = 1; }
    else {
        const int m = l - 3 * G;
        if (m < kTileY) { dx = -N; dy = m; role = 2; }
        else if (m < kTileY + 2) { dx = -N; dy = m == kTileY ? -1 : kTileY; role = 1; }
        else if (m < 2 * kTileY + 3) { dx = TX; dy = m - kTileY - 3; role = 1; }
        else if (N == 1 && m < 3 * kTileY + 3) { dx = -2; dy = m - 2 * kTileY - 3; role = 1; }
    }
    int64_t qh = qo;
    int hslot = own, hi = t.i, hj = t.j;
    if (role) {
        int ix = ti0 + dx, jy = tj0 + dy;
        ix = px ? (ix + nx) % nx : max(0, min(nx - N, ix));
        jy = py ? (jy + ny) % ny : max(0, min(ny - 1, jy));
        qh = (int64_t)jy * nx + ix;
        hslot = (dy + 2) * W + dx + XL;
        hi = ix;
        hj = jy;
    }
    // lanes of the z' halo waves without a z' role evaluate at their own
    // group's place (in bounds; the result is dropped)
    const int hs = role == 2 ? hslot : own;
    const int lw = __builtin_amdgcn_readfirstlane(l);
    // the waves holding halo lanes load in every lane; those holding z'
    // halo lanes evaluate the halo groups in every lane
    const bool hwave = lw < kHalo;
    const bool swave = lw < G || (lw >= 3 * G && lw < 3 * G + kTileY);
    const int i0 = t.i, j = t.j;
    const bool hxm = i0 > 0 || px, hxp = i0 + N - 1 < nx - 1 || px;
    const bool hym = j > 0 || py, hyp = j < ny - 1 || py;
    const bool gxm = hi > 0 || px, gxp = hi + N - 1 < nx - 1 || px;
    const bool gym = hj > 0 || py, gyp = hj < ny - 1 || py;
    // Dirichlet high walls in delta: x+ of the group's last cell, y+ of all
    const bool hwx = !hxp && (bm & 2), hwy = !hyp && (bm & 8);
    const K wxm = (bm & 1) ? cf.dirichlet() : cf.neumann();
    const K wxp = (bm & 2) ? cf.dirichlet() : cf.neumann();
    const K wym = (bm & 4) ? cf.dirichlet() : cf.neumann();
    const K wyp = (bm & 8) ? cf.dirichlet() : cf.neumann();
    const K wzm = (bm & 16) ? cf.dirichlet() : cf.neumann();
    const K wzp = (bm & 32) ? cf.dirichlet() : cf.neumann();
    struct Raw {
        V z, q, hz, hq;
        KR k, hk;
    };
    // loads past the tile re-read a plane inside the tile and the grid
    const int klast = min(t.k1, nz - 1);
    auto load = [&](int kk) {
        kk = min(kk, klast);
        const int64_t base = (int64_t)kk * P;
        Raw R{};
        R.z = zin[(base + qo) / N];
        R.q = qv[(base + qo) / N];
        R.k = KP::load(cf, base + qo);
        if (hwave) {
            R.hz = zin[(base + qh) / N];
            R.hq = qv[(base + qh) / N];
            R.hk = KP::load(cf, base + qh);
        }
        return R;
    };
    // delta's terms of one plane's groups: faces toward x-, y- and z- and the
    // Dirichlet high walls; the x-/y- neighbours' z' from LDS, their keys as
    // the operator row read them
    auto delta = [&](const T *Lz, const T (&zc)[N], const T (&zd)[N], const T (&bd)[N],
                     const K (&kd)[N], K kxl, const K (&kyd)[N],
                     bool dtop) __attribute__((always_inline)) {
        const V zym = *(const V *)(Lz + own - W);
        T zl = hxm ? Lz[own - 1] : T(0);
        K kl = kxl;
        double d = 0.0;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const Areas6<T> ar = cf.areas(i0 + n, j, 0, 0);
            const T ex = zc[n] - zl, ey = zc[n] - (hym ? zym[n] : T(0)), ez = zc[n] - zd[n];
            T sn = (cf.beta(kd[n], kl) * ar.xm * ex * ex + cf.beta(kd[n], kyd[n]) * ar.ym * ey * ey) +
                   bd[n] * ez * ez;
            const T w = ((n == N - 1 && hwx) ? ar.xp : T(0)) + (hwy ? ar.yp : T(0)) +
                        (dtop ? ar.zp : T(0));
            sn += w * cf.beta(kd[n], cf.dirichlet()) * (zc[n] * zc[n]);
            d += (double)sn;
            zl = zc[n];
            kl = kd[n];
        }
        return d;
    };
    const int kb = t.k0 > 0 ? t.k0 - 1 : 0;
    // carried per group: p one plane down (vzm) and at this plane (vc), the
    // key (kc, and as loaded: kr), the low z face coefficient (bzm), z at
    // this plane (uc), the previous direction at this plane (qc, also the
    // catch-up form's direction one back); for the previous plane's delta
    // its z' (z1), z' one more plane down (z2), its low z face coefficient
    // (bd1), its keys and those of its x-/y- neighbours; the same for the
    // halo group (h*) without delta
    T vzm[N], vc[N], bzm[N], uc[N], qc[N], z1[N], z2[N], bd1[N];
    T hvzm[N], hvc[N], hbzm[N], huc[N];
    K kc[N], k1[N], ky1[N], hkc[N];
    K kx1 = wxm;
    KR kr, hkr;
    {
        K kzm[N], hkzm[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            vzm[n] = hvzm[n] = z1[n] = z2[n] = bd1[n] = T(0);
            kzm[n] = hkzm[n] = wzm;
            k1[n] = ky1[n] = wzm;
        }
        if (kb > 0) {
            const Raw R = load(kb - 1);
#pragma unroll
            for (int n = 0; n < N; ++n) {
                vzm[n] = R.z[n] + beta * R.q[n];
                hvzm[n] = R.hz[n] + beta * R.hq[n];
            }
            KP::split(R.k, kzm);
            KP::split(R.hk, hkzm);
        }
        const Raw A = load(kb);
#pragma unroll
        for (int n = 0; n < N; ++n) {
            vc[n] = A.z[n] + beta * A.q[n];
            hvc[n] = A.hz[n] + beta * A.hq[n];
            uc[n] = A.z[n];
            huc[n] = A.hz[n];
            qc[n] = A.q[n];
        }
        kr = A.k;
        hkr = A.hk;
        KP::split(kr, kc);
        KP::split(hkr, hkc);
#pragma unroll
        for (int n = 0; n < N; ++n) {
            bzm[n] = cf.beta(kc[n], kzm[n]) * cf.areas(i0 + n, j, kb, 0).zm;
            hbzm[n] = cf.beta(hkc[n], hkzm[n]) * cf.areas(hi + n, hj, kb, 0).zm;
        }
    }
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    int b = 0;
    for (int k = kb; k < t.k1; ++k, b ^= 1) {
        const bool emit = k >= t.k0;
        const bool top = k == nz - 1;
        const int64_t c = (int64_t)k * P;
        // stage plane k's p and keys
        {
            V pv_n, hv_n;
#pragma unroll
            for (int n = 0; n < N; ++n) {
                pv_n[n] = vc[n];
                hv_n[n] = hvc[n];
            }
            *(V *)(L.p[b] + own) = pv_n;
            KP::put(L.k[b] + own, kr);
            if (role) {
                *(V *)(L.p[b] + hslot) = hv_n;
                KP::put(L.k[b] + hslot, hkr);
            }
        }
        // plane k + 1 (z neighbours now, staged next), and this plane's
        // catch-up operands, in flight across the barrier
        const Raw Rn = load(k + 1);
        X xo[N];
        V v0;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            xo[n] = X(0);
            v0[n] = T(0);
        }
        if (XM == 3 && emit) {
            if constexpr (kXGroup) {
                const XV xv = __builtin_nontemporal_load(&((GLB XV *)x)[(c + qo) / N]);
#pragma unroll
                for (int n = 0; n < N; ++n) xo[n] = xv[n];
            } else {
#pragma unroll
                for (int n = 0; n < N; ++n) xo[n] = __builtin_nontemporal_load(&x[c + qo + n]);
            }
            v0 = __builtin_nontemporal_load(&pv0[(c + qo) / N]);
        }
        __syncthreads();
        // the previous plane's delta (its z' staged before this barrier)
        if (k - 1 >= t.k0) {
            const double d = delta(L.z[b ^ 1], z1, z2, bd1, k1, kx1, ky1, false);
            if (t.active) a2 += d;
        }
        const T *Lp = L.p[b];
        const KE *Lk = L.k[b];
        T *Lz = L.z[b];
        V pn, hpn;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            pn[n] = top ? T(0) : Rn.z[n] + beta * Rn.q[n];
            hpn[n] = top ? T(0) : Rn.hz[n] + beta * Rn.hq[n];
        }
        K kzp[N], hkzp[N];
        KP::split(Rn.k, kzp);
        KP::split(Rn.hk, hkzp);
#pragma unroll
        for (int n = 0; n < N; ++n) {
            kzp[n] = top ? wzp : kzp[n];
            hkzp[n] = top ? wzp : hkzp[n];
        }
        // this plane's groups: q, z', the x update and the dot terms
        const V vym = *(const V *)(Lp + own - W), vyp = *(const V *)(Lp + own + W);
        K kym[N], kyp[N];
        KP::split(KP::get(Lk + own - W), kym);
        KP::split(KP::get(Lk + own + W), kyp);
        const T lvxm = Lp[own - 1], lvxp = Lp[own + N];
        const K lkxm = (K)Lk[own - 1], lkxp = (K)Lk[own + N];
        T zn[N];
        X xn[N];
        double g0 = 0.0, g1 = 0.0;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            kym[n] = hym ? kym[n] : wym;
            bd1[n] = bzm[n];   // this plane's low z face, for its delta
            const Areas6<T> ar = cf.areas(i0 + n, j, k, c + qo + n);
            const T vxm = n > 0 ? vc[n - 1] : (hxm ? lvxm : T(0));
            const K kxm = n > 0 ? kc[n - 1] : (hxm ? lkxm : wxm);
            const T vxp = n < N - 1 ? vc[n + 1] : (hxp ? lvxp : T(0));
            const K kxp = n < N - 1 ? kc[n + 1] : (hxp ? lkxp : wxp);
            passB_cell<T, X, C, XM>(cf, ar, kc[n], vc[n], vxm, kxm, vxp, kxp,
                                    hym ? vym[n] : T(0), kym[n],
                                    hyp ? vyp[n] : T(0), hyp ? kyp[n] : wyp, vzm[n], pn[n],
                                    kzp[n], bzm[n], uc[n], alpha, alpha_p0, alpha_p1, xo[n],
                                    v0[n], qc[n], xn[n], zn[n], g0, g1);
        }
        {
            V zv_n;
#pragma unroll
            for (int n = 0; n < N; ++n) zv_n[n] = zn[n];
            *(V *)(Lz + own) = zv_n;
            if (emit && t.active) {
                a0 += g0;
                a1 += g1;
                V pv_n;
#pragma unroll
                for (int n = 0; n < N; ++n) pv_n[n] = vc[n];
                __builtin_nontemporal_store(pv_n, &pdv[(c + qo) / N]);
                __builtin_nontemporal_store(zv_n, &zout[(c + qo) / N]);
                if (XM == 3) {
                    if constexpr (kXGroup) {
                        XV xv;
#pragma unroll
                        for (int n = 0; n < N; ++n) xv[n] = xn[n];
                        __builtin_nontemporal_store(xv, &((GLB XV *)x)[(c + qo) / N]);
                    } else {
#pragma unroll
                        for (int n = 0; n < N; ++n)
                            __builtin_nontemporal_store(xn[n], &x[c + qo + n]);
                    }
                }
            }
        }
        // the halo groups that need z': the row below the tile, the column left of it
        if (swave) {
            const V hym_v = *(const V *)(Lp + hs - W), hyp_v = *(const V *)(Lp + hs + W);
            K hkym[N], hkyp[N];
            KP::split(KP::get(Lk + hs - W), hkym);
            KP::split(KP::get(Lk + hs + W), hkyp);
            const T hlvxm = Lp[hs - 1], hlvxp = Lp[hs + N];
            const K hlkxm = (K)Lk[hs - 1], hlkxp = (K)Lk[hs + N];
            T hz[N];
            X hx[N];
            double d0 = 0.0, d1 = 0.0;
#pragma unroll
            for (int n = 0; n < N; ++n) {
                const Areas6<T> ar = cf.areas(hi + n, hj, k, 0);
                const T vxm = n > 0 ? hvc[n - 1] : (gxm ? hlvxm : T(0));
                const K kxm = n > 0 ? hkc[n - 1] : (gxm ? hlkxm : wxm);
                const T vxp = n < N - 1 ? hvc[n + 1] : (gxp ? hlvxp : T(0));
                const K kxp = n < N - 1 ? hkc[n + 1] : (gxp ? hlkxp : wxp);
                passB_cell<T, X, C, 0>(cf, ar, hkc[n], hvc[n], vxm, kxm, vxp, kxp,
                                       gym ? hym_v[n] : T(0), gym ? hkym[n] : wym,
                                       gyp ? hyp_v[n] : T(0), gyp ? hkyp[n] : wyp, hvzm[n],
                                       hpn[n], hkzp[n], hbzm[n], huc[n], alpha, alpha_p0,
                                       alpha_p1, X(0), T(0), T(0), hx[n], hz[n], d0, d1);
            }
            if (role == 2) {
                V hv;
#pragma unroll
                for (int n = 0; n < N; ++n) hv[n] = hz[n];
                *(V *)(Lz + hslot) = hv;
            }
        }
        // carry up one plane
        kx1 = hxm ? lkxm : wxm;
#pragma unroll
        for (int n = 0; n < N; ++n) {
            z2[n] = z1[n];
            z1[n] = zn[n];
            k1[n] = kc[n];
            ky1[n] = kym[n];
            vzm[n] = vc[n];
            vc[n] = pn[n];
            kc[n] = kzp[n];
            uc[n] = Rn.z[n];
            qc[n] = Rn.q[n];
            hvzm[n] = hvc[n];
            hvc[n] = hpn[n];
            hkc[n] = hkzp[n];
            huc[n] = Rn.hz[n];
        }
        kr = Rn.k;
        hkr = Rn.hk;
    }
    // the last plane's delta
    __syncthreads();
    if (t.k1 - 1 >= t.k0) {
        const double d = delta(L.z[b ^ 1], z1, z2, bd1, k1, kx1, ky1,
                               t.k1 == nz && (bm & 32));
        if (t.active) a2 += d;
    }
    // (a0, a1, a2 hold only active lanes' terms; acc[2] first, so that the
    // stores ending this form and pass B address the same elements and their
    // merged tail stays out of scratch)
    acc[2] += a2;
    acc[0] += a0;
    acc[1] += a1;
}

// Pass A / pass B for the tile form of the slot (four cells per thread for
// FP32 only: FP64 kernels do not carry its registers).
template <typename T, class C>
__device__ __forceinline__ void passA(const Slot &S, const SlotState &st, int64_t lt,
                                      const C &cf, double (&acc)[3])
{
    if constexpr (std::is_same<T, float>::value) {
        if (S.cpt == 4) { group_passA<T, C, 4>(S, st, lt, cf, acc); return; }
    }
    if (S.cpt == 2) group_passA<T, C, 2>(S, st, lt, cf, acc);
    else body_passA<T>(S, st, lt, cf, acc);
}

template <typename T, typename X, class C, int XM>
__device__ __forceinline__ void passB(const Slot &S, const SlotState &st, int64_t lt,
                                      const C &cf, double (&acc)[3])
{
    if constexpr (std::is_same<T, float>::value) {
        if (S.cpt == 4) { group_passB<T, X, C, XM, 4>(S, st, lt, cf, acc); return; }
    }
    if (S.cpt == 2) group_passB<T, X, C, XM, 2>(S, st, lt, cf, acc);
    else body_passB<T, X, C, XM>(S, st, lt, cf, acc);
}

// K1_CHECK64: ||b - A x||^2 with the FP64 operator.
template <class C>
__device__ void body_check64(const Slot &S, const SlotState &st, int64_t lt,
                             const C &cf, double (&acc)[3])
{
    using K = typename C::Key;
    for_rows(S, lt, [&](const TileCtx &t) {
        if (!t.active) return;
        const GLB double *__restrict__ x = gp((const double *)S.x);
        const GLB double *__restrict__ rhs = gp(S.rhs);
        const Nbr<K> n = make_nbr(t, S, cf);
        auto xv = [&](int64_t m) -> double { return x[m]; };
        const int64_t P = t.P;
        int64_t c = (int64_t)t.k0 * P + t.q;
        double vc = x[c];
        K kc = cf.load(c);
        double vzm = 0.0;
        K kzm = n.wzm;
        if (t.k0 > 0) { vzm = x[c - P]; kzm = cf.load(c - P); }
        double a = 0.0;
        for (int k = t.k0; k < t.k1; ++k, c += P) {
            const bool top = k == S.nz - 1;
            double vzp = 0.0;
            K kzp = n.wzp;
            if (!top) { vzp = x[c + P]; kzp = cf.load(c + P); }
            double q, dg;
            apply_cell<double>(xv, cf, c, n, vc, kc, vzm, kzm, vzp, kzp,
                               cf.areas(t.i, t.j, k, c), q, dg);
            if (!cf.solid(kc)) {
                const double r = (-S.h2 * vol_at(S, c) * rhs[c] - st.bshift) - q;
                a += r * r;
            }
            vzm = vc; kzm = kc;
            vc = vzp; kc = kzp;
        }
        acc[0] += a;
    });
}

// K1_IR_INIT: x = 0 (cold) or hull entries cleared (warm), d = 0, the
// direction buffers zeroed; acc = [b.b].
template <class C>
__device__ void body_ir_init(const Slot &S, const SlotState &st, int64_t lt,
                             const C &cf, double (&acc)[3])
{
    for_rows(S, lt, [&](const TileCtx &t) {
        if (!t.active) return;
        GLB double *__restrict__ x = gp(S.x);
        GLB float *__restrict__ d = gp(S.d32);
        GLB float *__restrict__ pa = gp((float *)S.dir0);
        GLB float *__restrict__ pb = gp((float *)S.dir1);
        GLB float *__restrict__ pc = gp((float *)S.dir2);
        const GLB double *__restrict__ rhs = gp(S.rhs);
        int64_t c = (int64_t)t.k0 * t.P + t.q;
        const bool warm = st.warm != 0;
        double a = 0.0;
        for (int k = t.k0; k < t.k1; ++k, c += t.P) {
            const bool solid = cf.solid(cf.load(c));
            if (!warm || solid) x[c] = 0.0;
            d[c] = 0.0f;
            pa[c] = 0.0f;
            pb[c] = 0.0f;
            pc[c] = 0.0f;
            const double b = solid ? 0.0 : -S.h2 * vol_at(S, c) * rhs[c] - st.bshift;
            a += b * b;
        }
        acc[0] += a;
    });
}

// K1_IR_RESID: r = b - A64 (x + s d) in FP64, and the scaled inner right-hand
// side in z form, z32 = (scale r) / diag32, with diag32 the diagonal the
// FP32 passes use (cf32).  acc = [r.r, r32.z32, r32.r32].
template <class C64, class C32>
__device__ void body_ir_resid(const Slot &S, const SlotState &st, int64_t lt,
                              const C64 &cf, const C32 &cf32, double (&acc)[3])
{
    using K = typename C64::Key;
    using KF = typename C32::Key;
    for_rows(S, lt, [&](const TileCtx &t) {
        if (!t.active) return;
        const GLB double *__restrict__ x = gp((const double *)S.x);
        const GLB float *__restrict__ d = gp((const float *)S.d32);
        GLB float *__restrict__ z = gp((float *)S.z);
        const GLB double *__restrict__ rhs = gp(S.rhs);
        const double s = st.upd_s;
        const double scale = st.scale;
        const Nbr<K> n = make_nbr(t, S, cf);
        const Nbr<KF> nf = make_nbr(t, S, cf32);
        auto xe = [&](int64_t m) -> double { return refined(x[m], s, d[m]); };
        const int64_t P = t.P;
        int64_t c = (int64_t)t.k0 * P + t.q;
        double vc = xe(c);
        K kc = cf.load(c);
        KF fc = cf32.load(c);
        double vzm = 0.0;
        K kzm = n.wzm;
        KF fzm = nf.wzm;
        if (t.k0 > 0) { vzm = xe(c - P); kzm = cf.load(c - P); fzm = cf32.load(c - P); }
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int k = t.k0; k < t.k1; ++k, c += P) {
            const bool top = k == S.nz - 1;
            double vzp = 0.0;
            K kzp = n.wzp;
            KF fzp = nf.wzp;
            if (!top) { vzp = xe(c + P); kzp = cf.load(c + P); fzp = cf32.load(c + P); }
            double q, dg;
            apply_cell<double>(xe, cf, c, n, vc, kc, vzm, kzm, vzp, kzp,
                               cf.areas(t.i, t.j, k, c), q, dg);
            const bool solid = cf.solid(kc);
            const double r = solid ? 0.0 : ((-S.h2 * vol_at(S, c) * rhs[c] - st.bshift) - q);
            const float dg32 = diag_cell<float>(cf32, c, nf, fc, fzm, fzp,
                                                cf32.areas(t.i, t.j, k, c));
            const float z32 = dg32 > 0.0f ? (float)((scale * r) / (double)dg32) : 0.0f;
            z[c] = z32;
            const double rz = (double)dg32 * (double)z32;
            a0 += r * r;
            a1 += rz * (double)z32;
            a2 += rz * rz;
            vzm = vc; kzm = kc; fzm = fc;
            vc = vzp; kc = kzp; fc = fzp;
        }
        acc[0] += a0;
        acc[1] += a1;
        acc[2] += a2;
    });
}

// K1_FLUSH_X: the updates the last one or two iterations left pending, in
// order: x += alpha_p0 p_p0 (+= alpha_p1 p_p1) (FP64), or the same on the
// inner solve's correction d (FP32+IR).  The latest pending direction is the
// current buffer, the one before it the previous buffer.
__device__ void body_flush_x(const Slot &S, const SlotState &st, int64_t lt, double (&acc)[3])
{
    const int two = st.xpend == 2;
    const int b0 = two ? dir_prev(st.pbuf) : st.pbuf;
    for_rows(S, lt, [&](const TileCtx &t) {
        if (!t.active) return;
        int64_t c = (int64_t)t.k0 * t.P + t.q;
        if (S.d32) {
            GLB float *__restrict__ d = gp(S.d32);
            const GLB float *__restrict__ p0 = gp((const float *)dir_buf(S, b0));
            const GLB float *__restrict__ p1 = gp((const float *)dir_buf(S, st.pbuf));
            const float a0 = (float)st.alpha_p0, a1 = (float)st.alpha_p1;
            for (int k = t.k0; k < t.k1; ++k, c += t.P) {
                const float v = fmaf(a0, p0[c], d[c]);
                d[c] = two ? fmaf(a1, p1[c], v) : v;
            }
            return;
        }
        GLB double *__restrict__ x = gp(S.x);
        const GLB double *__restrict__ p0 = gp((const double *)dir_buf(S, b0));
        const GLB double *__restrict__ p1 = gp((const double *)dir_buf(S, st.pbuf));
        const double a0 = st.alpha_p0, a1 = st.alpha_p1;
        for (int k = t.k0; k < t.k1; ++k, c += t.P) {
            const double v = fma(a0, p0[c], x[c]);
            x[c] = two ? fma(a1, p1[c], v) : v;
        }
    });
}

// K2_IR_UPDATE: x += s d, d = 0.
__device__ void body_ir_update(const Slot &S, const SlotState &st, int64_t lt,
                               double (&acc)[3])
{
    for_rows(S, lt, [&](const TileCtx &t) {
        if (!t.active) return;
        GLB double *__restrict__ x = gp(S.x);
        GLB float *__restrict__ d = gp(S.d32);
        const double s = st.upd_s;
        int64_t c = (int64_t)t.k0 * t.P + t.q;
        for (int k = t.k0; k < t.k1; ++k, c += t.P) {
            x[c] = refined(x[c], s, d[c]);
            d[c] = 0.0f;
        }
    });
}

// K2_ZERO_X: x = 0 (zero source with a warm start).
__device__ void body_zero_x(const Slot &S, const SlotState &st, int64_t lt,
                            double (&acc)[3])
{
    for_rows(S, lt, [&](const TileCtx &t) {
        if (!t.active) return;
        GLB double *__restrict__ x = gp(S.x);
        int64_t c = (int64_t)t.k0 * t.P + t.q;
        for (int k = t.k0; k < t.k1; ++k, c += t.P) x[c] = 0.0;
    });
}

// Singular problems (no Dirichlet wall: the constant over the fluid is the
// null vector).  K1_MEAN_B: acc = [sum of b, count] over fluid cells, so
// the source can be made mean-free; K1_MEAN_X: acc = [sum of x] over fluid
// cells; K2_SUB_X: x -= that mean, leaving the zero-mean solution.
template <class C>
__device__ void body_mean_b(const Slot &S, const SlotState &st, int64_t lt,
                            const C &cf, double (&acc)[3])
{
    for_rows(S, lt, [&](const TileCtx &t) {
        if (!t.active) return;
        const GLB double *__restrict__ rhs = gp(S.rhs);
        double a = 0.0, m = 0.0;
        int64_t c = (int64_t)t.k0 * t.P + t.q;
        for (int k = t.k0; k < t.k1; ++k, c += t.P) {
            if (cf.solid(cf.load(c))) continue;
            a += -S.h2 * vol_at(S, c) * rhs[c];
            m += 1.0;
        }
        acc[0] += a;
        acc[1] += m;
    });
}

template <class C>
__device__ void body_mean_x(const Slot &S, const SlotState &st, int64_t lt,
                            const C &cf, double (&acc)[3])
{
    for_rows(S, lt, [&](const TileCtx &t) {
        if (!t.active) return;
        const GLB double *__restrict__ x = gp((const double *)S.x);
        double a = 0.0;
        int64_t c = (int64_t)t.k0 * t.P + t.q;
        for (int k = t.k0; k < t.k1; ++k, c += t.P)
            if (!cf.solid(cf.load(c))) a += x[c];
        acc[0] += a;
    });
}

template <class C>
__device__ void body_sub_x(const Slot &S, const SlotState &st, int64_t lt,
                           const C &cf, double (&acc)[3])
{
    for_rows(S, lt, [&](const TileCtx &t) {
        if (!t.active) return;
        GLB double *__restrict__ x = gp(S.x);
        const double m = st.xshift;
        int64_t c = (int64_t)t.k0 * t.P + t.q;
        for (int k = t.k0; k < t.k1; ++k, c += t.P)
            if (!cf.solid(cf.load(c))) x[c] -= m;
    });
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

// After pass B: it caught x up (two updates were pending: none now) or left
// this iteration's update pending beside the ones before it.
__device__ __forceinline__ void note_x_update(SlotState &st)
{
    if (st.xpend == 2) { st.xpend = 0; return; }
    if (st.xpend == 0) st.alpha_p0 = st.alpha;
    else st.alpha_p1 = st.alpha;
    st.xpend += 1;
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
        if (!(pap > 0.0) || !isfinite(pap)) {
            // x keeps the last iterate: apply the pending updates first
            if (st.xpend) { st.status = PCG_EBREAKDOWN; st.phase = K1_FLUSH_X; }
            else finish(st, PCG_EBREAKDOWN);
            break;
        }
        st.pap = pap;
        st.alpha = st.rz / pap;
        st.pbuf = dir_next(st.pbuf);
        st.first = 0;
        // one-sweep iterations: this pass A gave the first p.A p; the first
        // sweep forms the same direction again (beta = 0)
        if (st.fused) { st.beta = 0.0; st.phase = K2_CG_F; }
        else st.phase = K2_CG_B;
        break;
    }
    case K2_CG_F: {
        // tot = [r.z, r.r, z.A z] of the new residual
        st.iter += 1;
        st.rr = tot[1];
        note_x_update(st);   // with the alpha this sweep used
        st.pbuf = dir_next(st.pbuf);
        st.zsel ^= 1;
        if (!isfinite(tot[0]) || !isfinite(tot[1]) || !isfinite(tot[2])) {
            finish(st, PCG_EBREAKDOWN);
            break;
        }
        const double beta = tot[0] / st.rz;
        const double pap = tot[2] - beta * tot[0] / st.alpha;
        st.beta = beta;
        st.rz = tot[0];
        st.pap = pap;
        const bool ok = pap > 0.0 && isfinite(pap);
        if (ok) st.alpha = tot[0] / pap;
        if (st.rr <= st.tol2 || st.iter >= st.maxit) {
            st.phase = st.xpend ? K1_FLUSH_X : K1_CHECK64;
            st.after = K1_CHECK64;
        } else if (!ok) {
            if (st.xpend) { st.status = PCG_EBREAKDOWN; st.phase = K1_FLUSH_X; }
            else finish(st, PCG_EBREAKDOWN);
        } else {
            st.phase = K2_CG_F;   // the next K1 launch passes this slot by
        }
        break;
    }
    case K2_CG_B: {
        st.iter += 1;
        st.rr = tot[1];
        st.beta = tot[0] / st.rz;
        st.rz = tot[0];
        note_x_update(st);
        if (!isfinite(st.rr) || !isfinite(st.rz)) { finish(st, PCG_EBREAKDOWN); break; }
        if (st.rr <= st.tol2 || st.iter >= st.maxit) {
            st.phase = st.xpend ? K1_FLUSH_X : K1_CHECK64;
            st.after = K1_CHECK64;   // after the flush
        } else {
            st.phase = K1_CG_A;
        }
        break;
    }
    case K1_FLUSH_X: {
        // then the action its scheduler left in `after`; nothing after an error
        st.xpend = 0;
        st.phase = K2_NONE;
        if (st.status != PCG_PENDING) st.after = PH_DONE;
        break;
    }
    case K1_CHECK64: {
        st.rr_true = tot[0];
        const int end = st.singular ? K1_MEAN_X : PH_DONE;
        if (tot[0] <= st.tol2) { st.phase = K2_NONE; st.after = end; st.status = PCG_OK; }
        else if (st.iter >= st.maxit) { st.phase = K2_NONE; st.after = end; st.status = PCG_MAXIT; }
        else if (st.fused && st.iter > 0) {
            // the last sweep left alpha and beta for the next one
            if (st.pap > 0.0 && isfinite(st.pap)) st.phase = K2_CG_F;
            else finish(st, PCG_EBREAKDOWN);
        } else { st.phase = K2_NONE; st.after = K1_CG_A; }
        break;
    }
    case K1_MEAN_B: {
        st.nfluid = tot[1];
        st.bshift = tot[1] > 0.0 ? tot[0] / tot[1] : 0.0;
        if (!isfinite(st.bshift)) { finish(st, PCG_EDOMAIN); break; }
        st.phase = K2_NONE;   // then the initialisation held in `after`
        break;
    }
    case K1_MEAN_X: {
        st.xshift = st.nfluid > 0.0 ? tot[0] / st.nfluid : 0.0;
        st.phase = K2_SUB_X;
        break;
    }
    case K2_SUB_X:
        st.phase = PH_DONE;
        if (st.status == PCG_PENDING) st.status = PCG_OK;
        break;
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
        st.zsel = 0;   // the residual phase wrote z into its first buffer
        if (!isfinite(rr)) { finish(st, PCG_EBREAKDOWN); break; }
        st.phase = K2_IR_UPDATE;
        if (rr <= st.tol2) { st.final_upd = 1; st.status = PCG_OK; }
        else if (st.iter >= st.maxit || st.outer > kMaxOuter) { st.final_upd = 1; st.status = PCG_MAXIT; }
        else {
            st.final_upd = 0;
            st.rz = tot[1];
            st.rr0_inner = tot[2];
            st.rr = tot[2];
            // ask the inner solve for its usual reduction, but never for more
            // than this trip needs to bring the outer residual to half of tol
            const double need2 = 0.25 * st.tol2 / rr;
            st.inner_goal2 = need2 > st.inner_tol2 ? need2 : st.inner_tol2;
        }
        break;
    }
    case K2_IR_UPDATE: {
        if (st.final_upd) { st.phase = st.singular ? K1_MEAN_X : PH_DONE; break; }
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
            st.phase = st.xpend ? K1_FLUSH_X : K2_NONE;   // d complete first
            st.after = K1_IR_RESID;
            break;
        }
        st.pap = pap;
        st.alpha = st.rz / pap;
        st.pbuf = dir_next(st.pbuf);
        st.first = 0;
        if (st.fused) { st.beta = 0.0; st.phase = K2_IR_F; }
        else st.phase = K2_IR_B;
        break;
    }
    case K2_IR_F: {
        // tot = [r.z, r.r, z.A z] of the new inner residual
        st.iter += 1;
        st.inner_iter += 1;
        st.rr = tot[1];
        note_x_update(st);   // d, as x in FP64
        st.pbuf = dir_next(st.pbuf);
        st.zsel ^= 1;
        if (!isfinite(tot[1])) { finish(st, PCG_EBREAKDOWN); break; }
        const double beta = tot[0] / st.rz;
        const double pap = tot[2] - beta * tot[0] / st.alpha;
        st.beta = beta;
        st.rz = tot[0];
        st.pap = pap;
        const bool ok = pap > 0.0 && isfinite(pap);
        if (ok) st.alpha = tot[0] / pap;
        const bool inner_done = st.rr <= st.inner_goal2 * st.rr0_inner ||
                                st.inner_iter >= st.inner_maxit ||
                                st.iter >= st.maxit;
        if (inner_done || !ok) {
            // refine (a vanished direction too, as after pass A); d complete first
            st.scale = pow2_scale(sqrt(st.rr_true * st.inner_tol2));
            st.phase = st.xpend ? K1_FLUSH_X : K1_IR_RESID;
            st.after = K1_IR_RESID;
        } else {
            st.phase = K2_IR_F;
        }
        break;
    }
    case K2_IR_B: {
        st.iter += 1;
        st.inner_iter += 1;
        st.rr = tot[1];
        st.beta = tot[0] / st.rz;
        st.rz = tot[0];
        note_x_update(st);   // d, as x in FP64
        if (!isfinite(st.rr)) { finish(st, PCG_EBREAKDOWN); break; }
        const bool inner_done = st.rr <= st.inner_goal2 * st.rr0_inner ||
                                st.inner_iter >= st.inner_maxit ||
                                st.iter >= st.maxit;
        if (inner_done) {
            // the outer residual reads x + s d: d complete first
            st.scale = pow2_scale(sqrt(st.rr_true * st.inner_tol2));
            st.phase = st.xpend ? K1_FLUSH_X : K1_IR_RESID;
            st.after = K1_IR_RESID;
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

// An iteration is two launches per coefficient mode in use: the first-half
// actions, then K2 (operator apply and vector update).  The first-half
// actions are pass A (K1, per mode) and the rare ones (set-up, FP64
// residuals, flushes: the "K0" actions, any mode); kernel position 3 serves
// both for one mode and the K0 actions of every slot, position 1 pass A
// alone for the other modes in use.  A slot is in exactly one first-half
// phase, so it is worked on by exactly one launch.  Position 0 (the K0
// actions alone) is kept for the body dispatch but not launched: a kernel
// boundary of its own cost more than the fused kernel's larger register
// footprint (at most 232 VGPRs, two waves per SIMD, what the grids of two
// workgroups per CU use).  K1 and K2 come in three coefficient modes
// (density, classes, cut cells), each serving only the slots of its mode.
// Coefficient mode of a slot: 0 per-cell density, 1 density classes,
// 2 per-cell density with free-slip cut cells (area/volume fractions);
// 3 classes and 4 per-cell density on 2-D plane tiles (LDS-staged pass B).
__device__ __forceinline__ int slot_mode(const Slot &S)
{
    if (S.ax) return 2;
    if (S.tx > 0) return S.cls ? 3 : 4;
    return S.cls ? 1 : 0;
}

// The first-half actions of K0 in one coefficient source.
template <class C>
__device__ __forceinline__ void run_k0_fp64(int ph, const Slot &S, const SlotState &st,
                                            int64_t lt, const C &cf, double (&acc)[3])
{
    if (ph == K1_INIT64) body_init64(S, st, lt, cf, acc);
    else if (ph == K1_CHECK64) body_check64(S, st, lt, cf, acc);
}

template <class C64, class C32>
__device__ __forceinline__ void run_k0_ir(int ph, const Slot &S, const SlotState &st,
                                          int64_t lt, const C64 &cf, const C32 &cf32,
                                          double (&acc)[3])
{
    if (ph == K1_IR_INIT) body_ir_init(S, st, lt, cf, acc);
    else if (ph == K1_IR_RESID) body_ir_resid(S, st, lt, cf, cf32, acc);
}

// First-half actions outside pass A (set-up, FP64 residuals, flushes).
__device__ __forceinline__ bool k0_phase(int ph)
{
    return ph == K1_INIT64 || ph == K1_CHECK64 || ph == K1_IR_INIT ||
           ph == K1_IR_RESID || ph == K1_MEAN_B || ph == K1_MEAN_X || ph == K1_FLUSH_X;
}

template <int FAMILY, int WHICH, int MODE>
__device__ __forceinline__ void run_body(int ph, const Slot &S,
                                         const SlotState &st, int64_t lt,
                                         const double *tab64, const float *tab32,
                                         double (&acc)[3])
{
    if (WHICH == 3) {   // K0 and K1 of MODE in one launch
        if (k0_phase(ph)) run_body<FAMILY, 0, 0>(ph, S, st, lt, tab64, tab32, acc);
        else run_body<FAMILY, 1, MODE>(ph, S, st, lt, tab64, tab32, acc);
        return;
    }
    if constexpr (WHICH == 2 && MODE >= 3) {
        // second-half launches alone: the first-half actions too
        if (k0_phase(ph)) { run_body<FAMILY, 0, 0>(ph, S, st, lt, tab64, tab32, acc); return; }
        if (ph == K1_CG_A || ph == K1_IR_A) {
            run_body<FAMILY, 1, MODE>(ph, S, st, lt, tab64, tab32, acc);
            return;
        }
    }
    const RhoCoef<double> r64{ gp(S.rho64) };
    const ClsCoef<double> c64{ gp(S.cls), tab64 };
    if (WHICH == 0) {
        // rare actions: every slot, whatever its coefficient source
        if (ph == K1_MEAN_B) { body_mean_b(S, st, lt, r64, acc); return; }
        if (ph == K1_MEAN_X) { body_mean_x(S, st, lt, r64, acc); return; }
        if (ph == K1_FLUSH_X) { body_flush_x(S, st, lt, acc); return; }
        if (FAMILY == PCG_PREC_FP64) {
            if (S.ax) run_k0_fp64(ph, S, st, lt, frac_coef<double>(S, S.rho64), acc);
            else if (S.cls) run_k0_fp64(ph, S, st, lt, c64, acc);
            else run_k0_fp64(ph, S, st, lt, r64, acc);
        } else {
            if (S.ax)
                run_k0_ir(ph, S, st, lt, frac_coef<double>(S, S.rho64),
                          frac_coef<float>(S, S.rho32), acc);
            else if (S.cls) run_k0_ir(ph, S, st, lt, c64, ClsCoef<float>{ gp(S.cls), tab32 }, acc);
            else run_k0_ir(ph, S, st, lt, r64, RhoCoef<float>{ gp(S.rho32) }, acc);
        }
        return;
    }
    if (MODE >= 3) {
        // 2-D plane tiles: both passes LDS-staged (two FP64 or four FP32 cells a thread)
        if (FAMILY == PCG_PREC_FP64) {
            if (WHICH == 1) {
                // one-cell-a-thread tiles run pass A once, for the first p.A p
                // of their one-sweep iteration: cell by cell, unstaged
                if (ph == K1_CG_A) {
                    if (__builtin_amdgcn_readfirstlane(S.cpt) == 1) {
                        if (MODE == 3) body_passA<double>(S, st, lt, c64, acc);
                        else body_passA<double>(S, st, lt, r64, acc);
                    } else if (MODE == 3) lds_passA<double, ClsCoef<double>, 2>(S, st, lt, c64, acc);
                    else lds_passA<double, RhoCoef<double>, 2>(S, st, lt, r64, acc);
                }
            } else if (ph == K2_CG_B) {
                const bool catch_up = __builtin_amdgcn_readfirstlane(st.xpend) == 2;
                if (MODE == 3) {
                    if (catch_up) lds_passB<double, double, ClsCoef<double>, 3, 2>(S, st, lt, c64, acc);
                    else lds_passB<double, double, ClsCoef<double>, 0, 2>(S, st, lt, c64, acc);
                } else {
                    if (catch_up) lds_passB<double, double, RhoCoef<double>, 3, 2>(S, st, lt, r64, acc);
                    else lds_passB<double, double, RhoCoef<double>, 0, 2>(S, st, lt, r64, acc);
                }
            } else if (ph == K2_CG_F) {
                const bool catch_up = __builtin_amdgcn_readfirstlane(st.xpend) == 2;
                const bool one = __builtin_amdgcn_readfirstlane(S.cpt) == 1;   // 64 x 4 tiles
                if (MODE == 3) {
                    if (one) {
                        if (catch_up) lds_sweep_cg<double, double, ClsCoef<double>, 3, 1>(S, st, lt, c64, acc);
                        else lds_sweep_cg<double, double, ClsCoef<double>, 0, 1>(S, st, lt, c64, acc);
                    } else if (catch_up) lds_sweep_cg<double, double, ClsCoef<double>, 3, 2>(S, st, lt, c64, acc);
                    else lds_sweep_cg<double, double, ClsCoef<double>, 0, 2>(S, st, lt, c64, acc);
                } else {
                    if (one) {
                        if (catch_up) lds_sweep_cg<double, double, RhoCoef<double>, 3, 1>(S, st, lt, r64, acc);
                        else lds_sweep_cg<double, double, RhoCoef<double>, 0, 1>(S, st, lt, r64, acc);
                    } else if (catch_up) lds_sweep_cg<double, double, RhoCoef<double>, 3, 2>(S, st, lt, r64, acc);
                    else lds_sweep_cg<double, double, RhoCoef<double>, 0, 2>(S, st, lt, r64, acc);
                }
            } else if (ph == K2_ZERO_X) body_zero_x(S, st, lt, acc);
            else if (ph == K2_SUB_X) body_sub_x(S, st, lt, r64, acc);
        } else {
            const RhoCoef<float> r32{ gp(S.rho32) };
            const ClsCoef<float> c32{ gp(S.cls), tab32 };
            if (WHICH == 1) {
                if (ph == K1_IR_A) {
                    if (__builtin_amdgcn_readfirstlane(S.cpt) == 1) {
                        if (MODE == 3) body_passA<float>(S, st, lt, c32, acc);
                        else body_passA<float>(S, st, lt, r32, acc);
                    } else if (MODE == 3) lds_passA<float, ClsCoef<float>, 4>(S, st, lt, c32, acc);
                    else lds_passA<float, RhoCoef<float>, 4>(S, st, lt, r32, acc);
                }
            } else if (ph == K2_IR_B) {
                const bool catch_up = __builtin_amdgcn_readfirstlane(st.xpend) == 2;
                if (MODE == 3) {
                    if (catch_up) lds_passB<float, float, ClsCoef<float>, 3, 4>(S, st, lt, c32, acc);
                    else lds_passB<float, float, ClsCoef<float>, 0, 4>(S, st, lt, c32, acc);
                } else {
                    if (catch_up) lds_passB<float, float, RhoCoef<float>, 3, 4>(S, st, lt, r32, acc);
                    else lds_passB<float, float, RhoCoef<float>, 0, 4>(S, st, lt, r32, acc);
                }
            } else if (ph == K2_IR_F) {
                const bool catch_up = __builtin_amdgcn_readfirstlane(st.xpend) == 2;
                const bool one = __builtin_amdgcn_readfirstlane(S.cpt) == 1;   // 64 x 4 tiles
                if (MODE == 3) {
                    if (one) {
                        if (catch_up) lds_sweep_cg<float, float, ClsCoef<float>, 3, 1>(S, st, lt, c32, acc);
                        else lds_sweep_cg<float, float, ClsCoef<float>, 0, 1>(S, st, lt, c32, acc);
                    } else if (catch_up) lds_sweep_cg<float, float, ClsCoef<float>, 3, 4>(S, st, lt, c32, acc);
                    else lds_sweep_cg<float, float, ClsCoef<float>, 0, 4>(S, st, lt, c32, acc);
                } else {
                    if (one) {
                        if (catch_up) lds_sweep_cg<float, float, RhoCoef<float>, 3, 1>(S, st, lt, r32, acc);
                        else lds_sweep_cg<float, float, RhoCoef<float>, 0, 1>(S, st, lt, r32, acc);
                    } else if (catch_up) lds_sweep_cg<float, float, RhoCoef<float>, 3, 4>(S, st, lt, r32, acc);
                    else lds_sweep_cg<float, float, RhoCoef<float>, 0, 4>(S, st, lt, r32, acc);
                }
            } else if (ph == K2_IR_UPDATE) body_ir_update(S, st, lt, acc);
            else if (ph == K2_ZERO_X) body_zero_x(S, st, lt, acc);
            else if (ph == K2_SUB_X) body_sub_x(S, st, lt, r64, acc);
        }
        return;
    }
    if (FAMILY == PCG_PREC_FP64) {
        if (WHICH == 1) {
            if (ph == K1_CG_A) {
                if (MODE == 2) passA<double>(S, st, lt, frac_coef<double>(S, S.rho64), acc);
                else if (MODE == 1) passA<double>(S, st, lt, c64, acc);
                else passA<double>(S, st, lt, r64, acc);
            }
        } else {
            if (ph == K2_CG_B) {
                // x is read and written every third iteration (XM 0, 0, 3)
                const bool catch_up = __builtin_amdgcn_readfirstlane(st.xpend) == 2;
                if (MODE == 2) {
                    const FracCoef<double> f = frac_coef<double>(S, S.rho64);
                    if (catch_up) passB<double, double, FracCoef<double>, 3>(S, st, lt, f, acc);
                    else passB<double, double, FracCoef<double>, 0>(S, st, lt, f, acc);
                } else if (MODE == 1) {
                    if (catch_up) passB<double, double, ClsCoef<double>, 3>(S, st, lt, c64, acc);
                    else passB<double, double, ClsCoef<double>, 0>(S, st, lt, c64, acc);
                } else {
                    if (catch_up) passB<double, double, RhoCoef<double>, 3>(S, st, lt, r64, acc);
                    else passB<double, double, RhoCoef<double>, 0>(S, st, lt, r64, acc);
                }
            } else if (ph == K2_ZERO_X) body_zero_x(S, st, lt, acc);
            else if (ph == K2_SUB_X) body_sub_x(S, st, lt, r64, acc);
        }
    } else {
        const RhoCoef<float> r32{ gp(S.rho32) };
        const ClsCoef<float> c32{ gp(S.cls), tab32 };
        if (WHICH == 1) {
            if (ph == K1_IR_A) {
                if (MODE == 2) passA<float>(S, st, lt, frac_coef<float>(S, S.rho32), acc);
                else if (MODE == 1) passA<float>(S, st, lt, c32, acc);
                else passA<float>(S, st, lt, r32, acc);
            }
        } else {
            if (ph == K2_IR_B) {
                // d is read and written every third iteration, as x in FP64
                const bool catch_up = __builtin_amdgcn_readfirstlane(st.xpend) == 2;
                if (MODE == 2) {
                    const FracCoef<float> f = frac_coef<float>(S, S.rho32);
                    if (catch_up) passB<float, float, FracCoef<float>, 3>(S, st, lt, f, acc);
                    else passB<float, float, FracCoef<float>, 0>(S, st, lt, f, acc);
                } else if (MODE == 1) {
                    if (catch_up) passB<float, float, ClsCoef<float>, 3>(S, st, lt, c32, acc);
                    else passB<float, float, ClsCoef<float>, 0>(S, st, lt, c32, acc);
                } else {
                    if (catch_up) passB<float, float, RhoCoef<float>, 3>(S, st, lt, r32, acc);
                    else passB<float, float, RhoCoef<float>, 0>(S, st, lt, r32, acc);
                }
            } else if (ph == K2_IR_UPDATE) body_ir_update(S, st, lt, acc);
            else if (ph == K2_ZERO_X) body_zero_x(S, st, lt, acc);
            else if (ph == K2_SUB_X) body_sub_x(S, st, lt, r64, acc);
        }
    }
}

template <int WHICH, int MODE>
__device__ __forceinline__ bool serves(const Slot &S, int ph, bool k2only)
{
    if (WHICH == 0) return k0_phase(ph);
    if (WHICH == 3 && k0_phase(ph)) return true;
    if (slot_mode(S) != MODE) return false;
    if (WHICH == 1 || WHICH == 3) return ph == K1_CG_A || ph == K1_IR_A;
    // second-half launches alone (one-sweep solves on plane tiles): also
    // the first-half actions of this mode's slots
    if (MODE >= 3 && k2only && (k0_phase(ph) || ph == K1_CG_A || ph == K1_IR_A)) return true;
    return ph >= 11 && ph <= 19;
}

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
        const GLB double *__restrict__ part = gp((const double *)S.partials);
#pragma unroll 8
        for (int64_t t = threadIdx.x; t < S.ntiles; t += kBlock) {
            tot[0] += part[kMaxPartials * t + 0];
            tot[1] += part[kMaxPartials * t + 1];
            tot[2] += part[kMaxPartials * t + 2];
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

// WHICH = 0, 1, 2: launch position within the iteration; MODE: coefficient
// source of the slots served by K1/K2 (0 density, 1 classes).
template <int FAMILY, int WHICH, int MODE>
__global__ void __launch_bounds__(kBlock)
k_iter(const BatchHeader *__restrict__ hdr, const Slot *__restrict__ slots)
{
    __shared__ double lds[kMaxPartials * 4];
    __shared__ double s_tab64[kClasses * kClasses];
    __shared__ float s_tab32[kClasses * kClasses];
    __shared__ int s_last;
    const int64_t T = hdr->total_tiles;
    const int ns = hdr->nslots;
    const bool k2only = hdr->k2only != 0;
    const int G = (int)gridDim.x;
    const int g = xcd_major((int)blockIdx.x, G);
    // strided: tiles g, g + G, ...; chunked: tiles [g T / G, (g + 1) T / G)
    const bool chunked = hdr->chunked != 0;
    const int64_t t_first = chunked ? (T * g) / G : g;
    const int64_t t_end = chunked ? (T * (g + 1)) / G : T;
    const int64_t t_step = chunked ? 1 : G;
    int cur = -1, cur_ph = 0;
    int64_t cur_end = 0;
    bool cur_served = false;
    uint32_t run = 0;
    for (int64_t t = t_first; t < t_end; t += t_step) {
        // tiles only increase: search again only when t leaves the slot
        const int s = (cur >= 0 && t < cur_end) ? cur : find_slot(slots, ns, t);
        const Slot &S = slots[s];
        if (s != cur) {
            if (run) arrive(slots[cur], cur_ph, run, lds, &s_last);
            cur = s;
            cur_end = S.tile_begin + S.ntiles;
            run = 0;
            cur_ph = S.st->phase;
            cur_served = serves<WHICH, MODE>(S, cur_ph, k2only);
            if (cur_served && S.cls) {   // class table of this slot into LDS
                const bool need64 = FAMILY == PCG_PREC_FP64 || WHICH == 0 ||
                                    ((WHICH == 3 || WHICH == 2) && k0_phase(cur_ph));
                const bool need32 = FAMILY == PCG_PREC_FP32_IR;
                for (int i = threadIdx.x; i < kClasses * kClasses; i += kBlock) {
                    if (need64) s_tab64[i] = gp(S.tab64)[i];
                    if (need32) s_tab32[i] = gp(S.tab32)[i];
                }
                __syncthreads();
            }
        }
        if (!cur_served) continue;
        const int ph = cur_ph;
        double acc[3] = { 0.0, 0.0, 0.0 };
        run_body<FAMILY, WHICH, MODE>(ph, S, *S.st, t - S.tile_begin, s_tab64, s_tab32, acc);
        block_sum<3>(acc, lds);
        if (threadIdx.x == 0) {
            GLB double *dst = gp(S.partials) + kMaxPartials * (t - S.tile_begin);
            dst[0] = acc[0];
            dst[1] = acc[1];
            dst[2] = acc[2];
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

// The hull mask one bit per cell for the host's connectivity check: row r
// takes words_per_row 32-bit words from bits[r * words_per_row], bit j of
// word w the cell x = 32 w + j (1 = hull); the bits past the row's end are
// set, so every row ends in a hull bit.  An eighth of the mask's bytes
// cross to the host, and the host finds fluid runs a word at a time.
__global__ void __launch_bounds__(256)
k_pack_mask(const uint8_t *__restrict__ mask, uint32_t *__restrict__ bits, int nx,
            int words_per_row, int64_t nwords)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nwords;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / words_per_row;
        const int x0 = (int)(t - r * words_per_row) * 32;   // < nx
        const int cnt = nx - x0 < 32 ? nx - x0 : 32;
        const uint8_t *__restrict__ m = mask + r * nx + x0;
        uint32_t v = cnt < 32 ? ~0u << cnt : 0u;
        for (int j = 0; j < cnt; ++j) v |= (uint32_t)(m[j] != 0) << j;
        bits[t] = v;
    }
}

// One round of density classification, chained on the device: round r reads
// the candidate found by round r-1 (words[r-1]; round 0 uses 0), labels the
// cells whose density equals it with class r-1, and leaves the smallest
// density above it in words[r] (all ones when none is left, after which
// later rounds do nothing).  Densities are positive, so the order of their
// bit patterns is numeric order.  Round 0 also marks hull cells.
__global__ void __launch_bounds__(256)
k_classify(const double *__restrict__ r64, uint8_t *__restrict__ cls, int64_t n,
           int round, unsigned long long *__restrict__ words)
{
    __shared__ unsigned long long wmin[4];
    const unsigned long long cand = round > 0 ? words[round - 1] : 0ull;
    if (cand == ~0ull) return;
    unsigned long long local = ~0ull;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const double v = r64[c];
        if (isinf(v)) {
            if (round == 0) cls[c] = (uint8_t)kClsSolid;
            continue;
        }
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        if (b == cand) cls[c] = (uint8_t)(round - 1);
        else if (b > cand && b < local) local = b;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(local, off, 64);
        local = o < local ? o : local;
    }
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = wmin[0];
        for (int w = 1; w < 4; ++w) m = wmin[w] < m ? wmin[w] : m;
        if (m != ~0ull) atomicMin(&words[round], m);
    }
}

// ------------------------------------------------------------------------
// velocity projection and divergence (the step after each pressure solve)
// ------------------------------------------------------------------------

// Face-velocity correction with the solve's face coefficients, on every MAC
// face: out_f = wt (a_f [+ b_f] - dt beta_f (p_hi - p_lo) / h).  Interior
// faces between cells c-1 and c are written by cell c; wall faces use the
// mirrored ghost -p_c (Dirichlet: gradient 2 p_c / h with coefficient
// 1/rho_c, i.e. beta(c, wall) p_c with beta = 2/rho_c) or get no correction
// (Neumann, hull: beta = 0).  wt = 1 without b is the first-stage update
// u* = u^k - dt grad(P*)/rho; wt = 1/2 with b = u^k is the second-stage
// average.  Face arrays are u[nz][ny][nx+1], v[nz][ny+1][nx], w[nz+1][ny][nx];
// out may be a (each face is read and written by one thread).  On a periodic
// axis face 0 is the face between the last and the first cell (corrected by
// the first cell) and the last face is written as its copy.
struct FaceSet {
    const double *u, *v, *w;
};
struct ProjOut {
    double *u, *v, *w;
};

template <bool ADD>
__device__ inline double face_in(const FaceSet &a, const FaceSet &b, int axis, int64_t f)
{
    const double *A = axis == 0 ? a.u : axis == 1 ? a.v : a.w;
    if (!ADD) return gp(A)[f];
    const double *B = axis == 0 ? b.u : axis == 1 ? b.v : b.w;
    return gp(A)[f] + gp(B)[f];
}

template <bool ADD, class C>
__device__ void project_cells(const Slot &S, const C &cf, const double *__restrict__ p,
                              double s, double wt, FaceSet a, FaceSet b, ProjOut o)
{
    using K = typename C::Key;
    const int nx = S.nx, ny = S.ny, nz = S.nz;
    const int64_t P = (int64_t)nx * ny, n = P * nz;
    const int bm = S.bcmask;
    const bool perx = S.permask & 1, pery = S.permask & 2;
    const GLB double *__restrict__ pg = gp(p);
    GLB double *ou = gp(o.u);
    GLB double *ov = gp(o.v);
    GLB double *ow = gp(o.w);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx);
        const int j = (int)((c / nx) % ny);
        const int k = (int)(c / P);
        const K kc = cf.load(c);
        const double pc = pg[c];
        const int64_t fu = ((int64_t)k * ny + j) * (nx + 1) + i;
        const int64_t fv = ((int64_t)k * (ny + 1) + j) * nx + i;
        const int64_t fw = c;
        if (i > 0) {
            ou[fu] = wt * (face_in<ADD>(a, b, 0, fu) - s * cf.beta(cf.load(c - 1), kc) * (pc - pg[c - 1]));
        } else if (perx) {   // shared face with the row's last cell, and its repeat
            const int64_t m = c + nx - 1;
            const double u0 = nx > 1 ? wt * (face_in<ADD>(a, b, 0, fu) - s * cf.beta(cf.load(m), kc) * (pc - pg[m]))
                                     : wt * face_in<ADD>(a, b, 0, fu);
            ou[fu] = u0;
            ou[fu + nx] = u0;
        } else {
            ou[fu] = wt * (face_in<ADD>(a, b, 0, fu) - s * cf.beta(kc, (bm & 1) ? cf.dirichlet() : cf.neumann()) * pc);
        }
        if (i == nx - 1 && !perx)
            ou[fu + 1] = wt * (face_in<ADD>(a, b, 0, fu + 1) + s * cf.beta(kc, (bm & 2) ? cf.dirichlet() : cf.neumann()) * pc);
        if (j > 0) {
            ov[fv] = wt * (face_in<ADD>(a, b, 1, fv) - s * cf.beta(cf.load(c - nx), kc) * (pc - pg[c - nx]));
        } else if (pery) {
            const int64_t m = c + (int64_t)(ny - 1) * nx;
            const double v0 = ny > 1 ? wt * (face_in<ADD>(a, b, 1, fv) - s * cf.beta(cf.load(m), kc) * (pc - pg[m]))
                                     : wt * face_in<ADD>(a, b, 1, fv);
            ov[fv] = v0;
            ov[fv + (int64_t)ny * nx] = v0;
        } else {
            ov[fv] = wt * (face_in<ADD>(a, b, 1, fv) - s * cf.beta(kc, (bm & 4) ? cf.dirichlet() : cf.neumann()) * pc);
        }
        if (j == ny - 1 && !pery)
            ov[fv + nx] = wt * (face_in<ADD>(a, b, 1, fv + nx) + s * cf.beta(kc, (bm & 8) ? cf.dirichlet() : cf.neumann()) * pc);
        if (k > 0) ow[fw] = wt * (face_in<ADD>(a, b, 2, fw) - s * cf.beta(cf.load(c - P), kc) * (pc - pg[c - P]));
        else ow[fw] = wt * (face_in<ADD>(a, b, 2, fw) - s * cf.beta(kc, (bm & 16) ? cf.dirichlet() : cf.neumann()) * pc);
        if (k == nz - 1)
            ow[fw + P] = wt * (face_in<ADD>(a, b, 2, fw + P) + s * cf.beta(kc, (bm & 32) ? cf.dirichlet() : cf.neumann()) * pc);
    }
}

template <bool ADD>
__device__ void project_slot(const Slot &S, double *s_tab64, const double *p, double s,
                             double wt, FaceSet a, FaceSet b, ProjOut o)
{
    if (S.cls) {
        for (int i = threadIdx.x; i < kClasses * kClasses; i += blockDim.x)
            s_tab64[i] = gp(S.tab64)[i];
        __syncthreads();
        project_cells<ADD>(S, ClsCoef<double>{ gp(S.cls), s_tab64 }, p, s, wt, a, b, o);
    } else {
        project_cells<ADD>(S, RhoCoef<double>{ gp(S.rho64) }, p, s, wt, a, b, o);
    }
}

__global__ void __launch_bounds__(256)
k_project(const Slot *__restrict__ slot, const double *__restrict__ p, double s, double wt,
          FaceSet a, FaceSet b, ProjOut o)
{
    __shared__ double s_tab64[kClasses * kClasses];
    if (b.u) project_slot<true>(*slot, s_tab64, p, s, wt, a, b, o);
    else project_slot<false>(*slot, s_tab64, p, s, wt, a, b, o);
}

// Source of the pressure equation from face velocities:
// rhs_c = ((du + dv) + dw) / h / dt with du = U_{i+1/2} - U_{i-1/2} (and so
// on), U = a [+ b], in fluid cells; 0 in hull cells.  With cut cells every
// face value is weighted by its area fraction and the sum divided by the
// cell's volume fraction.  With b the second-stage
// source div(u* + u^k)/dt, without it the first-stage div(u^k)/dt.  On a
// periodic axis the high face of the last cell is face 0 (the last face of
// the array is not read).
template <bool ADD>
__device__ void rhs_cells(const Slot &S, double h, double dt, FaceSet a, FaceSet b,
                          double *__restrict__ rhs)
{
    const int nx = S.nx, ny = S.ny, nz = S.nz;
    const int64_t P = (int64_t)nx * ny, n = P * nz;
    const bool perx = S.permask & 1, pery = S.permask & 2;
    const RhoCoef<double> cf{ gp(S.rho64) };
    GLB double *out = gp(rhs);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        if (cf.solid(cf.load(c))) { out[c] = 0.0; continue; }
        const int i = (int)(c % nx);
        const int j = (int)((c / nx) % ny);
        const int k = (int)(c / P);
        const int64_t fu = ((int64_t)k * ny + j) * (nx + 1) + i;
        const int64_t fv = ((int64_t)k * (ny + 1) + j) * nx + i;
        // the high face of a periodic row's last cell is the row's face 0
        const int64_t fu1 = (perx && i == nx - 1) ? fu - i : fu + 1;
        const int64_t fv1 = (pery && j == ny - 1) ? fv - (int64_t)j * nx : fv + nx;
        if (S.ax) {   // cut cells: area-weighted faces over the volume fraction
            const GLB double *ax = gp(S.ax), *ay = gp(S.ay), *az = gp(S.az);
            const double du = ax[fu1] * face_in<ADD>(a, b, 0, fu1) - ax[fu] * face_in<ADD>(a, b, 0, fu);
            const double dv = ay[fv1] * face_in<ADD>(a, b, 1, fv1) - ay[fv] * face_in<ADD>(a, b, 1, fv);
            const double dw = az[c + P] * face_in<ADD>(a, b, 2, c + P) - az[c] * face_in<ADD>(a, b, 2, c);
            out[c] = ((du + dv) + dw) / (gp(S.vol)[c] * h) / dt;
            continue;
        }
        const double du = face_in<ADD>(a, b, 0, fu1) - face_in<ADD>(a, b, 0, fu);
        const double dv = face_in<ADD>(a, b, 1, fv1) - face_in<ADD>(a, b, 1, fv);
        const double dw = face_in<ADD>(a, b, 2, c + P) - face_in<ADD>(a, b, 2, c);
        out[c] = ((du + dv) + dw) / h / dt;
    }
}

__global__ void __launch_bounds__(256)
k_rhs(const Slot *__restrict__ slot, double h, double dt, FaceSet a, FaceSet b,
      double *__restrict__ rhs)
{
    if (b.u) rhs_cells<true>(*slot, h, dt, a, b, rhs);
    else rhs_cells<false>(*slot, h, dt, a, b, rhs);
}

// (D u)_c = (u_{i+1/2} - u_{i-1/2} + v_{j+1/2} - v_{j-1/2} + w_{k+1/2} -
// w_{k-1/2}) / h over fluid cells (periodic axes and cut cells as in the
// source kernel):
// per-workgroup sum of squares and maximum magnitude, combined on the host in
// workgroup order.
__global__ void __launch_bounds__(256)
k_divnorm(const Slot *__restrict__ slot, double inv_h, const double *__restrict__ u,
          const double *__restrict__ v, const double *__restrict__ w,
          double *__restrict__ part)
{
    __shared__ double lds[8];
    const Slot &S = *slot;
    const int nx = S.nx, ny = S.ny, nz = S.nz;
    const int64_t P = (int64_t)nx * ny, n = P * nz;
    const RhoCoef<double> cf{ gp(S.rho64) };
    const bool perx = S.permask & 1, pery = S.permask & 2;
    double ss = 0.0, mx = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        if (cf.solid(cf.load(c))) continue;
        const int i = (int)(c % nx);
        const int j = (int)((c / nx) % ny);
        const int k = (int)(c / P);
        const int64_t fu = ((int64_t)k * ny + j) * (nx + 1) + i;
        const int64_t fv = ((int64_t)k * (ny + 1) + j) * nx + i;
        const int64_t fu1 = (perx && i == nx - 1) ? fu - i : fu + 1;
        const int64_t fv1 = (pery && j == ny - 1) ? fv - (int64_t)j * nx : fv + nx;
        double d;
        if (S.ax) {   // cut cells: area-weighted faces over the volume fraction
            const GLB double *ax = gp(S.ax), *ay = gp(S.ay), *az = gp(S.az);
            d = ((ax[fu1] * u[fu1] - ax[fu] * u[fu]) + (ay[fv1] * v[fv1] - ay[fv] * v[fv]) +
                 (az[c + P] * w[c + P] - az[c] * w[c])) / gp(S.vol)[c] * inv_h;
        } else {
            d = ((u[fu1] - u[fu]) + (v[fv1] - v[fv]) + (w[c + P] - w[c])) * inv_h;
        }
        ss += d * d;
        mx = fmax(mx, fabs(d));
    }
    double a[1] = { ss };
    ss = wave_sum(a[0]);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) { lds[threadIdx.x >> 6] = ss; lds[4 + (threadIdx.x >> 6)] = mx; }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
        part[2 * blockIdx.x + 1] = fmax(fmax(lds[4], lds[5]), fmax(lds[6], lds[7]));
    }
}

// Validation of cut-cell fractions: every area in [0, 1] and every fluid
// cell's volume in (0, 1] (NaN fails both); sets *bad otherwise.
__global__ void __launch_bounds__(256)
k_check_frac(const double *__restrict__ ax, const double *__restrict__ ay,
             const double *__restrict__ az, const double *__restrict__ vol,
             const double *__restrict__ rho64, int64_t nu, int64_t nv, int64_t nw,
             int64_t n, int *bad)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = true;
    for (int64_t f = i0; f < nu; f += stride) ok = ok && ax[f] >= 0.0 && ax[f] <= 1.0;
    for (int64_t f = i0; f < nv; f += stride) ok = ok && ay[f] >= 0.0 && ay[f] <= 1.0;
    for (int64_t f = i0; f < nw; f += stride) ok = ok && az[f] >= 0.0 && az[f] <= 1.0;
    for (int64_t c = i0; c < n; c += stride)
        ok = ok && (isinf(rho64[c]) || (vol[c] > 0.0 && vol[c] <= 1.0));
    if (!ok) atomicOr(bad, 1);
}

// Copy probe: one element per thread, one pass (the fastest plain copy
// shape measured on this part).
__global__ void __launch_bounds__(256)
k_copy(const double *__restrict__ src, double *__restrict__ dst, int64_t n)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) dst[c] = src[c];
}

// Triad probe (STREAM's a = b + s c), one element per thread like the copy.
__global__ void __launch_bounds__(256)
k_triad(double *__restrict__ a, const double *__restrict__ b, const double *__restrict__ c,
        double s, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = fma(s, c[i], b[i]);
}

// ------------------------------------------------------------------------
// host-callable launchers
// ------------------------------------------------------------------------

// Device memory of the allocation-free entry point (pcg_solve_static): the
// slot table, slot state and one solve's vectors live here instead of in a
// caller's workspace.  Each device the library runs on holds its own copy
// until the process ends; host code reaches it only through the address
// static_scratch returns (the array's name is not a device address on the
// host).
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// Address and size of the current device's copy of `scratch`, looked up once
// per device (with that device current) and kept.
hipError_t static_scratch(void **ptr, size_t *bytes)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = a;
    }
    *ptr = addr[dev];
    *bytes = kStaticScratchBytes;
    return hipSuccess;
}

hipError_t launch_iter(int family, int which, int mode, int grid,
                       const BatchHeader *hdr, const Slot *slots, hipStream_t s)
{
    const dim3 g(grid), b(kBlock);
#define PCG_LAUNCH(F, W, M) hipLaunchKernelGGL((k_iter<F, W, M>), g, b, 0, s, hdr, slots)
#define PCG_MODES(F, W, NM)                                       \
    do {                                                          \
        if (mode == 0) PCG_LAUNCH(F, W, 0);                       \
        else if (mode == 1) PCG_LAUNCH(F, W, 1);                  \
        else if (mode == 2) PCG_LAUNCH(F, W, 2);                  \
        else if (NM > 3 && mode == 3) PCG_LAUNCH(F, W, 3);        \
        else if (NM > 4 && mode == 4) PCG_LAUNCH(F, W, 4);        \
        else return hipErrorInvalidValue;                         \
    } while (0)
    if (family == PCG_PREC_FP64) {
        if (which == 3) PCG_MODES(PCG_PREC_FP64, 3, 5);
        else if (which == 1) PCG_MODES(PCG_PREC_FP64, 1, 5);
        else PCG_MODES(PCG_PREC_FP64, 2, 5);
    } else {
        if (which == 3) PCG_MODES(PCG_PREC_FP32_IR, 3, 5);
        else if (which == 1) PCG_MODES(PCG_PREC_FP32_IR, 1, 5);
        else PCG_MODES(PCG_PREC_FP32_IR, 2, 5);
    }
#undef PCG_MODES
#undef PCG_LAUNCH
    return hipGetLastError();
}

hipError_t launch_classify(const double *r64, uint8_t *cls, int64_t n, int round,
                           unsigned long long *words, hipStream_t s)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_classify, dim3((unsigned)blocks), dim3(256), 0, s, r64, cls,
                       n, round, words);
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

hipError_t launch_project(const Slot *slot, const double *p, double s, double wt,
                          const double *const a[3], const double *const b[3],
                          double *const out[3], int blocks, hipStream_t st)
{
    const FaceSet fa{ a[0], a[1], a[2] };
    const FaceSet fb{ b ? b[0] : nullptr, b ? b[1] : nullptr, b ? b[2] : nullptr };
    const ProjOut o{ out[0], out[1], out[2] };
    hipLaunchKernelGGL(k_project, dim3(blocks), dim3(256), 0, st, slot, p, s, wt, fa, fb, o);
    return hipGetLastError();
}

hipError_t launch_rhs(const Slot *slot, double h, double dt, const double *const a[3],
                      const double *const b[3], double *rhs, int blocks, hipStream_t st)
{
    const FaceSet fa{ a[0], a[1], a[2] };
    const FaceSet fb{ b ? b[0] : nullptr, b ? b[1] : nullptr, b ? b[2] : nullptr };
    hipLaunchKernelGGL(k_rhs, dim3(blocks), dim3(256), 0, st, slot, h, dt, fa, fb, rhs);
    return hipGetLastError();
}

hipError_t launch_divnorm(const Slot *slot, double inv_h, const double *u,
                          const double *v, const double *w, double *part, int blocks,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_divnorm, dim3(blocks), dim3(256), 0, st, slot, inv_h, u, v, w,
                       part);
    return hipGetLastError();
}

hipError_t launch_check_frac(const double *ax, const double *ay, const double *az,
                             const double *vol, const double *rho64, int64_t nu, int64_t nv,
                             int64_t nw, int64_t n, int *bad, hipStream_t s)
{
    int64_t blocks = (nw + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_check_frac, dim3((unsigned)blocks), dim3(256), 0, s, ax, ay, az, vol,
                       rho64, nu, nv, nw, n, bad);
    return hipGetLastError();
}

hipError_t launch_triad(double *a, const double *b, const double *c, double sc, size_t n,
                        hipStream_t s)
{
    const int64_t blocks = ((int64_t)n + 255) / 256;
    if (blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_triad, dim3((unsigned)blocks), dim3(256), 0, s, a, b, c, sc,
                       (int64_t)n);
    return hipGetLastError();
}

hipError_t launch_pack_mask(const uint8_t *mask, uint32_t *bits, int nx,
                            int words_per_row, int64_t nwords, hipStream_t s)
{
    int64_t blocks = (nwords + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_pack_mask, dim3((unsigned)blocks), dim3(256), 0, s, mask, bits,
                       nx, words_per_row, nwords);
    return hipGetLastError();
}

hipError_t launch_copy(const double *src, double *dst, size_t n, hipStream_t s)
{
    const int64_t blocks = ((int64_t)n + 255) / 256;
    if (blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, src, dst,
                       (int64_t)n);
    return hipGetLastError();
}

}  // namespace pcgmi
