"""Pins of the CPU reference against facts that do not come from it.

Each test checks the reference against something fixed by the paper's
equations and by mathematics: hand-solved tiny problems, exact discrete
eigenvectors, second-order convergence to a manufactured continuous solution,
symmetry and definiteness, a dense direct solve assembled independently, a
1-D reduction solved by a banded routine, the divergence of the projected
velocity, invariances, and the finite termination of conjugate gradients.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

GOLD = os.path.join(os.path.dirname(__file__), "golden")
D, N = 1, 0
ALL_D = (D, D, D, D, D, D)
TANK = (N, N, N, N, N, D)


def _grid(nx, ny, nz):
    h = 1.0 / nz
    x = (np.arange(nx) + 0.5) * h
    y = (np.arange(ny) + 0.5) * h
    z = (np.arange(nz) + 0.5) * h
    return h, x[None, None, :], y[None, :, None], z[:, None, None]


# --------------------------------------------------------------------------
# hand-solved problems (tests/golden/hand_solved.json)
# --------------------------------------------------------------------------

def _gold_cases():
    with open(os.path.join(GOLD, "hand_solved.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _gold_cases(), ids=lambda c: c["name"])
def test_hand_solved(orc, case):
    shp = (case["nz"], case["ny"], case["nx"])
    rho = np.array(case["rho"], float).reshape(shp)
    mask = np.array(case["mask"], np.uint8).reshape(shp)
    rhs = np.array(case["rhs"], float).reshape(shp)
    want = np.array(case["p"], float).reshape(shp)
    # operator: L applied to the hand solution gives the source on fluid cells
    Lp = orc.apply(rho, mask, case["bc"], case["h"], want)
    fluid = mask == 0
    np.testing.assert_allclose(Lp[fluid], rhs[fluid], rtol=1e-12, atol=1e-12)
    # solver
    r = orc.pcg(rho, mask, case["bc"], case["h"], rhs, tol=1e-14, maxit=50)
    assert r.status == orc.OK
    np.testing.assert_allclose(r.p, want, rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# exact discrete eigenvectors
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape,c,modes", [
    ((8, 8, 8), 1.0, (1, 1, 1)),
    ((12, 10, 8), 2.5, (1, 2, 3)),
    ((5, 9, 7), 1000.0, (2, 1, 1)),
])
def test_eigvec_all_dirichlet(orc, shape, c, modes):
    """prod_d sin(m_d pi x_d / L_d) at cell centres is an exact eigenvector
    of the face-Dirichlet operator with eigenvalue
    -(1/c) sum_d 2(1 - cos(m_d pi h / L_d)) / h^2."""
    nx, ny, nz = shape
    h, x, y, z = _grid(nx, ny, nz)
    L = (nx * h, ny * h, nz * h)
    m = modes
    v = (np.sin(m[0] * math.pi * x / L[0]) * np.sin(m[1] * math.pi * y / L[1])
         * np.sin(m[2] * math.pi * z / L[2]))
    lam = sum(2.0 * (1.0 - math.cos(m[d] * math.pi * h / L[d])) for d in range(3))
    rho = np.full((nz, ny, nx), c)
    mask = np.zeros((nz, ny, nx), np.uint8)
    Lv = orc.apply(rho, mask, ALL_D, h, v)
    np.testing.assert_allclose(Lv, -(lam / c) / h**2 * v, rtol=0,
                               atol=1e-11 * np.abs(lam / c / h**2))
    # the solver returns the eigenvector for the matching source
    r = orc.pcg(rho, mask, ALL_D, h, -(lam / c) / h**2 * v, tol=1e-13)
    assert r.status == orc.OK
    np.testing.assert_allclose(r.p, v, rtol=0, atol=1e-9)


@pytest.mark.parametrize("shape", [(8, 8, 8), (10, 6, 12)])
def test_eigvec_tank(orc, shape):
    """Neumann on x, y and the bottom, p = 0 on top:
    cos(pi x/Lx) cos(pi y/Ly) cos(pi z/(2 Lz)) is exact with eigenvalue
    -[2(1-cos(pi h/Lx)) + 2(1-cos(pi h/Ly)) + 2(1-cos(pi h/(2Lz)))]/h^2."""
    nx, ny, nz = shape
    h, x, y, z = _grid(nx, ny, nz)
    Lx, Ly, Lz = nx * h, ny * h, nz * h
    v = (np.cos(math.pi * x / Lx) * np.cos(math.pi * y / Ly)
         * np.cos(math.pi * z / (2 * Lz)))
    lam = (2 * (1 - math.cos(math.pi * h / Lx)) + 2 * (1 - math.cos(math.pi * h / Ly))
           + 2 * (1 - math.cos(math.pi * h / (2 * Lz))))
    rho = np.ones((nz, ny, nx))
    mask = np.zeros((nz, ny, nx), np.uint8)
    Lv = orc.apply(rho, mask, TANK, h, v)
    np.testing.assert_allclose(Lv, -lam / h**2 * v, rtol=0,
                               atol=1e-11 * lam / h**2)


# --------------------------------------------------------------------------
# manufactured continuous solution: second order
# --------------------------------------------------------------------------

def test_manufactured_second_order(orc):
    """Sigma = -3 pi^2 sin(pi x) sin(pi y) sin(pi z) with p = 0 on all walls
    of the unit cube has the continuous solution sin sin sin; the discrete
    error must fall by about 4 per halving of h."""
    errs = []
    for n in (8, 16, 32):
        h, x, y, z = _grid(n, n, n)
        exact = np.sin(math.pi * x) * np.sin(math.pi * y) * np.sin(math.pi * z)
        rhs = -3 * math.pi**2 * exact
        rho = np.ones((n, n, n))
        r = orc.pcg(rho, np.zeros((n, n, n), np.uint8), ALL_D, h, rhs, tol=1e-12)
        assert r.status == orc.OK
        errs.append(np.abs(r.p - exact).max())
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    for q in ratios:
        assert 3.5 < q < 4.5, (errs, ratios)


# --------------------------------------------------------------------------
# symmetry and definiteness
# --------------------------------------------------------------------------

def _two_phase_wedge(F, nx, ny, nz, bc=(D, N, N, D, N, D)):
    c = F.make_two_phase(nx, ny, nz, surface_seed=5, velocity_seed=6,
                         wedge=F.Wedge(), bc=bc)
    return c


def test_symmetric_positive_definite(orc, F):
    c = _two_phase_wedge(F, 14, 12, 10)
    assert c.mask.any() and (c.rho == F.RHO_AIR).any() and (c.rho == F.RHO_WATER).any()
    fluid = c.mask == 0
    rng = np.random.default_rng(3)
    for _ in range(5):
        x = rng.standard_normal(c.shape) * fluid
        y = rng.standard_normal(c.shape) * fluid
        Lx = orc.apply(c.rho, c.mask, c.bc, c.h, x)
        Ly = orc.apply(c.rho, c.mask, c.bc, c.h, y)
        a, b = np.vdot(x, Ly), np.vdot(y, Lx)
        scale = np.linalg.norm(x) * np.linalg.norm(Ly)
        assert abs(a - b) <= 1e-13 * scale
        assert np.vdot(x, Lx) < 0.0          # -L is positive definite


# --------------------------------------------------------------------------
# dense direct solve, assembled here from the definition
# --------------------------------------------------------------------------

def _dense_minus_h2L(rho, mask, bc):
    nz, ny, nx = rho.shape
    n = rho.size
    A = np.zeros((n, n))
    idx = lambda i, j, k: (k * ny + j) * nx + i
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = idx(i, j, k)
                if mask[k, j, i]:
                    A[c, c] = 1.0
                    continue
                for f, (di, dj, dk) in enumerate([(-1, 0, 0), (1, 0, 0), (0, -1, 0),
                                                  (0, 1, 0), (0, 0, -1), (0, 0, 1)]):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                        if mask[kk, jj, ii]:
                            continue
                        b = 2.0 / (rho[k, j, i] + rho[kk, jj, ii])
                        m = idx(ii, jj, kk)
                        A[c, c] += b
                        A[c, m] -= b
                    elif bc[f] == D:
                        A[c, c] += 2.0 / rho[k, j, i]
    return A


@pytest.mark.parametrize("shape,bc,wedge", [
    ((6, 5, 8), TANK, True),
    ((8, 8, 8), (D, N, N, D, N, D), True),
    ((7, 4, 6), ALL_D, False),
])
def test_dense_cholesky(orc, F, shape, bc, wedge):
    nx, ny, nz = shape
    c = F.make_two_phase(nx, ny, nz, surface_seed=11, velocity_seed=12,
                         wedge=F.Wedge() if wedge else None, bc=bc)
    A = _dense_minus_h2L(c.rho, c.mask, c.bc)
    b = (-c.h**2 * c.rhs * (c.mask == 0)).ravel()
    Lc = np.linalg.cholesky(A)
    p = scipy.linalg.solve_triangular(Lc.T, scipy.linalg.solve_triangular(Lc, b, lower=True))
    r = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-14, maxit=5000)
    assert r.status in (orc.OK, orc.MAXIT)
    scale = np.abs(p).max()
    assert np.abs(r.p.ravel() - p).max() <= 1e-10 * scale


def _textbook_jacobi_pcg_iters(A, b, tol, maxit=10000):
    """Hestenes-Stiefel conjugate gradients preconditioned by the diagonal of
    A (Saad, Iterative Methods for Sparse Linear Systems, Alg. 9.1), on a
    dense matrix: the iteration at which ||r|| <= tol ||b|| first holds."""
    d = np.diag(A).copy()
    x = np.zeros_like(b)
    r = b.copy()
    z = r / d
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    for k in range(1, maxit + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= tol * nb:
            return k
        z = r / d
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return maxit


@pytest.mark.parametrize("shape,bc,wedge,seed", [
    ((6, 5, 8), TANK, True, 11),
    ((8, 8, 8), (D, N, N, D, N, D), True, 11),
    ((12, 6, 3), ALL_D, True, 11),
    ((16, 4, 2), (D, D, N, N, D, D), True, 7),
])
def test_pcg_iterations_match_textbook(orc, F, shape, bc, wedge, seed):
    """The reference's iteration count equals that of textbook Jacobi-PCG on
    the independently assembled matrix.  This pins the preconditioner
    (Jacobi, reading R9), which the solution pins cannot see since any
    diagonal leads to the same answer.  In these cases the relative residual
    is at least 1.1 tol one iteration before the stop and at most 0.97 tol
    at it, so rounding differences between the two cannot move the count."""
    nx, ny, nz = shape
    c = F.make_two_phase(nx, ny, nz, surface_seed=seed, velocity_seed=seed + 1,
                         wedge=F.Wedge() if wedge else None, bc=bc)
    A = _dense_minus_h2L(c.rho, c.mask, c.bc)
    b = (-c.h**2 * c.rhs * (c.mask == 0)).ravel()
    k_ref = _textbook_jacobi_pcg_iters(A, b, 1e-8)
    r = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-8)
    assert r.status == orc.OK
    assert r.iters == k_ref, (r.iters, k_ref)


# --------------------------------------------------------------------------
# 1-D reduction: flat interface, Neumann sides, source depending on z only
# --------------------------------------------------------------------------

def test_column_reduction_banded(orc):
    nx, ny, nz = 3, 4, 16
    h = 1.0 / nz
    zc = (np.arange(nz) + 0.5) * h
    rho1 = np.where(zc < 0.5, 1000.0, 1.2)
    sig1 = np.cos(3 * zc) + 0.3
    rho = np.broadcast_to(rho1[:, None, None], (nz, ny, nx)).copy()
    rhs = np.broadcast_to(sig1[:, None, None], (nz, ny, nx)).copy()
    mask = np.zeros((nz, ny, nx), np.uint8)
    r = orc.pcg(rho, mask, TANK, h, rhs, tol=1e-12)
    assert r.status == orc.OK
    # tridiagonal -h^2 L restricted to the column
    bf = 2.0 / (rho1[:-1] + rho1[1:])          # faces k+1/2
    diag = np.zeros(nz)
    diag[:-1] += bf
    diag[1:] += bf
    diag[-1] += 2.0 / rho1[-1]                 # p = 0 on the top face
    ab = np.zeros((3, nz))
    ab[0, 1:] = -bf
    ab[1] = diag
    ab[2, :-1] = -bf
    p1 = scipy.linalg.solve_banded((1, 1), ab, -h**2 * sig1)
    for j in range(ny):
        for i in range(nx):
            np.testing.assert_allclose(r.p[:, j, i], p1, rtol=1e-8,
                                       atol=1e-12 * np.abs(p1).max())


# --------------------------------------------------------------------------
# divergence of the projected velocity
# --------------------------------------------------------------------------

@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_projection_divergence(orc, F, tol):
    """With Sigma = D u / dt, u - dt (1/rho) grad p has divergence
    dt (Sigma - L p): its norm relative to ||D u|| is the relative residual."""
    c = _two_phase_wedge(F, 20, 16, 18, bc=TANK)
    r = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=tol)
    assert r.status == orc.OK
    div0 = orc.divergence(c.u, c.v, c.w, c.h)
    u, v, w = orc.project(c.rho, c.mask, c.bc, c.h, c.dt, r.p, c.u, c.v, c.w)
    div1 = orc.divergence(u, v, w, c.h)
    ratio = np.linalg.norm(div1) / np.linalg.norm(div0)
    assert ratio <= tol
    assert abs(ratio - r.relres) <= 1e-6 * r.relres + 1e-15
    # hull and Neumann faces keep zero normal velocity
    assert np.all(u[:, :, 0] == 0) and np.all(w[0] == 0)


# --------------------------------------------------------------------------
# invariances
# --------------------------------------------------------------------------

def test_density_scaling(orc, F):
    c = _two_phase_wedge(F, 12, 10, 12, bc=TANK)
    r1 = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-12)
    r3 = orc.pcg(3.0 * c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-12)
    np.testing.assert_allclose(r3.p, 3.0 * r1.p, rtol=0,
                               atol=1e-8 * np.abs(r1.p).max())


def test_axis_swap_and_mirror(orc, F):
    c = _two_phase_wedge(F, 12, 10, 8, bc=(D, N, N, N, N, D))
    base = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-12).p
    s = np.abs(base).max()
    # swap x and y (and their boundary kinds)
    bc_t = (c.bc[2], c.bc[3], c.bc[0], c.bc[1], c.bc[4], c.bc[5])
    t = lambda a: np.ascontiguousarray(np.swapaxes(a, 1, 2))
    pt = orc.pcg(t(c.rho), t(c.mask), bc_t, c.h, t(c.rhs), tol=1e-12).p
    np.testing.assert_allclose(pt, t(base), rtol=0, atol=1e-8 * s)
    # mirror in x (swap x- and x+)
    bc_m = (c.bc[1], c.bc[0]) + tuple(c.bc[2:])
    m = lambda a: np.ascontiguousarray(a[:, :, ::-1])
    pm = orc.pcg(m(c.rho), m(c.mask), bc_m, c.h, m(c.rhs), tol=1e-12).p
    np.testing.assert_allclose(pm, m(base), rtol=0, atol=1e-8 * s)


# --------------------------------------------------------------------------
# conjugate gradients terminate in at most n steps (up to rounding)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("nz", [2, 5, 8])
def test_finite_termination(orc, nz):
    """On an n-unknown SPD system CG terminates in at most n steps in exact
    arithmetic; a steepest-descent or mis-scaled update does not."""
    h = 1.0 / nz
    rho = np.where((np.arange(nz) + 0.5) * h < 0.5, 1000.0, 1.2)[:, None, None].copy()
    rhs = np.linspace(1.0, 2.0, nz)[:, None, None].copy()
    r = orc.pcg(rho, np.zeros_like(rho, np.uint8), TANK, h, rhs, tol=1e-12, maxit=200)
    assert r.status == orc.OK
    assert r.iters <= nz + 1


# --------------------------------------------------------------------------
# failure reporting
# --------------------------------------------------------------------------

def test_failures(orc):
    n = 4
    rho = np.ones((n, n, n))
    mask = np.zeros((n, n, n), np.uint8)
    rhs = np.ones((n, n, n))
    h = 1.0 / n
    P = 2
    # one no-flux region: singular; a constant source is all null space
    r = orc.pcg(rho, mask, (N,) * 6, h, rhs)
    assert r.status == orc.OK and r.iters == 0 and not r.p.any()
    assert orc.pcg(rho, mask, (P, P, N, N, N, D), h, rhs).status == orc.OK
    assert orc.pcg(rho, mask, (N, N, N, N, P, P), h, rhs).status == orc.EUNSUPPORTED
    assert orc.pcg(rho, mask, (P, N, N, N, N, D), h, rhs).status == orc.EINVAL
    bad = rho.copy(); bad[1, 1, 1] = -1.0
    assert orc.pcg(bad, mask, TANK, h, rhs).status == orc.EDOMAIN
    bad[1, 1, 1] = np.nan
    assert orc.pcg(bad, mask, TANK, h, rhs).status == orc.EDOMAIN
    # a negative density inside the hull is ignored
    m2 = mask.copy(); m2[1, 1, 1] = 1; bad[1, 1, 1] = -1.0
    assert orc.pcg(bad, m2, TANK, h, rhs).status == orc.OK
    # sealed fluid pocket: one fluid cell at the bottom centre walled by hull
    m3 = np.zeros((n, n, n), np.uint8)
    m3[0:2, 0:3, 0:3] = 1
    m3[0, 1, 1] = 0
    assert not orc.connected(m3, TANK)
    assert orc.pcg(rho, m3, TANK, h, rhs).status == orc.ESINGULAR
    # two no-flux regions: the constant on each is a null vector
    assert orc.components(m3, (N,) * 6) == (2, 2)
    assert orc.pcg(rho, m3, (N,) * 6, h, rhs).status == orc.ESINGULAR
    # zero source: p = 0 with no iteration
    r = orc.pcg(rho, mask, TANK, h, np.zeros_like(rhs))
    assert r.status == orc.OK and r.iters == 0 and not r.p.any()
    # iteration cap
    r = orc.pcg(rho, mask, TANK, h, rhs, tol=1e-14, maxit=1)
    assert r.status == orc.MAXIT and r.iters == 1


# --------------------------------------------------------------------------
# the two-stage Runge-Kutta pressure pair (Section 2.1)
# --------------------------------------------------------------------------

def _pair_case(F, nx=16, ny=12, nz=14, shift=0.6):
    c = F.make_two_phase(nx, ny, nz, surface_seed=21, velocity_seed=22,
                         wedge=F.Wedge(), bc=TANK)
    rho_s = F.stage_density(nx, ny, nz, surface_seed=21, velocity_seed=22,
                            phase_shift=shift)
    return c, rho_s


def test_source_matches_generator(orc, F):
    """The oracle's source is the generator's div(u)/dt (zero on the hull)."""
    c = _two_phase_wedge(F, 12, 10, 9, bc=TANK)
    np.testing.assert_array_equal(orc.source(c.u, c.v, c.w, c.h, c.dt, c.mask), c.rhs)


def test_source_linear_field(orc):
    """u = (a x, b y, c z) on the faces has divergence a + b + c in every cell."""
    nx, ny, nz = 5, 4, 6
    h = 1.0 / nz
    a, b, cc, dt = 0.75, -2.0, 0.5, 1e-3
    u = np.broadcast_to(a * np.arange(nx + 1) * h, (nz, ny, nx + 1)).copy()
    v = np.broadcast_to((b * np.arange(ny + 1) * h)[:, None], (nz, ny + 1, nx)).copy()
    w = np.broadcast_to((cc * np.arange(nz + 1) * h)[:, None, None], (nz + 1, ny, nx)).copy()
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[2, 1, 3] = 1
    s = orc.source(u, v, w, h, dt, mask)
    expect = np.full((nz, ny, nx), (a + b + cc) / dt)
    expect[2, 1, 3] = 0.0
    np.testing.assert_allclose(s, expect, rtol=1e-12)


def test_pair_same_density_is_idempotent(orc, F):
    """With rho(phi*) = rho(phi^k) the second stage re-solves the first
    stage's equation (its source differs by the first residual), so
    P^{k+1} = P* and u^{k+1} = u* up to that residual."""
    c, _ = _pair_case(F)
    out = orc.rk2_pair(c.rho, c.rho, c.mask, c.bc, c.h, c.dt, c.u, c.v, c.w, tol=1e-12)
    assert np.abs(out["p_next"] - out["p_star"]).max() <= 1e-8 * np.abs(out["p_star"]).max()
    for a, b in zip(out["u_next"], out["u_star"]):
        assert np.abs(a - b).max() <= 1e-8 * np.abs(b).max()
    # a dropped one-half would double u*; a dropped u^k in the second source
    # would leave half of u^k's divergence: both far outside these bounds
    d0 = np.linalg.norm(orc.divergence(c.u, c.v, c.w, c.h))
    assert np.linalg.norm(orc.divergence(*out["u_next"], c.h)) <= 1e-10 * d0


@pytest.mark.parametrize("shift", [0.3, 1.5])
def test_pair_divergence_free(orc, F, shift):
    """D u^{k+1} = (dt/2) (Sigma_2 - L* P^{k+1}): solenoidal to the second
    solve's residual, which needs rho(phi*) in both the solve and the
    face update."""
    c, rho_s = _pair_case(F, shift=shift)
    assert (rho_s != c.rho).any()
    tol = 1e-10
    out = orc.rk2_pair(c.rho, rho_s, c.mask, c.bc, c.h, c.dt, c.u, c.v, c.w, tol=tol)
    s2 = orc.source(*(a + b for a, b in zip(out["u_star"], (c.u, c.v, c.w))), c.h, c.dt,
                    c.mask)
    d1 = np.linalg.norm(orc.divergence(*out["u_next"], c.h))
    assert d1 <= 0.5 * c.dt * tol * np.linalg.norm(s2) * 1.01
    # u* is solenoidal under the first-stage density
    ds = np.linalg.norm(orc.divergence(*out["u_star"], c.h))
    assert ds <= c.dt * tol * np.linalg.norm(c.rhs) * 1.01


def test_pair_dense(orc, F):
    """Both stage pressures against dense Cholesky solves assembled from the
    definition, on a tiny wedge case."""
    nx, ny, nz = 6, 5, 8
    c = F.make_two_phase(nx, ny, nz, surface_seed=31, velocity_seed=32, wedge=F.Wedge(),
                         bc=TANK)
    rho_s = F.stage_density(nx, ny, nz, surface_seed=31, velocity_seed=32, phase_shift=2.0)
    out = orc.rk2_pair(c.rho, rho_s, c.mask, c.bc, c.h, c.dt, c.u, c.v, c.w, tol=1e-14)
    fluid = c.mask == 0

    def dense(rho, rhs):
        A = _dense_minus_h2L(rho, c.mask, c.bc)
        Lc = np.linalg.cholesky(A)
        b = (-c.h**2 * rhs * fluid).ravel()
        return scipy.linalg.solve_triangular(
            Lc.T, scipy.linalg.solve_triangular(Lc, b, lower=True)).reshape(rho.shape)

    p1 = dense(c.rho, c.rhs)
    assert np.abs(out["p_star"] - p1).max() <= 1e-10 * np.abs(p1).max()
    s2 = orc.source(*(a + b for a, b in zip(out["u_star"], (c.u, c.v, c.w))), c.h, c.dt,
                    c.mask)
    p2 = dense(rho_s, s2)
    assert np.abs(out["p_next"] - p2).max() <= 1e-10 * np.abs(p2).max()


# --------------------------------------------------------------------------
# periodic walls and the singular (no Dirichlet wall) problem
# --------------------------------------------------------------------------

P_ = 2   # periodic wall kind


@pytest.mark.parametrize("shape,modes", [((12, 10, 8), (1, 2)), ((9, 14, 7), (2, 1))])
def test_eigvec_periodic(orc, shape, modes):
    """Periodic x and y, p = 0 on the bottom and top faces:
    cos(2 pi m1 x/Lx + a) cos(2 pi m2 y/Ly + b) sin(pi z/Lz) at cell centres
    is an exact eigenvector, eigenvalue sum of 2(1 - cos(theta h))/h^2."""
    nx, ny, nz = shape
    h, x, y, z = _grid(nx, ny, nz)
    Lx, Ly, Lz = nx * h, ny * h, nz * h
    m1, m2 = modes
    v = (np.cos(2 * math.pi * m1 * x / Lx + 0.3) * np.cos(2 * math.pi * m2 * y / Ly + 1.1)
         * np.sin(math.pi * z / Lz))
    lam = (2 * (1 - math.cos(2 * math.pi * m1 * h / Lx)) + 2 * (1 - math.cos(2 * math.pi * m2 * h / Ly))
           + 2 * (1 - math.cos(math.pi * h / Lz))) / h**2
    rho = np.ones((nz, ny, nx))
    mask = np.zeros((nz, ny, nx), np.uint8)
    bc = (P_, P_, P_, P_, D, D)
    Lv = orc.apply(rho, mask, bc, h, v)
    assert np.abs(Lv + lam * v).max() <= 1e-10 * lam
    r = orc.pcg(rho, mask, bc, h, -lam * v, tol=1e-13)
    assert r.status == orc.OK
    assert np.abs(r.p - v).max() <= 1e-9


@pytest.mark.parametrize("shape,modes,const", [((10, 8, 12), (1, 0, 2), 0.0),
                                               ((7, 9, 6), (0, 3, 1), 37.0)])
def test_eigvec_pure_neumann(orc, shape, modes, const):
    """No-flux walls only: cos(pi m x/Lx) cos(pi m y/Ly) cos(pi m z/Lz) (not
    all m zero) is an exact eigenvector of zero mean.  A constant added to
    the source lies along the null vector and must not change the
    zero-mean answer."""
    nx, ny, nz = shape
    h, x, y, z = _grid(nx, ny, nz)
    m1, m2, m3 = modes
    v = (np.cos(math.pi * m1 * x / (nx * h)) * np.cos(math.pi * m2 * y / (ny * h))
         * np.cos(math.pi * m3 * z / (nz * h)))
    lam = sum(2 * (1 - math.cos(math.pi * m * h / (n * h))) for m, n in zip(modes, shape)) / h**2
    rho = np.full((nz, ny, nx), 3.0)
    mask = np.zeros((nz, ny, nx), np.uint8)
    bc = (N,) * 6
    assert orc.components(mask, bc) == (1, 1)
    r = orc.pcg(rho, mask, bc, h, -lam / 3.0 * v + const, tol=1e-13)
    assert r.status == orc.OK
    assert abs(r.p.mean()) <= 1e-12
    assert np.abs(r.p - v).max() <= 1e-9


def _dense_minus_h2L_periodic(rho, mask, bc):
    """-h^2 L with periodic x/y wrap, assembled cell by cell from the face
    rules (beta = 2/(rho_c + rho_n), hull faces closed, Dirichlet ghost)."""
    nz, ny, nx = rho.shape
    n = rho.size
    A = np.zeros((n, n))
    idx = lambda i, j, k: (k * ny + j) * nx + i
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = idx(i, j, k)
                if mask[k, j, i]:
                    A[c, c] = 1.0
                    continue
                for f, (di, dj, dk) in enumerate([(-1, 0, 0), (1, 0, 0), (0, -1, 0),
                                                  (0, 1, 0), (0, 0, -1), (0, 0, 1)]):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if bc[f] == P_:
                        if (nx if f < 2 else ny) == 1:
                            continue
                        ii, jj = ii % nx, jj % ny
                    if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                        if mask[kk, jj, ii]:
                            continue
                        b = 2.0 / (rho[k, j, i] + rho[kk, jj, ii])
                        A[c, c] += b
                        A[c, idx(ii, jj, kk)] -= b
                    elif bc[f] == D:
                        A[c, c] += 2.0 / rho[k, j, i]
    return A


@pytest.mark.parametrize("shape,bc", [
    ((9, 6, 7), (P_, P_, N, N, N, N)),        # strut walls: singular
    ((8, 5, 6), (P_, P_, N, N, N, D)),        # periodic x with a p = 0 top
    ((5, 7, 6), (N, N, P_, P_, N, N)),        # periodic y, singular
])
def test_dense_periodic(orc, F, shape, bc):
    """Two-phase wedge field: against a dense solve of the independently
    assembled matrix (least-squares minimum-norm solution of the fluid block
    for the singular cases, which is the zero-mean one)."""
    nx, ny, nz = shape
    c = F.make_two_phase(nx, ny, nz, surface_seed=41, velocity_seed=42,
                         wedge=F.Wedge(), bc=bc)
    fluid = (c.mask == 0).ravel()
    A = _dense_minus_h2L_periodic(c.rho, c.mask, bc)[np.ix_(fluid, fluid)]
    b = (-c.h**2 * c.rhs).ravel()[fluid]
    singular = D not in bc
    if singular:
        b = b - b.mean()
        want = np.linalg.lstsq(A, b, rcond=None)[0]
        assert abs(want.mean()) <= 1e-10 * np.abs(want).max()
    else:
        want = np.linalg.solve(A, b)
    r = orc.pcg(c.rho, c.mask, bc, c.h, c.rhs, tol=1e-14, maxit=20000)
    assert r.status in (orc.OK, orc.MAXIT)
    got = r.p.ravel()[fluid]
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()


def test_periodic_roll_invariance(orc, F):
    """Rolling every input by s cells along a periodic axis rolls p."""
    c = F.make_two_phase(12, 8, 10, surface_seed=51, velocity_seed=52, wedge=F.Wedge(),
                         bc=(P_, P_, N, N, N, D))
    r0 = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-12)
    s = 5
    roll = lambda a: np.roll(a, s, axis=2)
    r1 = orc.pcg(roll(c.rho), roll(c.mask), c.bc, c.h, roll(c.rhs), tol=1e-12)
    assert r0.status == r1.status == orc.OK
    assert np.abs(roll(r0.p) - r1.p).max() <= 1e-9 * np.abs(r0.p).max()


@pytest.mark.parametrize("bc", [(P_, P_, N, N, N, N), (N, N, P_, P_, N, D)])
def test_projection_divergence_periodic(orc, F, bc):
    """The projection identity with periodic faces: the shared face is
    corrected once and its repeat copied, and D u_new / ||D u|| is the
    relative residual."""
    c = F.make_two_phase(14, 12, 10, surface_seed=61, velocity_seed=62,
                         wedge=F.Wedge(), bc=bc)
    assert np.array_equal(c.u[:, :, 0], c.u[:, :, -1]) or bc[0] != P_
    tol = 1e-10
    r = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=tol)
    assert r.status == orc.OK
    div0 = orc.divergence(c.u, c.v, c.w, c.h)
    u, v, w = orc.project(c.rho, c.mask, c.bc, c.h, c.dt, r.p, c.u, c.v, c.w)
    if bc[0] == P_:
        assert np.array_equal(u[:, :, 0], u[:, :, -1])
    if bc[2] == P_:
        assert np.array_equal(v[:, 0, :], v[:, -1, :])
    div1 = orc.divergence(u, v, w, c.h)
    ratio = np.linalg.norm(div1) / np.linalg.norm(div0)
    assert ratio <= tol * 1.01


# --------------------------------------------------------------------------
# free-slip cut cells: area and volume fractions (Section 2.2.1)
# --------------------------------------------------------------------------

def _ones_frac(nx, ny, nz):
    return (np.ones((nz, ny, nx + 1)), np.ones((nz, ny + 1, nx)),
            np.ones((nz + 1, ny, nx)), np.ones((nz, ny, nx)))


def test_fractions_of_one_are_the_binary_form(orc, F):
    """Fractions of one give the binary operator (to the rounding of the
    reference's threaded dot products, which are not bit-reproducible)."""
    c = _two_phase_wedge(F, 14, 12, 10, bc=TANK)
    r0 = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-10)
    r1 = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-10, frac=_ones_frac(14, 12, 10))
    assert r0.iters == r1.iters
    assert np.abs(r0.p - r1.p).max() <= 1e-13 * np.abs(r0.p).max()
    Lp0 = orc.apply(c.rho, c.mask, c.bc, c.h, r0.p)
    Lp1 = orc.apply(c.rho, c.mask, c.bc, c.h, r0.p, frac=_ones_frac(14, 12, 10))
    assert np.array_equal(Lp0, Lp1)


@pytest.mark.parametrize("alpha", [0.25, 0.8])
def test_eigvec_anisotropic_area(orc, alpha):
    """Every z face (walls included) open to the fraction alpha: the operator
    is Lx + Ly + alpha Lz, so the all-Dirichlet sine product stays an exact
    eigenvector with eigenvalue lx + ly + alpha lz."""
    nx, ny, nz = 10, 8, 12
    h, x, y, z = _grid(nx, ny, nz)
    Lx, Ly, Lz = nx * h, ny * h, nz * h
    v = np.sin(math.pi * x / Lx) * np.sin(2 * math.pi * y / Ly) * np.sin(math.pi * z / Lz)
    l1 = lambda m, L: 2 * (1 - math.cos(m * math.pi * h / L)) / h**2
    lam = l1(1, Lx) + l1(2, Ly) + alpha * l1(1, Lz)
    ax, ay, az, vol = _ones_frac(nx, ny, nz)
    az = az * alpha
    rho = np.ones((nz, ny, nx))
    mask = np.zeros((nz, ny, nx), np.uint8)
    Lv = orc.apply(rho, mask, ALL_D, h, v, frac=(ax, ay, az, vol))
    assert np.abs(Lv + lam * v).max() <= 1e-10 * lam
    r = orc.pcg(rho, mask, ALL_D, h, -lam * v, tol=1e-13, frac=(ax, ay, az, vol))
    assert r.status == orc.OK and np.abs(r.p - v).max() <= 1e-9


def test_uniform_volume_scales_the_answer(orc, F):
    """V = v everywhere divides the operator by v, so p = v p(V = 1)."""
    c = _two_phase_wedge(F, 12, 10, 9, bc=TANK)
    ax, ay, az, vol = _ones_frac(12, 10, 9)
    r0 = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-12)
    r1 = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-12, frac=(ax, ay, az, 0.37 * vol))
    assert np.abs(r1.p - 0.37 * r0.p).max() <= 1e-9 * np.abs(r0.p).max()


def _random_frac(rng, mask):
    nz, ny, nx = mask.shape
    ax = rng.uniform(0.05, 1.0, (nz, ny, nx + 1))
    ay = rng.uniform(0.05, 1.0, (nz, ny + 1, nx))
    az = rng.uniform(0.05, 1.0, (nz + 1, ny, nx))
    vol = rng.uniform(0.1, 1.0, (nz, ny, nx))
    return ax, ay, az, vol


def test_dense_with_fractions(orc, F):
    """Against a dense solve of sum_f A_f beta_f (p_c - p_n) = -h^2 V Sigma
    assembled here face by face."""
    nx, ny, nz = 7, 6, 8
    c = F.make_two_phase(nx, ny, nz, surface_seed=91, velocity_seed=92, wedge=F.Wedge(),
                         bc=(D, N, N, D, N, D))
    rng = np.random.default_rng(93)
    ax, ay, az, vol = _random_frac(rng, c.mask)
    n = nx * ny * nz
    A = np.zeros((n, n))
    idx = lambda i, j, k: (k * ny + j) * nx + i
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                ci = idx(i, j, k)
                if c.mask[k, j, i]:
                    A[ci, ci] = 1.0
                    continue
                faces = [(-1, 0, 0, ax[k, j, i]), (1, 0, 0, ax[k, j, i + 1]),
                         (0, -1, 0, ay[k, j, i]), (0, 1, 0, ay[k, j + 1, i]),
                         (0, 0, -1, az[k, j, i]), (0, 0, 1, az[k + 1, j, i])]
                for f, (di, dj, dk, a) in enumerate(faces):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                        if c.mask[kk, jj, ii]:
                            continue
                        b = a * 2.0 / (c.rho[k, j, i] + c.rho[kk, jj, ii])
                        A[ci, ci] += b
                        A[ci, idx(ii, jj, kk)] -= b
                    elif c.bc[f] == D:
                        A[ci, ci] += a * 2.0 / c.rho[k, j, i]
    b = (-c.h**2 * vol * c.rhs * (c.mask == 0)).ravel()
    want = np.linalg.solve(A, b)
    r = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-14, maxit=5000,
                frac=(ax, ay, az, vol))
    assert r.status in (orc.OK, orc.MAXIT)
    assert np.abs(r.p.ravel() - want).max() <= 1e-10 * np.abs(want).max()
    # symmetric positive definite on the fluid block
    fl = (c.mask == 0).ravel()
    Af = A[np.ix_(fl, fl)]
    assert np.abs(Af - Af.T).max() <= 1e-14 * np.abs(Af).max()
    assert np.linalg.eigvalsh(Af).min() > 0.0


def test_projection_divergence_with_fractions(orc, F):
    """Cut-cell wedge: the volume-weighted area divergence of the projected
    velocity, relative to that of the input, is the relative residual."""
    c = F.make_two_phase(24, 20, 18, surface_seed=95, velocity_seed=96, wedge=F.Wedge(),
                         bc=TANK, fractions=True)
    ax, ay, az, vol = c.frac
    assert ((vol > 0) & (vol < 1)).sum() > 50
    tol = 1e-10
    r = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=tol, frac=c.frac)
    assert r.status == orc.OK
    d0 = vol * orc.divergence(c.u, c.v, c.w, c.h, frac=c.frac)
    u, v, w = orc.project(c.rho, c.mask, c.bc, c.h, c.dt, r.p, c.u, c.v, c.w)
    d1 = vol * orc.divergence(u, v, w, c.h, frac=c.frac)
    fl = c.mask == 0
    ratio = np.linalg.norm(d1[fl]) / np.linalg.norm(d0[fl])
    assert ratio <= tol * 1.01
    assert abs(ratio - r.relres) <= 1e-6 * r.relres
    # the source is the generator's area divergence
    np.testing.assert_allclose(orc.source(c.u, c.v, c.w, c.h, c.dt, c.mask, frac=c.frac),
                               c.rhs, rtol=1e-12, atol=1e-12 * np.abs(c.rhs).max())


# --------------------------------------------------------------------------
# the residual checker (relres): Eq. (pois) residual, volume-weighted for cut
# cells (Section 2.2.1), mean-free source for singular problems
# --------------------------------------------------------------------------

def test_relres_of_zero_pressure_is_one(orc, F):
    """p = 0 leaves the whole source as residual, with or without fractions,
    in anchored and singular problems alike."""
    rng = np.random.default_rng(41)
    for bc in (TANK, (2, 2, N, N, N, N)):
        c = _two_phase_wedge(F, 12, 10, 9, bc=bc)
        z = np.zeros_like(c.rho)
        assert orc.relres(c.rho, c.mask, c.bc, c.h, c.rhs, z) == 1.0
        fr = _random_frac(rng, c.mask)
        assert orc.relres(c.rho, c.mask, c.bc, c.h, c.rhs, z, frac=fr) == 1.0


@pytest.mark.parametrize("case", _gold_cases(), ids=lambda c: c["name"])
def test_relres_of_hand_solutions(orc, case):
    """The hand-solved answers leave no residual (to the rounding of their
    decimal digits)."""
    shp = (case["nz"], case["ny"], case["nx"])
    rho = np.array(case["rho"], float).reshape(shp)
    mask = np.array(case["mask"], np.uint8).reshape(shp)
    rhs = np.array(case["rhs"], float).reshape(shp)
    want = np.array(case["p"], float).reshape(shp)
    assert orc.relres(rho, mask, case["bc"], case["h"], rhs, want) <= 1e-14
    assert orc.relres(rho, mask, case["bc"], case["h"], rhs, 0.5 * want) > 0.1


def test_relres_cut_cells_by_hand(orc):
    """A two-cell water column (rho = 1, h = 1, p = 0 on top, Neumann
    elsewhere), lower cell of volume fraction 1/2, all faces open.  For
    p = (1, 0) the finite-volume rows give sum_f A beta (p_c - p_n) = (1, -1),
    so L p = -(1, -1) / V = (-2, 1).  With Sigma = (2, 4) the weighted
    residual V (Sigma - L p) is (0.5 * 4, 1 * 3) = (2, 3) against the
    weighted source V Sigma = (1, 4): relres = sqrt(13 / 17).  (Dropping V
    would give sqrt(25 / 20).)"""
    rho = np.ones((2, 1, 1))
    mask = np.zeros((2, 1, 1), np.uint8)
    frac = (np.ones((2, 1, 2)), np.ones((2, 2, 1)), np.ones((3, 1, 1)),
            np.array([0.5, 1.0]).reshape(2, 1, 1))
    rhs = np.array([2.0, 4.0]).reshape(2, 1, 1)
    p = np.array([1.0, 0.0]).reshape(2, 1, 1)
    rr = orc.relres(rho, mask, TANK, 1.0, rhs, p, frac=frac)
    assert abs(rr - math.sqrt(13.0 / 17.0)) <= 1e-15


def test_relres_singular_by_hand(orc):
    """Two cells in a row, every wall Neumann (singular: constants are in
    the null space).  L p = (p1 - p0, p0 - p1); the source (3, 1) is solved
    with its mean removed, (1, -1).  p = (0, 1) solves it exactly; p = (0, 2)
    leaves (-1, 1), as large as the mean-free source; p = 0 leaves all of
    it.  (Keeping the mean would give sqrt(8 / 10) for p = (0, 1).)"""
    rho = np.ones((1, 1, 2))
    mask = np.zeros((1, 1, 2), np.uint8)
    bc = (N, N, N, N, N, N)
    rhs = np.array([3.0, 1.0]).reshape(1, 1, 2)
    pv = lambda a, b: np.array([a, b], float).reshape(1, 1, 2)
    assert orc.relres(rho, mask, bc, 1.0, rhs, pv(0, 1)) == 0.0
    assert orc.relres(rho, mask, bc, 1.0, rhs, pv(0, 2)) == 1.0
    assert orc.relres(rho, mask, bc, 1.0, rhs, pv(0, 0)) == 1.0
    assert orc.relres(rho, mask, bc, 1.0, rhs, pv(5, 6)) == 0.0


@pytest.mark.parametrize("bc", [TANK, (2, 2, N, N, N, N)], ids=["anchored", "singular"])
def test_relres_ignores_hull_entries(orc, F, bc):
    """Whatever a caller holds in hull cells, of the source or of the
    pressure, does not change the residual (to the rounding of the threaded
    sums, whose order is not fixed)."""
    c = _two_phase_wedge(F, 16, 12, 10, bc=bc)
    hull = c.mask == 1
    assert hull.sum() > 10
    rng = np.random.default_rng(43)
    p = rng.standard_normal(c.shape) * (c.mask == 0)
    r0 = orc.relres(c.rho, c.mask, c.bc, c.h, c.rhs, p)
    rhs_g, p_g = c.rhs.copy(), p.copy()
    rhs_g[hull] = 1e6 * rng.standard_normal(hull.sum())
    p_g[hull] = 1e6 * rng.standard_normal(hull.sum())
    assert abs(orc.relres(c.rho, c.mask, c.bc, c.h, rhs_g, p_g) - r0) <= 1e-13 * r0


def test_relres_is_the_weighted_residual(orc, F):
    """Against the norms written out here from the (separately pinned)
    operator: ||V (Sigma - L p)|| / ||V Sigma|| over fluid cells, for a
    random p on a hull with random fractions."""
    c = _two_phase_wedge(F, 14, 11, 9, bc=TANK)
    rng = np.random.default_rng(44)
    fr = _random_frac(rng, c.mask)
    vol = fr[3]
    fl = c.mask == 0
    for frac, v in ((None, np.ones_like(vol)), (fr, vol)):
        p = 1e-3 * rng.standard_normal(c.shape)
        Lp = orc.apply(c.rho, c.mask, c.bc, c.h, p, frac=frac)
        want = (np.linalg.norm((v * (c.rhs - Lp))[fl])
                / np.linalg.norm((v * c.rhs)[fl]))
        got = orc.relres(c.rho, c.mask, c.bc, c.h, c.rhs, p, frac=frac)
        assert abs(got - want) <= 1e-12 * want


@pytest.mark.parametrize("bc,with_frac", [(TANK, False), (TANK, True),
                                          ((2, 2, N, N, N, N), False),
                                          ((2, 2, N, N, N, N), True)])
def test_relres_matches_what_pcg_stops_on(orc, F, bc, with_frac):
    """The residual of pcg's answer is the one pcg reports (the scaled
    system's, recomputed at exit), in anchored and singular problems, with
    and without fractions."""
    c = _two_phase_wedge(F, 15, 12, 11, bc=bc)
    frac = _random_frac(np.random.default_rng(45), c.mask) if with_frac else None
    for tol in (1e-6, 1e-9):
        r = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=tol, frac=frac)
        assert r.status == orc.OK
        rr = orc.relres(c.rho, c.mask, c.bc, c.h, c.rhs, r.p, frac=frac)
        assert rr <= tol
        assert abs(rr - r.relres) <= 1e-5 * r.relres


def test_relres_singular_source_mean(orc, F):
    """In a singular problem the residual is blind to a constant added to
    the source (its mean is removed) and to a constant added to the
    pressure (the null vector); in an anchored problem it is not."""
    for bc, singular in (((2, 2, N, N, N, N), True), (TANK, False)):
        c = _two_phase_wedge(F, 13, 12, 10, bc=bc)
        fl = c.mask == 0
        r = orc.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-9)
        assert r.status == orc.OK
        r0 = orc.relres(c.rho, c.mask, c.bc, c.h, c.rhs, r.p)
        shift = 0.3 * np.abs(c.rhs).max()
        r1 = orc.relres(c.rho, c.mask, c.bc, c.h, c.rhs + shift * fl, r.p)
        p_shift = r.p + 0.1 * np.abs(r.p).max() * fl
        r2 = orc.relres(c.rho, c.mask, c.bc, c.h, c.rhs, p_shift)
        if singular:
            assert abs(r1 - r0) <= 1e-4 * r0 and abs(r2 - r0) <= 1e-4 * r0
        else:
            assert r1 > 1e3 * r0 and r2 > 1e3 * r0
