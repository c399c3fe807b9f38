"""Seeded synthetic inputs for the pressure-projection solve.

This module only draws and lays out inputs: a density field, a hull mask, the
six boundary kinds, face velocities and the source term they imply.  It holds
none of the solver's arithmetic (no face coefficients, no operator, no Krylov
step), so the plain CPU reference and the HIP path can both consume it without
sharing code.

Layout everywhere: cell arrays are C-ordered ``[nz, ny, nx]`` (x fastest, flat
index ``(k*ny + j)*nx + i``); face velocities are ``u[nz, ny, nx+1]``,
``v[nz, ny+1, nx]``, ``w[nz+1, ny, nx]``.  The grid is uniform with spacing
``h = 1/nz`` so the vertical extent is always 1 (mean surface at 0.5, keel at
0.3) and ``Lx = nx*h``, ``Ly = ny*h``.

Physical content follows Section 2 of the paper:
* density ``rho(phi) = lambda + (1-lambda) H(phi)`` (Eq. density) with a sharp
  step H sampled at cell centres: water (1000) below the free surface, air
  (1.2) above, a tie going to air.  A mollified step is available as an option.
* the hull enters through a signed distance psi (positive outside, negative
  inside, Section 2.2); here psi is the analytic distance to a vertical-sided
  wedge, and a cell is solid when psi at its centre is negative.
* the source of the pressure equation is the divergence of ``u/dt`` (first
  RK2 stage of Section 2.1 with the remaining terms R set to zero).  Face
  velocities are uniform random in [-1, 1] and zero on every face that carries
  no flux: a Neumann wall, or a face touching a solid cell.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

# Boundary kinds, in the order x-, x+, y-, y+, z-, z+ (same values as the C ABI).
NEUMANN = 0
DIRICHLET = 1
PERIODIC = 2

RHO_WATER = 1000.0
RHO_AIR = 1.2

# Neumann on five walls and p = 0 on the top face.
TANK_BC = (NEUMANN, NEUMANN, NEUMANN, NEUMANN, NEUMANN, DIRICHLET)


@dataclasses.dataclass
class Wedge:
    """Vertical-sided wedge piercing the surface: apex at (ax*Lx, 0.5*Ly),
    opening toward +x up to x = back*Lx, half-angle ``half_angle_deg``,
    keel at z = 0.5 - draft, sides reaching the top of the domain."""
    ax: float = 0.3
    back: float = 0.8
    half_angle_deg: float = 15.0
    draft: float = 0.2


@dataclasses.dataclass
class Case:
    nx: int
    ny: int
    nz: int
    h: float
    rho: np.ndarray          # f64 [nz, ny, nx]
    mask: np.ndarray         # u8 [nz, ny, nx], 1 = solid (hull) cell
    bc: tuple                # 6 boundary kinds
    dt: float
    u: Optional[np.ndarray]  # f64 [nz, ny, nx+1]
    v: Optional[np.ndarray]  # f64 [nz, ny+1, nx]
    w: Optional[np.ndarray]  # f64 [nz+1, ny, nx]
    rhs: np.ndarray          # f64 [nz, ny, nx]; the source Sigma
    name: str = ""
    seed: int = 0
    # free-slip cut cells: (ax u-shaped, ay v-shaped, az w-shaped, vol cell)
    frac: Optional[tuple] = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def cell_centres(nx: int, ny: int, nz: int, h: float):
    """1-D coordinates of cell centres along x, y, z."""
    return ((np.arange(nx) + 0.5) * h, (np.arange(ny) + 0.5) * h,
            (np.arange(nz) + 0.5) * h)


def surface_modes(rng: np.random.Generator, nmodes: int = 8, kmin: int = 2,
                  kmax: int = 16):
    """Draw (kx, ky, theta) for ``nmodes`` cosine modes: kx, ky uniform
    integers in [kmin, kmax], a random sign on ky, phase uniform in [0, 2pi)."""
    kx = rng.integers(kmin, kmax + 1, size=nmodes)
    ky = rng.integers(kmin, kmax + 1, size=nmodes)
    sgn = np.where(rng.random(nmodes) < 0.5, -1, 1)
    theta = rng.random(nmodes) * 2.0 * math.pi
    return kx.astype(np.float64), (ky * sgn).astype(np.float64), theta


def surface_elevation(xc, yc, Lx, Ly, modes, amp=0.01, mean=0.5):
    """eta(x, y) = mean + sum_m amp*cos(2pi(kx x/Lx + ky y/Ly) + theta) on the
    (ny, nx) grid of column centres."""
    eta = np.full((yc.size, xc.size), mean, dtype=np.float64)
    if modes is None:
        return eta
    X = xc[None, :] / Lx
    Y = yc[:, None] / Ly
    for kx, ky, th in zip(*modes):
        eta += amp * np.cos(2.0 * math.pi * (kx * X + ky * Y) + th)
    return eta


def wedge_psi(x, y, z, Lx, Ly, wedge: Wedge):
    """Signed distance-like function of the wedge (negative inside): the max
    of the signed distances to its four bounding half-spaces, which has the
    exact sign of the true distance."""
    t = math.radians(wedge.half_angle_deg)
    xa = wedge.ax * Lx
    yc = 0.5 * Ly
    c, s = math.cos(t), math.sin(t)
    d1 = ((y - yc) * c - (x - xa) * s)          # + side
    d2 = (-(y - yc) * c - (x - xa) * s)         # - side
    d3 = x - wedge.back * Lx                    # flat back (transom)
    d4 = (0.5 - wedge.draft) - z                # keel plane
    return np.maximum(np.maximum(d1, d2), np.maximum(d3, d4))


def wedge_mask(nx, ny, nz, h, wedge: Wedge):
    xc, yc, zc = cell_centres(nx, ny, nz, h)
    psi = wedge_psi(xc[None, None, :], yc[None, :, None], zc[:, None, None],
                    nx * h, ny * h, wedge)
    return (psi < 0.0).astype(np.uint8)


def _sampled_fraction(psi, centres, spans, near, sub):
    """Fraction of sub x ... sub sample points with psi >= 0 (outside the
    body) around each centre, over the spans given per axis (0 for an axis
    the sample set does not extend along); only `near` entries are sampled,
    the others take the sign of psi at the centre."""
    x0, y0, z0 = centres
    frac = (psi(x0, y0, z0) >= 0.0).astype(np.float64)
    idx = np.nonzero(near)
    if idx[0].size == 0:
        return frac
    offs = (np.arange(sub) + 0.5) / sub - 0.5
    grids = [offs * sp if sp > 0 else np.zeros(1) for sp in spans]
    ox, oy, oz = np.meshgrid(*grids, indexing="ij")
    ox, oy, oz = ox.ravel(), oy.ravel(), oz.ravel()
    xs = np.broadcast_to(x0, near.shape)[idx][:, None] + ox[None, :]
    ys = np.broadcast_to(y0, near.shape)[idx][:, None] + oy[None, :]
    zs = np.broadcast_to(z0, near.shape)[idx][:, None] + oz[None, :]
    frac[idx] = (psi(xs, ys, zs) >= 0.0).mean(axis=1)
    return frac


def wedge_fractions(nx, ny, nz, h, wedge: Wedge, sub: int = 4):
    """Area fractions of every MAC face and volume fractions of every cell
    open to the fluid around the wedge (the finite-volume free-slip hull of
    Section 2.2.1): the share of sub^2 (faces) or sub^3 (cells) sample points
    outside the body.  Only faces and cells within reach of the surface are
    sampled (the max of the half-space distances never exceeds the true
    distance for this convex body, so larger |psi| decides by sign).  Faces
    touching a cell with no fluid are closed."""
    Lx, Ly = nx * h, ny * h
    psi = lambda x, y, z: wedge_psi(x, y, z, Lx, Ly, wedge)
    xc, yc, zc = cell_centres(nx, ny, nz, h)
    xf = np.arange(nx + 1) * h
    yf = np.arange(ny + 1) * h
    zf = np.arange(nz + 1) * h
    X, Y, Z = xc[None, None, :], yc[None, :, None], zc[:, None, None]
    r_cell, r_face = 0.87 * h, 0.71 * h
    shape_c = (nz, ny, nx)
    pc = np.broadcast_to(psi(X, Y, Z), shape_c)
    vol = _sampled_fraction(psi, (X, Y, Z), (h, h, h), np.abs(pc) < r_cell, sub)
    pu = np.broadcast_to(psi(xf[None, None, :], Y, Z), (nz, ny, nx + 1))
    ax = _sampled_fraction(psi, (xf[None, None, :], Y, Z), (0, h, h), np.abs(pu) < r_face, sub)
    pv = np.broadcast_to(psi(X, yf[None, :, None], Z), (nz, ny + 1, nx))
    ay = _sampled_fraction(psi, (X, yf[None, :, None], Z), (h, 0, h), np.abs(pv) < r_face, sub)
    pw = np.broadcast_to(psi(X, Y, zf[:, None, None]), (nz + 1, ny, nx))
    az = _sampled_fraction(psi, (X, Y, zf[:, None, None]), (h, h, 0), np.abs(pw) < r_face, sub)
    ax, ay, az, vol = (np.array(np.broadcast_to(a, sh), dtype=np.float64, order="C")
                       for a, sh in ((ax, (nz, ny, nx + 1)), (ay, (nz, ny + 1, nx)),
                                     (az, (nz + 1, ny, nx)), (vol, shape_c)))
    solid = vol == 0.0
    ax[:, :, 1:][solid] = 0.0
    ax[:, :, :-1][solid] = 0.0
    ay[:, 1:, :][solid] = 0.0
    ay[:, :-1, :][solid] = 0.0
    az[1:, :, :][solid] = 0.0
    az[:-1, :, :][solid] = 0.0
    return ax, ay, az, vol


def source_with_fractions(u, v, w, h, dt, frac):
    """Sigma = div_A(u)/dt: face velocities weighted by their area fractions,
    summed, divided by the cell's volume fraction (0 where it is 0)."""
    ax, ay, az, vol = frac
    fu, fv, fw = ax * u, ay * v, az * w
    d = ((fu[:, :, 1:] - fu[:, :, :-1]) + (fv[:, 1:, :] - fv[:, :-1, :])
         + (fw[1:, :, :] - fw[:-1, :, :]))
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.where(vol > 0.0, d / (vol * h), 0.0)
    return out / dt


def density(nx, ny, nz, h, eta, rho_w=RHO_WATER, rho_a=RHO_AIR,
            mollify: float = 0.0):
    """rho = lambda + (1-lambda) H with H the water indicator (Eq. density),
    written dimensionally: rho_a + (rho_w - rho_a) H.  ``mollify`` > 0 uses a
    smooth step of half-width ``mollify`` cells instead of the sharp one."""
    _, _, zc = cell_centres(nx, ny, nz, h)
    dist = eta[None, :, :] - zc[:, None, None]       # > 0 below the surface
    if mollify > 0.0:
        eps = mollify * h
        s = np.clip(dist / eps, -1.0, 1.0)
        H = 0.5 * (1.0 + s + np.sin(math.pi * s) / math.pi)
        return rho_a + (rho_w - rho_a) * H
    return np.where(dist > 0.0, rho_w, rho_a).astype(np.float64)


# --------------------------------------------------------------------------
# face velocities and the source term
# --------------------------------------------------------------------------

def face_velocities(rng, nx, ny, nz):
    """u, v, w iid uniform in [-1, 1], drawn in the order u, v, w."""
    u = rng.uniform(-1.0, 1.0, size=(nz, ny, nx + 1))
    v = rng.uniform(-1.0, 1.0, size=(nz, ny + 1, nx))
    w = rng.uniform(-1.0, 1.0, size=(nz + 1, ny, nx))
    return u, v, w


def close_faces(u, v, w, mask, bc):
    """Zero the normal velocity on faces that carry no flux: Neumann walls and
    every face with a solid cell on either side.  Dirichlet (open) walls keep
    their velocity.  A periodic pair of walls is one face between the last
    and the first cell of a row: face 0 holds it (closed when either cell is
    solid, or when the row has one cell) and the last face repeats it.
    In place."""
    s = mask.astype(bool)
    # x faces: interior faces 1..nx-1 touch cells i-1 and i
    u[:, :, 1:-1][s[:, :, 1:] | s[:, :, :-1]] = 0.0
    u[:, :, 0][s[:, :, 0]] = 0.0
    u[:, :, -1][s[:, :, -1]] = 0.0
    v[:, 1:-1, :][s[:, 1:, :] | s[:, :-1, :]] = 0.0
    v[:, 0, :][s[:, 0, :]] = 0.0
    v[:, -1, :][s[:, -1, :]] = 0.0
    w[1:-1, :, :][s[1:, :, :] | s[:-1, :, :]] = 0.0
    w[0, :, :][s[0, :, :]] = 0.0
    w[-1, :, :][s[-1, :, :]] = 0.0
    if bc[0] == PERIODIC:
        shut = s[:, :, 0] | s[:, :, -1] if s.shape[2] > 1 else np.ones_like(s[:, :, 0])
        u[:, :, 0][shut] = 0.0
        u[:, :, -1] = u[:, :, 0]
    if bc[2] == PERIODIC:
        shut = s[:, 0, :] | s[:, -1, :] if s.shape[1] > 1 else np.ones_like(s[:, 0, :])
        v[:, 0, :][shut] = 0.0
        v[:, -1, :] = v[:, 0, :]
    if bc[0] == NEUMANN:
        u[:, :, 0] = 0.0
    if bc[1] == NEUMANN:
        u[:, :, -1] = 0.0
    if bc[2] == NEUMANN:
        v[:, 0, :] = 0.0
    if bc[3] == NEUMANN:
        v[:, -1, :] = 0.0
    if bc[4] == NEUMANN:
        w[0, :, :] = 0.0
    if bc[5] == NEUMANN:
        w[-1, :, :] = 0.0


def source_from_velocity(u, v, w, h, dt):
    """Sigma = div(u)/dt with the face-difference divergence on the MAC grid
    (the right-hand side of the first-stage pressure equation of the RK2
    scheme, remaining terms set to zero)."""
    div = ((u[:, :, 1:] - u[:, :, :-1]) + (v[:, 1:, :] - v[:, :-1, :])
           + (w[1:, :, :] - w[:-1, :, :])) / h
    return div / dt


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def make_two_phase(nx, ny, nz, *, surface_seed: Optional[int],
                   velocity_seed: int, wedge: Optional[Wedge] = None,
                   bc: Sequence[int] = TANK_BC, dt: float = 1e-3,
                   nmodes: int = 8, amp: float = 0.01, mollify: float = 0.0,
                   keep_velocity: bool = True, name: str = "",
                   fractions: bool = False) -> Case:
    """Two-phase tank: water below eta(x, y), air above, optional wedge hull.

    ``surface_seed=None`` gives the flat surface z = 0.5.  Velocities come
    from ``numpy.random.default_rng(velocity_seed)``; surface modes from
    ``default_rng(surface_seed)`` (the same generator when both seeds match,
    modes drawn first)."""
    h = 1.0 / nz
    modes, vel_rng = _draw_modes(surface_seed, velocity_seed, nmodes)
    rho = _density_from_modes(nx, ny, nz, modes, 0.0, amp, mollify)
    frac = None
    if wedge is not None and fractions:
        frac = wedge_fractions(nx, ny, nz, h, wedge)
        mask = (frac[3] == 0.0).astype(np.uint8)
    elif wedge is not None:
        mask = wedge_mask(nx, ny, nz, h, wedge)
    else:
        mask = np.zeros((nz, ny, nx), dtype=np.uint8)
    u, v, w = face_velocities(vel_rng, nx, ny, nz)
    close_faces(u, v, w, mask, bc)
    if frac is not None:
        # no flow through fully blocked faces
        u[frac[0] == 0.0] = 0.0
        v[frac[1] == 0.0] = 0.0
        w[frac[2] == 0.0] = 0.0
        rhs = source_with_fractions(u, v, w, h, dt, frac)
    else:
        rhs = source_from_velocity(u, v, w, h, dt)
    rhs[mask.astype(bool)] = 0.0
    if not keep_velocity:
        u = v = w = None
    return Case(nx, ny, nz, h, rho, mask, tuple(int(b) for b in bc), dt,
                u, v, w, np.ascontiguousarray(rhs), name=name,
                seed=velocity_seed, frac=frac)


def _draw_modes(surface_seed, velocity_seed, nmodes):
    """Surface modes and the velocity generator, drawn as make_two_phase
    draws them (modes first when both seeds match)."""
    vel_rng = np.random.default_rng(velocity_seed)
    if surface_seed is None:
        modes = None
    elif surface_seed == velocity_seed:
        modes = surface_modes(vel_rng, nmodes)
    else:
        modes = surface_modes(np.random.default_rng(surface_seed), nmodes)
    return modes, vel_rng


def _density_from_modes(nx, ny, nz, modes, phase_shift, amp, mollify):
    h = 1.0 / nz
    xc, yc, _ = cell_centres(nx, ny, nz, h)
    if modes is not None and phase_shift:
        kx, ky, th = modes
        modes = (kx, ky, th + phase_shift)
    eta = surface_elevation(xc, yc, nx * h, ny * h, modes, amp=amp)
    return density(nx, ny, nz, h, eta, mollify=mollify)


def stage_density(nx, ny, nz, *, surface_seed: Optional[int], velocity_seed: int,
                  phase_shift: float, nmodes: int = 8, amp: float = 0.01,
                  mollify: float = 0.0) -> np.ndarray:
    """Density of the surface moved for the second Runge-Kutta stage: the
    modes of make_two_phase with the same seeds, every phase advanced by
    ``phase_shift`` radians (a stand-in for the volume-fraction advance,
    which is not part of this package).  ``phase_shift = 0`` returns
    make_two_phase's density."""
    modes, _ = _draw_modes(surface_seed, velocity_seed, nmodes)
    return _density_from_modes(nx, ny, nz, modes, phase_shift, amp, mollify)


def naca4_half_thickness(s, t: float):
    """Half-thickness of a NACA four-digit symmetric section at chord
    fraction s in [0, 1] for thickness ratio t (the published four-digit
    thickness polynomial, chord 1)."""
    s = np.clip(s, 0.0, 1.0)
    return 5.0 * t * (0.2969 * np.sqrt(s) - 0.1260 * s - 0.3516 * s**2
                      + 0.2843 * s**3 - 0.1015 * s**4)


def strut_mask(nx, ny, nz, h, le_x: float, chord: float = 1.0, t: float = 0.24):
    """Surface-piercing vertical strut of NACA section 00(100 t): the half on
    y >= 0 of a section whose leading edge is at x = le_x and trailing edge
    at le_x - chord, through the whole depth (the y = 0 wall is its
    centreplane).  A cell is solid when its centre lies inside."""
    xc, yc, _ = cell_centres(nx, ny, nz, h)
    s = (le_x - xc) / chord
    inside = (s >= 0.0) & (s <= 1.0)
    half = np.where(inside, chord * naca4_half_thickness(s, t), -1.0)
    col = (yc[:, None] <= half[None, :])
    return np.ascontiguousarray(np.broadcast_to(col[None, :, :], (nz, ny, nx)), dtype=np.uint8)


STRUT_BC = (PERIODIC, PERIODIC, NEUMANN, NEUMANN, NEUMANN, NEUMANN)


def config_strut(nx: int = 512, ny: int = 128, nz: int = 128, surface_seed: int = 3,
                 velocity_seed: int = 4, dt: float = 1.25e-3, keep_velocity: bool = True,
                 name: str = "") -> Case:
    """Strut tank in the layout of the paper's NACA 0024 case (Section 3),
    lengths in chords: 4 long (periodic along x), 1 wide from the strut's
    centreplane, 0.8 of water under 0.2 of air (h = 1/nz, so nz = 128 gives
    the paper's spacing 1/128 on 512 x 128 x 128 cells).  No-flux walls on
    y, bottom and top, periodic x: a singular, compatible problem.  Leading
    edge at x = 3.6275 (the paper's x = 0 on its [-3.6275, 0.3725] domain),
    eight seeded surface modes of amplitude 0.01 about z = 0.8."""
    h = 1.0 / nz
    modes, vel_rng = _draw_modes(surface_seed, velocity_seed, 8)
    xc, yc, _ = cell_centres(nx, ny, nz, h)
    eta = surface_elevation(xc, yc, nx * h, ny * h, modes, amp=0.01, mean=0.8)
    rho = density(nx, ny, nz, h, eta)
    mask = strut_mask(nx, ny, nz, h, le_x=3.6275 * (nx * h) / 4.0, chord=(nx * h) / 4.0)
    u, v, w = face_velocities(vel_rng, nx, ny, nz)
    close_faces(u, v, w, mask, STRUT_BC)
    rhs = source_from_velocity(u, v, w, h, dt)
    rhs[mask.astype(bool)] = 0.0
    if not keep_velocity:
        u = v = w = None
    return Case(nx, ny, nz, h, rho, mask, STRUT_BC, dt, u, v, w, np.ascontiguousarray(rhs),
                name=name or f"strut{nx}x{ny}x{nz}", seed=velocity_seed)


def config1(n: int = 32, **kw) -> Case:
    """Plain FP64 case: n^3 cells on the unit cube, flat surface z = 0.5,
    no hull, Neumann on five walls and p = 0 on top, seed 0."""
    return make_two_phase(n, n, n, surface_seed=None, velocity_seed=0,
                          name=f"flat{n}", **kw)


def config_wedge(n: int = 256, **kw) -> Case:
    """n^3 grid, eight-mode surface (surface seed 1), wedge hull (half-angle
    15 deg, draft 0.2), velocity seed 2."""
    return make_two_phase(n, n, n, surface_seed=1, velocity_seed=2,
                          wedge=Wedge(), name=f"wedge{n}", **kw)


def log_uniform_edges(rng, lo, hi, k=3):
    """k integer edges, log-uniform in [lo, hi] then rounded."""
    e = np.exp(rng.uniform(math.log(lo), math.log(hi), size=k))
    return [int(min(hi, max(lo, round(float(x))))) for x in e]


def batch_member(i: int, lo: int = 16, hi: int = 128, **kw) -> Case:
    """Member i of the uneven batch: generator seed 1000+i draws the three
    edges (x, y, z order), then the surface modes, then the velocities.
    No hull."""
    seed = 1000 + i
    rng = np.random.default_rng(seed)
    nx, ny, nz = log_uniform_edges(rng, lo, hi)
    # the same generator continues into surface and velocities
    return _continue_two_phase(rng, nx, ny, nz, wedge=None, seed=seed,
                               name=f"batch{i}", **kw)


def served_request(i: int, lo: int = 24, hi: int = 192, **kw):
    """Request i of the served stream: generator seed 2000+i draws edges,
    then wedge presence (p = 0.5), then tolerance (1e-6 or 1e-8, p = 0.5),
    then surface and velocities.  Returns (case, tol)."""
    seed = 2000 + i
    rng = np.random.default_rng(seed)
    nx, ny, nz = log_uniform_edges(rng, lo, hi)
    has_wedge = bool(rng.random() < 0.5)
    tol = 1e-6 if rng.random() < 0.5 else 1e-8
    case = _continue_two_phase(rng, nx, ny, nz,
                               wedge=Wedge() if has_wedge else None,
                               seed=seed, name=f"req{i}", **kw)
    return case, tol


def arrival_times(n: int, rate: float, seed: int = 7) -> np.ndarray:
    """Poisson arrivals: cumulative exponential gaps with mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def _continue_two_phase(rng, nx, ny, nz, *, wedge, seed, name,
                        bc=TANK_BC, dt=1e-3, keep_velocity=True):
    h = 1.0 / nz
    xc, yc, _ = cell_centres(nx, ny, nz, h)
    modes = surface_modes(rng)
    eta = surface_elevation(xc, yc, nx * h, ny * h, modes)
    rho = density(nx, ny, nz, h, eta)
    mask = (wedge_mask(nx, ny, nz, h, wedge) if wedge is not None
            else np.zeros((nz, ny, nx), dtype=np.uint8))
    u, v, w = face_velocities(rng, nx, ny, nz)
    close_faces(u, v, w, mask, bc)
    rhs = source_from_velocity(u, v, w, h, dt)
    rhs[mask.astype(bool)] = 0.0
    if not keep_velocity:
        u = v = w = None
    return Case(nx, ny, nz, h, rho, mask, tuple(bc), dt, u, v, w,
                np.ascontiguousarray(rhs), name=name, seed=seed)


def random_vector(shape, seed):
    """Seeded uniform [-1, 1] vector (test operand)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=shape)
