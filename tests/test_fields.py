"""The seeded input generator: reproducibility and geometry."""
import math

import numpy as np


def test_reproducible(F):
    a = F.config1(16)
    b = F.config1(16)
    assert np.array_equal(a.rhs, b.rhs) and np.array_equal(a.rho, b.rho)
    c = F.config_wedge(24)
    d = F.config_wedge(24)
    assert np.array_equal(c.mask, d.mask) and np.array_equal(c.rhs, d.rhs)
    assert not np.array_equal(a.rhs, F.config_wedge(16).rhs)


def test_flat_surface_density(F):
    c = F.config1(32)
    assert np.all(c.rho[:16] == F.RHO_WATER)
    assert np.all(c.rho[16:] == F.RHO_AIR)
    assert not c.mask.any()
    assert c.bc == F.TANK_BC and c.h == 1.0 / 32


def test_wedge_geometry(F):
    w = F.Wedge()
    Lx = Ly = 1.0
    t = math.tan(math.radians(15))
    # points clearly inside / outside
    inside = F.wedge_psi(np.array(0.6), np.array(0.5 + 0.5 * 0.3 * t), np.array(0.8), Lx, Ly, w)
    assert inside < 0
    assert F.wedge_psi(np.array(0.6), np.array(0.5 + 1.5 * 0.3 * t), np.array(0.8), Lx, Ly, w) > 0
    assert F.wedge_psi(np.array(0.6), np.array(0.5), np.array(0.25), Lx, Ly, w) > 0   # below keel
    assert F.wedge_psi(np.array(0.29), np.array(0.5), np.array(0.8), Lx, Ly, w) > 0   # ahead of apex
    assert F.wedge_psi(np.array(0.81), np.array(0.5), np.array(0.8), Lx, Ly, w) > 0   # behind transom
    m = F.wedge_mask(64, 64, 64, 1 / 64, w)
    zc = (np.arange(64) + 0.5) / 64
    assert not m[zc < 0.3].any() and m[zc > 0.3].any()
    assert m[-1].any()        # pierces the top


def test_closed_faces_and_source(F):
    c = F.make_two_phase(20, 18, 16, surface_seed=1, velocity_seed=2,
                         wedge=F.Wedge())
    s = c.mask.astype(bool)
    assert s.any()
    assert np.all(c.rhs[s] == 0)
    assert np.all(c.u[:, :, 0] == 0) and np.all(c.u[:, :, -1] == 0)
    assert np.all(c.v[:, 0] == 0) and np.all(c.v[:, -1] == 0)
    assert np.all(c.w[0] == 0)
    assert np.any(c.w[-1] != 0)              # open top keeps its velocity
    # a face between a hull cell and a fluid cell is closed
    k, j, i = np.argwhere(s & ~np.roll(s, 1, axis=2))[0]
    assert c.u[k, j, i] == 0


def test_batch_and_stream_members(F):
    sizes = [F.batch_member(i, keep_velocity=False).shape for i in range(64)]
    flat = np.array(sizes)
    assert flat.min() >= 16 and flat.max() <= 128
    assert len(set(sizes)) > 50
    case, tol = F.served_request(3, keep_velocity=False)
    assert 24 <= min(case.shape) and max(case.shape) <= 192
    assert tol in (1e-6, 1e-8)
    t = F.arrival_times(100, rate=10.0)
    assert np.all(np.diff(t) > 0) and 5 < t[-1] < 20


def test_strut_layout():
    """The strut tank: NACA 0024 half-section through the whole depth,
    periodic x, no-flux elsewhere, surface about z = 0.8, the paper's
    spacing 1/128 on 512 x 128 x 128 cells."""
    from paper_1410_1942_amd import fields as F
    # four-digit thickness polynomial: zero at the leading edge, about t/2
    # at 30 % chord, a small open trailing edge
    assert F.naca4_half_thickness(0.0, 0.24) == 0.0
    assert abs(F.naca4_half_thickness(0.3, 0.24) - 0.12) < 2e-3
    assert 0.0 < F.naca4_half_thickness(1.0, 0.24) < 0.01
    c = F.config_strut(128, 32, 32)
    assert c.h == 1 / 32 and c.bc == F.STRUT_BC
    for a in (c.rho, c.mask, c.rhs, c.u, c.v, c.w):
        assert a.flags["C_CONTIGUOUS"]
    assert (c.mask == c.mask[0]).all()                 # vertical, surface piercing
    xc = (np.arange(128) + 0.5) * c.h
    for s in (0.1, 0.3, 0.7):
        i = int(np.argmin(np.abs((3.6275 - xc) - s)))
        width = c.mask[0, :, i].sum() * c.h              # solid cells from y = 0
        want = F.naca4_half_thickness(3.6275 - xc[i], 0.24)
        assert abs(width - want) <= c.h, (s, width, want)
    assert not c.mask[:, :, xc > 3.6275 + c.h].any() and not c.mask[:, :, xc < 2.6275 - c.h].any()
    # water below the mean level 0.8 away from the surface, air above
    assert (c.rho[int(0.5 / c.h)] == F.RHO_WATER).all()
    assert (c.rho[int(0.95 / c.h)] == F.RHO_AIR).all()
    # periodic faces consistent; no flux through the other walls
    assert np.array_equal(c.u[:, :, 0], c.u[:, :, -1])
    assert not c.v[:, 0].any() and not c.v[:, -1].any()
    assert not c.w[0].any() and not c.w[-1].any()
    # compatible: the source sums to zero over the fluid
    fl = c.mask == 0
    assert abs(c.rhs[fl].sum()) <= 1e-9 * np.abs(c.rhs[fl]).sum()
    full = F.config_strut(keep_velocity=False)
    assert full.ncells == 8388608 and full.h == 0.0078125


def test_wedge_fractions():
    """Sampled cut-cell fractions of the wedge: the solid volume sum(1 - V) h^3
    matches the prism's closed form (triangle of side 0.5 Lx and half-angle
    15 degrees, from the keel at 0.3 to the top), fractions lie in [0, 1],
    partial values only near the surface, and faces of empty cells closed."""
    import math
    from paper_1410_1942_amd import fields as F
    n = 48
    h = 1.0 / n
    ax, ay, az, vol = F.wedge_fractions(n, n, n, h, F.Wedge())
    want = 0.5**2 * math.tan(math.radians(15.0)) * 0.7
    got = (1.0 - vol).sum() * h**3
    assert abs(got - want) <= 0.01 * want, (got, want)
    for a in (ax, ay, az, vol):
        assert a.min() >= 0.0 and a.max() <= 1.0
    cut = (vol > 0) & (vol < 1)
    assert cut.sum() > 100
    xc, yc, zc = F.cell_centres(n, n, n, h)
    psi = F.wedge_psi(xc[None, None, :], yc[None, :, None], zc[:, None, None], 1.0, 1.0, F.Wedge())
    assert np.all(np.abs(np.broadcast_to(psi, vol.shape)[cut]) < 0.87 * h)
    solid = vol == 0
    assert not ax[:, :, 1:][solid].any() and not ax[:, :, :-1][solid].any()
    assert not az[1:][solid].any() and not az[:-1][solid].any()
    c = F.make_two_phase(24, 20, 18, surface_seed=1, velocity_seed=2, wedge=F.Wedge(),
                         fractions=True)
    assert np.array_equal(c.mask, (c.frac[3] == 0).astype(np.uint8))
    assert not c.u[c.frac[0] == 0].any()
