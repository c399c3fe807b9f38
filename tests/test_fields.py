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
