"""The two-stage Runge-Kutta pressure pair (Section 2.1) on the GPU: the
source and face-update kernels against the reference's, the in-place
coefficient rebuild against a fresh set-up, per-call warm starts, and the
whole pair against the reference's pair (GPU)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TANK = (0, 0, 0, 0, 0, 1)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def _t(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _case(F, shape, bc=TANK, shift=0.5, seeds=(41, 42)):
    nx, ny, nz = shape
    c = F.make_two_phase(nx, ny, nz, surface_seed=seeds[0], velocity_seed=seeds[1],
                         wedge=F.Wedge(), bc=bc)
    rho_s = F.stage_density(nx, ny, nz, surface_seed=seeds[0], velocity_seed=seeds[1],
                            phase_shift=shift)
    return c, rho_s


@pytest.mark.parametrize("shape,bc", [((37, 29, 26), TANK), ((20, 33, 17), (1, 0, 0, 1, 0, 1))])
def test_source_kernel(orc, F, torch_dev, shape, bc):
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Solver
    c, _ = _case(F, shape, bc)
    t = lambda a: _t(torch, dev, a)
    s = Solver(t(c.rho), t(c.mask), c.bc, c.h)
    u, v, w = t(c.u), t(c.v), t(c.w)
    r1 = s.rhs(c.dt, u, v, w).cpu().numpy()
    want1 = orc.source(c.u, c.v, c.w, c.h, c.dt, c.mask)
    scale = np.abs(want1).max()
    assert np.abs(r1 - want1).max() <= 1e-15 * scale
    assert np.all(r1[c.mask == 1] == 0.0)
    # the generator's source is the same definition
    assert np.abs(r1 - c.rhs).max() <= 1e-15 * scale
    # two velocity fields summed face by face
    rng = np.random.default_rng(5)
    u2, v2, w2 = (rng.uniform(-1, 1, a.shape) for a in (c.u, c.v, c.w))
    r2 = s.rhs(c.dt, u, v, w, add=(t(u2), t(v2), t(w2))).cpu().numpy()
    want2 = orc.source(c.u + u2, c.v + v2, c.w + w2, c.h, c.dt, c.mask)
    assert np.abs(r2 - want2).max() <= 1e-15 * np.abs(want2).max()
    s.close()


@pytest.mark.parametrize("flags", [0, 4])
def test_weighted_face_update(orc, F, torch_dev, flags):
    """out = w (a + b - dt grad(p)/rho), separate output and in place."""
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Solver
    c, _ = _case(F, (34, 27, 31))
    t = lambda a: _t(torch, dev, a)
    s = Solver(t(c.rho), t(c.mask), c.bc, c.h, flags=flags)
    p, st = s.solve(t(c.rhs), tol=1e-10)
    assert st["status"] == 0
    pn = p.cpu().numpy()
    rng = np.random.default_rng(6)
    b = [rng.uniform(-1, 1, a.shape) for a in (c.u, c.v, c.w)]
    ref = orc.project(c.rho, c.mask, c.bc, c.h, c.dt, pn,
                      *(x + y for x, y in zip((c.u, c.v, c.w), b)))
    ref = [0.5 * r for r in ref]
    scale = max(np.abs(r).max() for r in ref)
    a_dev = [t(x) for x in (c.u, c.v, c.w)]
    b_dev = [t(x) for x in b]
    out = [torch.empty_like(x) for x in a_dev]
    s.project(p, c.dt, *a_dev, add=b_dev, weight=0.5, out=out)
    for got, want in zip(out, ref):
        assert np.abs(got.cpu().numpy() - want).max() <= 1e-13 * scale
    # inputs untouched when the output is separate
    for got, want in zip(a_dev, (c.u, c.v, c.w)):
        np.testing.assert_array_equal(got.cpu().numpy(), want)
    # in place over a
    s.project(p, c.dt, *a_dev, add=b_dev, weight=0.5, out=a_dev)
    for got, want in zip(a_dev, out):
        assert torch.equal(got, want)
    s.close()


def test_update_density_equals_fresh_setup(F, torch_dev):
    """A rebuilt context solves exactly as one set up on the new field, also
    across a change between class coding and per-cell densities."""
    torch, dev = torch_dev
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import Solver
    c, rho_s = _case(F, (41, 30, 36))
    moll = F.make_two_phase(41, 30, 36, surface_seed=41, velocity_seed=42,
                            wedge=F.Wedge(), mollify=1.5).rho
    t = lambda a: _t(torch, dev, a)
    rhs, mask = t(c.rhs), t(c.mask)
    s = Solver(t(c.rho), mask, c.bc, c.h)
    assert s.density_classes() == 2
    for rho_new, ncls in ((rho_s, 2), (moll, 0), (c.rho, 2)):
        s.update_density(t(rho_new), mask)
        assert s.density_classes() == ncls
        p1, st1 = s.solve(rhs, tol=1e-9)
        f = Solver(t(rho_new), mask, c.bc, c.h)
        p2, st2 = f.solve(rhs, tol=1e-9)
        assert st1["status"] == 0 and st1["iters"] == st2["iters"]
        assert torch.equal(p1, p2)
        f.close()
    # a rejected field leaves no valid coefficients until a good rebuild
    bad = c.rho.copy()
    bad[3, 4, 5] = -1.0
    with pytest.raises(L.PCGError) as e:
        s.update_density(t(bad), mask)
    assert e.value.code == L.EDOMAIN
    with pytest.raises(L.PCGError) as e:
        s.solve(rhs, tol=1e-9)
    assert e.value.code == L.EINVAL
    with pytest.raises(L.PCGError) as e:
        s.rhs(c.dt, t(c.u), t(c.v), t(c.w))
    assert e.value.code == L.EINVAL
    s.update_density(t(c.rho), mask)
    p3, st3 = s.solve(rhs, tol=1e-9)
    assert st3["status"] == 0
    s.close()


def test_warm_start_per_call(F, torch_dev):
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Solver
    c, _ = _case(F, (32, 32, 32))
    t = lambda a: _t(torch, dev, a)
    s = Solver(t(c.rho), t(c.mask), c.bc, c.h)
    rhs = t(c.rhs)
    p, st0 = s.solve(rhs, tol=1e-9, warm=False)
    _, st1 = s.solve(rhs, p=p, tol=1e-9, warm=True)
    assert st1["status"] == 0 and st1["iters"] <= 1
    _, st2 = s.solve(rhs, p=p, tol=1e-9, warm=False)
    assert st2["iters"] == st0["iters"]
    s.close()


@pytest.mark.parametrize("shape,shift", [((40, 34, 30), 0.5), ((27, 45, 33), 2.0)])
def test_pressure_pair_matches_reference(orc, F, torch_dev, shape, shift):
    torch, dev = torch_dev
    from paper_1410_1942_amd import rk2
    from paper_1410_1942_amd.solver import Solver
    c, rho_s = _case(F, shape, shift=shift)
    t = lambda a: _t(torch, dev, a)
    ref = orc.rk2_pair(c.rho, rho_s, c.mask, c.bc, c.h, c.dt, c.u, c.v, c.w, tol=1e-12)
    mask = t(c.mask)
    s = Solver(t(c.rho), mask, c.bc, c.h)
    uk = [t(x) for x in (c.u, c.v, c.w)]
    tol = 1e-10
    p, un, info = rk2.pressure_pair(s, None, t(rho_s), mask, uk, c.dt, tol=tol)
    assert info["stage1"]["status"] == 0 and info["stage2"]["status"] == 0
    pn = p.cpu().numpy()
    assert np.abs(pn - ref["p_next"]).max() <= 1e-6 * np.abs(ref["p_next"]).max()
    scale = max(np.abs(r).max() for r in ref["u_next"])
    for got, want in zip(un, ref["u_next"]):
        assert np.abs(got.cpu().numpy() - want).max() <= 1e-6 * scale
    # u^{k} untouched; u^{k+1} solenoidal to the second solve's residual
    for got, want in zip(uk, (c.u, c.v, c.w)):
        np.testing.assert_array_equal(got.cpu().numpy(), want)
    d0, _ = s.divergence(*uk)
    d1, _ = s.divergence(*un)
    assert d1 <= 10 * tol * d0
    s.close()
