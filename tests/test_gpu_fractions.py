"""Free-slip cut cells (area and volume fractions, Section 2.2.1) on the GPU
against the CPU reference, through the C ABI (GPU).

Same bar as the other parity tests: the relative residual of the scaled
(volume-weighted) system recomputed by the reference <= tol, max error
<= 1e-6 against the reference solved to 1e-12, FP64 iteration counts within
2 %.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TANK = (0, 0, 0, 0, 0, 1)
P = 2


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def _to(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _case(F, shape, bc=TANK, s1=101, s2=102):
    nx, ny, nz = shape
    return F.make_two_phase(nx, ny, nz, surface_seed=s1, velocity_seed=s2,
                            wedge=F.Wedge(), bc=bc, fractions=True)


def _solver(torch_dev, case, precision=0, flags=0, with_frac=True):
    torch, dev = torch_dev
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import Solver
    t = lambda a: _to(torch, dev, a)
    s = Solver(t(case.rho), t(case.mask), case.bc, case.h, precision=precision,
               flags=flags | L.FRACTIONS)
    if with_frac:
        s.set_fractions(*(t(a) for a in case.frac))
    return s


@pytest.mark.parametrize("shape,bc", [((40, 34, 30), TANK), ((33, 20, 26), (1, 0, 0, 1, 0, 1)),
                                      ((36, 18, 24), (P, P, 0, 0, 0, 1)),
                                      ((30, 22, 18), (P, P, 0, 0, 0, 0))])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "ir"])
def test_fraction_parity(orc, F, torch_dev, shape, bc, precision):
    torch, dev = torch_dev
    case = _case(F, shape, bc)
    ax, ay, az, vol = case.frac
    assert ((vol > 0) & (vol < 1)).sum() > 30
    _say(f"case fractions {shape} bc={bc} prec={precision}")
    s = _solver(torch_dev, case, precision)
    assert s.density_classes() == 0
    tol = 1e-8
    p, st = s.solve(_to(torch, dev, case.rhs), tol=tol, raise_on_error=False)
    s.close()
    assert st["status"] == 0, st
    pn = p.cpu().numpy()
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-12, frac=case.frac)
    assert ref.status == orc.OK
    rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, pn, frac=case.frac)
    assert rr <= tol, rr
    assert abs(st["rel_res_true"] - rr) <= 1e-3 * rr + 1e-15
    scale = np.abs(ref.p).max()
    assert np.abs(pn - ref.p).max() <= 1e-6 * scale
    assert np.all(pn[case.mask == 1] == 0.0)
    if precision == 0:
        o8 = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=tol, frac=case.frac)
        assert abs(st["iters"] - o8.iters) <= max(2, 0.02 * o8.iters), (st, o8.iters)


def test_unit_fractions_equal_density_path(F, torch_dev):
    """Fractions of one give the per-cell density path's operator; the two
    kernels may fuse different products of a sum into one multiply-add, so
    the iterates agree to rounding rather than bit for bit."""
    torch, dev = torch_dev
    from paper_1410_1942_amd import _lib as L
    case = F.make_two_phase(37, 29, 26, surface_seed=103, velocity_seed=104,
                            wedge=F.Wedge(), bc=TANK)
    nx, ny, nz = 37, 29, 26
    ones = (np.ones((nz, ny, nx + 1)), np.ones((nz, ny + 1, nx)), np.ones((nz + 1, ny, nx)),
            np.ones((nz, ny, nx)))
    rhs = _to(torch, dev, case.rhs)
    case.frac = ones
    s = _solver(torch_dev, case)
    p1, st1 = s.solve(rhs, tol=1e-9)
    s.close()
    s0 = _solver(torch_dev, case, flags=L.NO_DENSITY_CLASSES, with_frac=False)
    p0, st0 = s0.solve(rhs, tol=1e-9)
    s0.close()
    assert abs(st0["iters"] - st1["iters"]) <= 1
    assert (p0 - p1).abs().max().item() <= 1e-12 * p0.abs().max().item()


def test_fraction_validation_and_clearing(F, torch_dev):
    torch, dev = torch_dev
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import Solver
    case = _case(F, (24, 20, 16))
    t = lambda a: _to(torch, dev, a)
    ax, ay, az, vol = case.frac
    s = _solver(torch_dev, case, with_frac=False)
    assert s.density_classes() == 2
    for bad in ("area", "nan", "volume"):
        a2, v2 = ax.copy(), vol.copy()
        if bad == "area":
            a2[3, 4, 5] = 1.5
        elif bad == "nan":
            a2[2, 2, 2] = np.nan
        else:
            v2[case.mask == 0] = 0.0     # a fluid cell with no volume
        with pytest.raises(L.PCGError) as e:
            s.set_fractions(t(a2), t(ay), t(az), t(v2))
        assert e.value.code == L.EDOMAIN
        assert s.density_classes() == 2   # left without fractions
    # partial sets are refused; a context without reserved room refuses too
    fake = ctypes.c_void_p(t(ax).data_ptr())
    assert s.lib.pcg_set_fractions(s._ctx, fake, None, None, None) == L.EINVAL
    # (a context with room for fractions keeps consecutive-cell tiles: the
    # plain context asks for the same form, so that the bits can match)
    plain = Solver(t(case.rho), t(case.mask), case.bc, case.h, flags=L.FLAT_TILES)
    with pytest.raises(L.PCGError) as e:
        plain.set_fractions(t(ax), t(ay), t(az), t(vol))
    assert e.value.code == L.EINVAL
    p_plain, _ = plain.solve(t(case.rhs), tol=1e-9)
    plain.close()
    # set, then clear: back to the class path and its bits
    s.set_fractions(t(ax), t(ay), t(az), t(vol))
    assert s.density_classes() == 0
    s.set_fractions()
    assert s.density_classes() == 2
    p_back, _ = s.solve(t(case.rhs), tol=1e-9)
    assert torch.equal(p_back, p_plain)
    s.close()


def test_fraction_source_divergence_projection(orc, F, torch_dev):
    """Area-weighted source and divergence against the reference, and the
    projection identity with cut cells."""
    torch, dev = torch_dev
    case = _case(F, (30, 26, 22))
    t = lambda a: _to(torch, dev, a)
    s = _solver(torch_dev, case)
    u, v, w = t(case.u), t(case.v), t(case.w)
    src = s.rhs(case.dt, u, v, w).cpu().numpy()
    want = orc.source(case.u, case.v, case.w, case.h, case.dt, case.mask, frac=case.frac)
    scale = np.abs(want).max()
    assert np.abs(src - want).max() <= 1e-14 * scale
    assert np.abs(src - case.rhs).max() <= 1e-14 * scale
    p, st = s.solve(t(case.rhs), tol=1e-10)
    assert st["status"] == 0
    d0 = s.divergence(u, v, w)
    div0 = orc.divergence(case.u, case.v, case.w, case.h, frac=case.frac)[case.mask == 0]
    assert abs(d0[0] - np.linalg.norm(div0)) <= 1e-12 * np.linalg.norm(div0)
    s.project(p, case.dt, u, v, w)
    pn = p.cpu().numpy()
    ur, vr, wr = orc.project(case.rho, case.mask, case.bc, case.h, case.dt, pn,
                             case.u, case.v, case.w)
    fs = max(np.abs(ur).max(), np.abs(vr).max(), np.abs(wr).max())
    for got, ref in ((u, ur), (v, vr), (w, wr)):
        assert np.abs(got.cpu().numpy() - ref).max() <= 1e-13 * fs
    vol = case.frac[3][case.mask == 0]
    div1 = orc.divergence(ur, vr, wr, case.h, frac=case.frac)[case.mask == 0]
    ratio = np.linalg.norm(vol * div1) / np.linalg.norm(vol * div0)
    rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, pn, frac=case.frac)
    assert rr <= 1e-10
    assert abs(ratio - rr) <= 1e-6 * rr
    s.close()
