"""Periodic walls and the singular no-flux problem on the GPU, against the
CPU reference, through the C ABI (GPU).

The strut case of Section 3 has no-flux walls and periodic walls along x:
one fluid region with no Dirichlet wall, whose operator is singular with
the constant as null vector.  Both sides solve for the mean-free source and
return the zero-mean solution, so the bar is the parity bar of the other
GPU tests (relative residual of the mean-free source <= tol, max error
<= 1e-6 against the reference solved to 1e-12, FP64 iteration counts within
2 %) plus a zero fluid mean.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = 2
STRUT = (P, P, 0, 0, 0, 0)
PX_TOP = (P, P, 0, 0, 0, 1)


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


def _solve(torch_dev, case, tol, precision=0, flags=0, **kw):
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Solver
    s = Solver(_to(torch, dev, case.rho), _to(torch, dev, case.mask), case.bc, case.h,
               precision=precision, flags=flags, **kw)
    p, st = s.solve(_to(torch, dev, case.rhs), tol=tol, raise_on_error=False)
    torch.cuda.synchronize()
    s.close()
    return p.cpu().numpy(), st


def _case(F, shape, bc, s1=71, s2=72, wedge=True):
    nx, ny, nz = shape
    return F.make_two_phase(nx, ny, nz, surface_seed=s1, velocity_seed=s2,
                            wedge=F.Wedge() if wedge else None, bc=bc)


CASES = [
    ((40, 34, 30), PX_TOP, True),           # periodic x, p = 0 on top
    ((33, 20, 26), STRUT, True),            # strut walls: singular
    ((17, 25, 12), (0, 0, P, P, 0, 0), True),   # periodic y, singular
    ((24, 18, 20), (0,) * 6, False),        # pure Neumann, no hull
    ((1, 16, 12), PX_TOP, False),           # one cell along the periodic axis
    ((2, 9, 7), STRUT, False),              # two cells along it
    ((21, 11, 9), (P, P, P, P, 0, 0), True),    # doubly periodic, singular
    ((4, 10, 6), STRUT, False),             # one four-cell group per row (FP32), both x edges wrap
    ((12, 1, 9), PX_TOP, False),            # a single row: y walls on both sides of every group
]


@pytest.mark.parametrize("shape,bc,wedge", CASES)
@pytest.mark.parametrize("precision,flags", [(0, 0), (0, 4), (1, 0)],
                         ids=["fp64", "fp64-density", "ir"])
def test_periodic_parity(orc, F, torch_dev, shape, bc, wedge, precision, flags):
    case = _case(F, shape, bc, wedge=wedge)
    _say(f"case periodic {shape} bc={bc} prec={precision} flags={flags}")
    tol = 1e-8
    p, st = _solve(torch_dev, case, tol, precision=precision, flags=flags)
    assert st["status"] == 0, st
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-12)
    assert ref.status == orc.OK
    rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, p)
    assert rr <= tol, (rr, st)
    assert abs(st["rel_res_true"] - rr) <= 1e-3 * rr + 1e-15
    scale = np.abs(ref.p).max()
    assert np.abs(p - ref.p).max() <= 1e-6 * scale
    fluid = case.mask == 0
    assert np.all(p[~fluid] == 0.0)
    if 1 not in bc:
        assert abs(p[fluid].mean()) <= 1e-12 * scale
    if precision == 0:
        o8 = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=tol)
        assert abs(st["iters"] - o8.iters) <= max(2, 0.02 * o8.iters), (st, o8.iters)


def test_constant_added_to_source_is_removed(orc, F, torch_dev):
    """Singular problem: a constant added to the source lies along the null
    vector and leaves the zero-mean answer unchanged."""
    case = _case(F, (30, 22, 18), STRUT)
    p0, st0 = _solve(torch_dev, case, 1e-10)
    case.rhs = case.rhs + 250.0 * (case.mask == 0)
    p1, st1 = _solve(torch_dev, case, 1e-10)
    assert st0["status"] == 0 and st1["status"] == 0
    assert np.abs(p1 - p0).max() <= 1e-7 * np.abs(p0).max()


@pytest.mark.parametrize("bc", [STRUT, PX_TOP, (0, 0, P, P, 0, 1)])
def test_periodic_projection_and_source(orc, F, torch_dev, bc):
    """Source kernel and face update on periodic axes, face by face against
    the reference; the repeated last face equals face 0."""
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Solver
    case = _case(F, (26, 20, 16), bc)
    t = lambda a: _to(torch, dev, a)
    s = Solver(t(case.rho), t(case.mask), case.bc, case.h)
    u, v, w = t(case.u), t(case.v), t(case.w)
    src = s.rhs(case.dt, u, v, w).cpu().numpy()
    want = orc.source(case.u, case.v, case.w, case.h, case.dt, case.mask)
    assert np.abs(src - want).max() <= 1e-15 * np.abs(want).max()
    assert np.abs(src - case.rhs).max() <= 1e-15 * np.abs(want).max()
    p, st = s.solve(t(case.rhs), tol=1e-10)
    assert st["status"] == 0
    d0 = s.divergence(u, v, w)
    s.project(p, case.dt, u, v, w)
    d1 = s.divergence(u, v, w)
    pn = p.cpu().numpy()
    ur, vr, wr = orc.project(case.rho, case.mask, case.bc, case.h, case.dt, pn,
                             case.u, case.v, case.w)
    scale = max(np.abs(ur).max(), np.abs(vr).max(), np.abs(wr).max())
    for got, ref in ((u, ur), (v, vr), (w, wr)):
        assert np.abs(got.cpu().numpy() - ref).max() <= 1e-13 * scale
    un, vn = u.cpu().numpy(), v.cpu().numpy()
    if bc[0] == P:
        assert np.array_equal(un[:, :, 0], un[:, :, -1])
    if bc[2] == P:
        assert np.array_equal(vn[:, 0, :], vn[:, -1, :])
    # divergence ratio = relative residual (recomputed by the oracle)
    rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, pn)
    assert rr <= 1e-10
    assert abs(d1[0] / d0[0] - rr) <= 1e-3 * rr
    s.close()


def test_singular_batch_bitwise_alone_and_mixed(F, torch_dev):
    """A singular periodic solve batched with anchored ones gives the same
    bits as alone, and so do they."""
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Batch
    cases = [_case(F, (28, 20, 18), STRUT, 81, 82), _case(F, (22, 26, 14), PX_TOP, 83, 84),
             _case(F, (30, 16, 20), (0, 0, 0, 0, 0, 1), 85, 86)]
    dev_cases = [(_to(torch, dev, c.rho), _to(torch, dev, c.mask), c.bc, c.h,
                  _to(torch, dev, c.rhs)) for c in cases]

    def run(which):
        b = Batch(256 << 20, 4, precision=0)
        outs = {}
        for i in which:
            rho, mask, bc, h, rhs = dev_cases[i]
            p = torch.empty_like(rhs)
            code, slot = b.admit(rho, mask, bc, h, rhs, p, tol=1e-9)
            assert code == 0
            outs[i] = (slot, p)
        while b.step(4):
            pass
        res = {}
        for i, (slot, p) in outs.items():
            code, st = b.poll(slot)
            assert code == 0 and st["status"] == 0, st
            res[i] = p.clone()
        b.close()
        return res

    mixed = run([0, 1, 2])
    for i in range(3):
        alone = run([i])
        assert torch.equal(alone[i], mixed[i]), i


def test_two_unanchored_regions_refused(F, torch_dev):
    """A hull wall that splits a no-flux tank leaves two singular regions."""
    torch, dev = torch_dev
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import Solver
    nx, ny, nz = 16, 10, 8
    rho = np.ones((nz, ny, nx))
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, :, 7] = 1
    with pytest.raises(L.PCGError) as e:
        Solver(_to(torch, dev, rho), _to(torch, dev, mask), (0,) * 6, 1.0 / nz)
    assert e.value.code == L.ESINGULAR
    # periodic x joins the two halves around the back: one region again
    s = Solver(_to(torch, dev, rho), _to(torch, dev, mask), STRUT, 1.0 / nz)
    s.close()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "ir"])
def test_strut_tank_parity(orc, F, torch_dev, precision):
    """The strut tank (NACA 0024 half-strut, periodic x, no-flux elsewhere)
    at 128 x 32 x 32 against the reference."""
    case = F.config_strut(128, 32, 32)
    _say(f"case strut128 prec={precision}")
    p, st = _solve(torch_dev, case, 1e-8, precision=precision)
    assert st["status"] == 0, st
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-12)
    rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, p)
    assert rr <= 1e-8
    assert np.abs(p - ref.p).max() <= 1e-6 * np.abs(ref.p).max()
    assert abs(p[case.mask == 0].mean()) <= 1e-12 * np.abs(ref.p).max()
