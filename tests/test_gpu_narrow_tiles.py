"""Narrow plane tiles (64 x 4 cells, one cell a thread, PCG_NARROW_TILES):
the one-sweep iteration on grids whose rows the wide tiles do not take (odd
lengths, or too little of a 128- or 256-cell tile), through the C ABI,
against the oracle.

The bar is the one-sweep form's: the converged answer against the oracle's
1e-12 solution, the FP64 iteration count against the oracle's, the k-th
iterate of a capped solve against the oracle's k-th iterate, and the answer
of the consecutive-cell tiles.  The cases cover odd and ragged rows, a row
shorter than a tile, a single row, every wall kind, periodic axes holding
whole tiles (and the fall-back when they do not), hulls, both coefficient
sources, short tiles, launch-grid independence, and a batch mixing narrow,
wide and consecutive-cell members.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TANK = (0, 0, 0, 0, 0, 1)
P = 2
FLAT_TILES = 16
PLANE = 32
TWO = 64
NARROW = 128
NO_CLASSES = 4


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


def _solve(torch_dev, case, tol=1e-8, flags=NARROW, maxit=1000000, form=None, **kw):
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Solver
    s = Solver(_to(torch, dev, case.rho), _to(torch, dev, case.mask), case.bc, case.h,
               flags=flags, **kw)
    try:
        if form is not None:
            assert s.tile_form_ex() == form, (s.tile_form_ex(), form)
        p, st = s.solve(_to(torch, dev, case.rhs), tol=tol, maxit=maxit, raise_on_error=False)
        torch.cuda.synchronize()
    finally:
        s.close()
    return p.cpu().numpy(), st


def _case(F, shape, bc, wedge=True, s1=61, s2=62):
    nx, ny, nz = shape
    return F.make_two_phase(nx, ny, nz, surface_seed=s1, velocity_seed=s2,
                            wedge=F.Wedge() if wedge else None, bc=bc)


NARROW_FORM = (64, 4, 1)
FLAT_FORM = (0, 0, 2)

CASES = [
    ((37, 9, 7), TANK, True, NARROW_FORM),                 # odd rows, one tile across
    ((65, 5, 6), (1, 1, 0, 1, 0, 1), True, NARROW_FORM),   # ragged: 64 + 1 columns
    ((101, 14, 5), (1, 1, 1, 1, 1, 1), True, NARROW_FORM), # Dirichlet everywhere, two tiles
    ((33, 1, 6), TANK, False, NARROW_FORM),                # a single row
    ((64, 8, 6), (P, P, P, P, 0, 1), False, NARROW_FORM),  # periodic x and y, whole tiles
    ((64, 12, 7), (P, P, 0, 0, 0, 0), True, NARROW_FORM),  # periodic x, no-flux: singular
    ((45, 13, 6), (0, 0, P, P, 0, 1), False, FLAT_FORM),   # periodic y, 13 rows: fall-back
    ((67, 8, 5), (P, P, 0, 0, 0, 1), False, FLAT_FORM),    # ragged periodic x: fall-back
]


@pytest.mark.parametrize("shape,bc,wedge,form", CASES, ids=lambda v: str(v))
@pytest.mark.parametrize("flags", [NARROW, NARROW | NO_CLASSES], ids=["classes", "density"])
def test_narrow_parity(orc, F, torch_dev, shape, bc, wedge, form, flags):
    case = _case(F, shape, bc, wedge)
    _say(f"case narrow {shape} bc={bc} wedge={wedge} flags={flags}")
    p, st = _solve(torch_dev, case, flags=flags, form=form)
    assert st["status"] == 0, st
    rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, p)
    assert rr <= 1e-8, (rr, st)
    assert abs(st["rel_res_true"] - rr) <= 1e-3 * rr + 1e-15
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-12)
    assert ref.status == orc.OK
    scale = np.abs(ref.p).max()
    assert np.abs(p - ref.p).max() <= 1e-6 * scale
    assert np.all(p[case.mask.astype(bool)] == 0.0)
    o8 = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-8)
    assert abs(st["iters"] - o8.iters) <= max(2, 0.02 * o8.iters), (st, o8.iters)
    # the consecutive-cell tiles (two passes) solve the same system
    pf, stf = _solve(torch_dev, case, flags=(flags & NO_CLASSES) | FLAT_TILES)
    assert abs(stf["iters"] - st["iters"]) <= max(1, 0.01 * st["iters"]), (st, stf)
    assert np.abs(pf - p).max() <= 1e-6 * scale


@pytest.mark.parametrize("k", [1, 2, 3, 13, 14])
def test_narrow_capped_iterate(orc, F, torch_dev, k):
    """Capped at k iterations the solution is the oracle's k-th PCG iterate,
    whatever k is modulo the interval of the deferred x update."""
    case = _case(F, (37, 9, 14), (1, 0, 0, 1, 0, 1))
    _say(f"case narrow capped k={k}")
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-30, maxit=k)
    scale = np.abs(ref.p).max()
    p, st = _solve(torch_dev, case, tol=1e-30, maxit=k, form=NARROW_FORM)
    assert st["status"] == 1 and st["iters"] == k, st
    assert np.abs(p - ref.p).max() <= 1e-10 * scale


@pytest.mark.parametrize("tz", [1, 3])
def test_narrow_tile_heights(orc, F, torch_dev, tz):
    """Short tiles: every tile above the bottom starts one plane low."""
    case = _case(F, (45, 10, 11), TANK)
    _say(f"case narrow tz={tz}")
    p, st = _solve(torch_dev, case, tz=tz, form=NARROW_FORM)
    assert st["status"] == 0, st
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-12)
    assert np.abs(p - ref.p).max() <= 1e-6 * np.abs(ref.p).max()


def test_narrow_grid_independence(F, torch_dev):
    """The result does not depend on the launch grid, bit for bit."""
    case = _case(F, (99, 18, 13), TANK)
    _say("case narrow grids")
    p1, s1 = _solve(torch_dev, case, grid_blocks=8)
    p2, s2 = _solve(torch_dev, case, grid_blocks=1024)
    assert s1["iters"] == s2["iters"]
    assert np.array_equal(p1, p2)


CASES_IR = [
    ((37, 9, 7), TANK, True),                   # odd rows
    ((100, 7, 6), (1, 1, 1, 1, 1, 1), True),    # rows of quads filling 39 % of a wide tile
    ((64, 6, 5), (P, P, 0, 0, 0, 0), True),     # periodic x, no-flux: singular
]


@pytest.mark.parametrize("shape,bc,wedge", CASES_IR, ids=lambda v: str(v))
@pytest.mark.parametrize("flags", [NARROW, NARROW | NO_CLASSES], ids=["classes", "density"])
def test_narrow_parity_ir(orc, F, torch_dev, shape, bc, wedge, flags):
    """The FP32 inner solve of the refinement on narrow tiles: the oracle's
    bar, and the consecutive-cell tiles' answer."""
    case = _case(F, shape, bc, wedge)
    _say(f"case narrow ir {shape} bc={bc} wedge={wedge} flags={flags}")
    p, st = _solve(torch_dev, case, flags=flags, precision=1, form=NARROW_FORM)
    assert st["status"] == 0, st
    rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, p)
    assert rr <= 1e-8, (rr, st)
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-12)
    scale = np.abs(ref.p).max()
    assert np.abs(p - ref.p).max() <= 1e-6 * scale
    assert np.all(p[case.mask.astype(bool)] == 0.0)
    pf, stf = _solve(torch_dev, case, flags=(flags & NO_CLASSES) | FLAT_TILES, precision=1)
    assert np.abs(pf - p).max() <= 1e-6 * scale
    # FP32 rounding of the one-sweep recurrences differs from the two
    # passes', and so can the inner count (the bar is the answer)
    _say(f"  inner iterations: narrow {st['iters']}, consecutive tiles {stf['iters']}")
    assert abs(stf["iters"] - st["iters"]) <= max(2, 0.25 * stf["iters"]), (st, stf)


@pytest.mark.parametrize("k", [3, 14])
def test_narrow_capped_iterate_ir(orc, F, torch_dev, k):
    """The FP32 inner solve on narrow tiles, capped at k iterations, returns
    its k-th iterate."""
    case = _case(F, (37, 6, 9), TANK)
    _say(f"case narrow ir capped k={k}")
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-30, maxit=k)
    scale = np.abs(ref.p).max()
    p, st = _solve(torch_dev, case, tol=1e-30, maxit=k, precision=1, form=NARROW_FORM)
    assert st["status"] == 1 and st["iters"] == k and st["outer_iters"] == 2, st
    assert np.abs(p - ref.p).max() <= 1e-4 * scale


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "ir"])
def test_narrow_in_a_batch(F, torch_dev, precision):
    """A batch mixing narrow, wide and consecutive-cell members gives each
    the result of its solo run, bit for bit."""
    import torch
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import Batch
    torch_, dev = torch_dev
    wide = 128 if precision == 0 else 256
    members = [(_case(F, (37, 12, 10), TANK, s1=71, s2=72), NARROW),
               (_case(F, (wide, 8, 9), (1, 0, 0, 1, 0, 1), s1=73, s2=74), 0),
               (_case(F, (41, 29, 23), TANK, s1=75, s2=76), 0),
               (_case(F, (70, 10, 8), TANK, s1=77, s2=78), NARROW)]

    def run(ms):
        b = Batch(1 << 28, len(ms), precision=precision)
        try:
            outs = []
            for c, fl in ms:
                p = torch.empty(c.shape, dtype=torch.float64, device=dev)
                code, slot = b.admit(_to(torch_, dev, c.rho), _to(torch_, dev, c.mask), c.bc,
                                     c.h, _to(torch_, dev, c.rhs), p, tol=1e-8, flags=fl)
                assert code == L.OK, code
                outs.append((slot, p))
            while b.step(1):
                pass
            res = [(b.poll(s)[1], p.cpu().numpy()) for s, p in outs]
        finally:
            b.close()
        return res

    _say(f"case narrow in a batch prec={precision}")
    mixed = run(members)
    for i, m in enumerate(members):
        (st1, p1), = run([m])
        assert mixed[i][0]["status"] == 0 and st1["status"] == 0
        assert mixed[i][0]["iters"] == st1["iters"], i
        assert np.array_equal(mixed[i][1], p1), i
    # all members on narrow tiles: one launch per iteration
    narrow_only = run([(c, NARROW) for c, _ in members[2:]] + [members[0]])
    assert all(st["status"] == 0 for st, _ in narrow_only)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "ir"])
def test_narrow_large_odd_rows(orc, F, torch_dev, precision):
    """A 191^3 wedge tank (rows of an odd length take narrow tiles at any
    size): the oracle's residual of the answer, and the consecutive-cell
    tiles' answer to the error the tolerance allows."""
    case = F.make_two_phase(191, 191, 191, surface_seed=81, velocity_seed=82,
                            wedge=F.Wedge(), keep_velocity=False)
    _say(f"case narrow 191^3 prec={precision}")
    p, st = _solve(torch_dev, case, tol=1e-9, flags=0, precision=precision, form=NARROW_FORM)
    assert st["status"] == 0, st
    rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, p)
    assert rr <= 1e-9, (rr, st)
    pf, stf = _solve(torch_dev, case, tol=1e-9, flags=FLAT_TILES, precision=precision,
                     form=FLAT_FORM)
    assert stf["status"] == 0, stf
    assert np.abs(p - pf).max() <= 1e-5 * np.abs(pf).max()
    if precision == 0:
        assert abs(st["iters"] - stf["iters"]) <= max(2, 0.01 * stf["iters"]), (st, stf)
