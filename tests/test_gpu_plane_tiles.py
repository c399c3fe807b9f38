"""The 2-D plane-tile form (128 x 4 FP64 or 256 x 4 FP32 tiles, in-plane
neighbours staged in LDS) of the two passes, through the C ABI, against the
oracle.  Solves on plane tiles run one sweep per iteration by default; the
cases here ask for the two passes (PCG_TWO_SWEEPS), whose one-sweep
counterpart has a test file of its own.

Grids whose rows are a multiple of 128 cells (FP64) or 256 (the FP32 inner
solve), or leave enough of the last tile of a row busy, take this form by
default; PCG_FLAT_TILES keeps the consecutive-cell tiles.  The cases cover
ragged tile rows (ny not a multiple of 4), ragged tile columns (nx not a
multiple of the tile width), a single row, every wall kind on every
side, periodic axes (and the fall-back to consecutive-cell tiles when a
periodic y axis does not hold whole tiles), hulls, both coefficient sources,
tile heights with tails, the iterate at an iteration cap of every phase of
the deferred x update, launch-grid independence, and a batch that mixes the
two tile forms.
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


def _solve(torch_dev, case, tol=1e-8, flags=PLANE | TWO, maxit=1000000, **kw):
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Solver
    s = Solver(_to(torch, dev, case.rho), _to(torch, dev, case.mask), case.bc, case.h,
               flags=flags, **kw)
    p, st = s.solve(_to(torch, dev, case.rhs), tol=tol, maxit=maxit, raise_on_error=False)
    torch.cuda.synchronize()
    s.close()
    return p.cpu().numpy(), st


def _case(F, shape, bc, wedge=True, s1=31, s2=32):
    nx, ny, nz = shape
    return F.make_two_phase(nx, ny, nz, surface_seed=s1, velocity_seed=s2,
                            wedge=F.Wedge() if wedge else None, bc=bc)


CASES = [
    ((128, 20, 9), TANK, True),                 # one tile across, five tile rows
    ((256, 7, 5), (1, 0, 0, 1, 0, 1), False),   # ragged last tile row (7 = 4 + 3)
    ((128, 1, 6), TANK, False),                 # a single row: three of four tile rows empty
    ((384, 9, 3), (1, 1, 1, 1, 1, 1), True),    # Dirichlet everywhere, three tiles across
    ((128, 16, 12), (P, P, P, P, 0, 1), True),  # periodic x and y holding whole tiles
    ((128, 12, 10), (P, P, 0, 0, 0, 0), True),  # periodic x, no-flux: singular
    ((128, 13, 6), (0, 0, P, P, 0, 1), False),  # periodic y, 13 rows: consecutive-cell tiles
    ((200, 9, 7), TANK, True),                  # ragged last tile column (200 = 128 + 72)
    ((66, 5, 6), (1, 1, 0, 1, 0, 1), True),     # one tile, 33 of its 64 groups in the grid
]


@pytest.mark.parametrize("shape,bc,wedge", CASES, ids=lambda v: str(v))
@pytest.mark.parametrize("flags", [PLANE | TWO, PLANE | TWO | NO_CLASSES],
                         ids=["classes", "density"])
def test_plane_tile_parity(orc, F, torch_dev, shape, bc, wedge, flags):
    case = _case(F, shape, bc, wedge)
    _say(f"case plane tiles {shape} bc={bc} wedge={wedge} flags={flags}")
    p, st = _solve(torch_dev, case, flags=flags)
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
    # the consecutive-cell tiles solve the same system in another summation order
    pf, stf = _solve(torch_dev, case, flags=flags | FLAT_TILES)
    assert abs(stf["iters"] - st["iters"]) <= 1, (st, stf)
    assert np.abs(pf - p).max() <= 1e-6 * scale


CASES_IR = [
    ((256, 9, 7), TANK, True),                  # one tile across, ragged tile rows
    ((256, 8, 6), (P, P, P, P, 0, 1), False),   # periodic x and y holding whole tiles
    ((512, 5, 4), (1, 1, 1, 1, 1, 1), True),    # Dirichlet everywhere, two tiles across
    ((256, 6, 5), (P, P, 0, 0, 0, 0), True),    # periodic x, no-flux: singular
    ((256, 13, 5), (0, 0, P, P, 0, 1), False),  # periodic y, 13 rows: consecutive-cell tiles
    ((260, 7, 6), TANK, True),                  # ragged last tile column (260 = 256 + 4)
]


@pytest.mark.parametrize("shape,bc,wedge", CASES_IR, ids=lambda v: str(v))
@pytest.mark.parametrize("flags", [PLANE | TWO, PLANE | TWO | NO_CLASSES],
                         ids=["classes", "density"])
def test_plane_tile_parity_ir(orc, F, torch_dev, shape, bc, wedge, flags):
    """FP32 stencil with FP64 refinement on 256 x 4 plane tiles (four cells a
    thread): the oracle's bar, and the consecutive-cell tiles' answer."""
    case = _case(F, shape, bc, wedge)
    _say(f"case plane tiles ir {shape} bc={bc} wedge={wedge} flags={flags}")
    p, st = _solve(torch_dev, case, flags=flags, precision=1)
    assert st["status"] == 0, st
    rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, p)
    assert rr <= 1e-8, (rr, st)
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-12)
    scale = np.abs(ref.p).max()
    assert np.abs(p - ref.p).max() <= 1e-6 * scale
    assert np.all(p[case.mask.astype(bool)] == 0.0)
    pf, stf = _solve(torch_dev, case, flags=flags | FLAT_TILES, precision=1)
    assert np.abs(pf - p).max() <= 1e-6 * scale


@pytest.mark.parametrize("k", [13, 14, 15])
def test_plane_tile_capped_iterate_ir(orc, F, torch_dev, k):
    """The FP32 inner solve on plane tiles, capped at k iterations, returns
    its k-th iterate of the same system (the deferred correction flushed)."""
    case = _case(F, (256, 6, 9), TANK)
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-30, maxit=k)
    scale = np.abs(ref.p).max()
    p, st = _solve(torch_dev, case, tol=1e-30, maxit=k, precision=1)
    assert st["status"] == 1 and st["iters"] == k and st["outer_iters"] == 2, st
    assert np.abs(p - ref.p).max() <= 1e-4 * scale


@pytest.mark.parametrize("tz", [1, 3, 8])
def test_plane_tile_heights(orc, F, torch_dev, tz):
    case = _case(F, (128, 10, 11), TANK)
    _say(f"case plane tiles tz={tz}")
    p, st = _solve(torch_dev, case, tz=tz)
    assert st["status"] == 0, st
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-12)
    assert np.abs(p - ref.p).max() <= 1e-6 * np.abs(ref.p).max()


@pytest.mark.parametrize("k", [13, 14, 15, 16, 17])
def test_plane_tile_capped_iterate(orc, F, torch_dev, k):
    """Capped at k iterations the solution is the oracle's k-th PCG iterate,
    whatever k is modulo the interval of the deferred x update."""
    case = _case(F, (128, 9, 14), TANK)
    _say(f"case plane tiles capped k={k}")
    ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-30, maxit=k)
    prev = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-30, maxit=k - 1)
    scale = np.abs(ref.p).max()
    assert np.abs(ref.p - prev.p).max() > 1e-3 * scale
    p, st = _solve(torch_dev, case, tol=1e-30, maxit=k)
    assert st["status"] == 1 and st["iters"] == k, st
    assert np.abs(p - ref.p).max() <= 1e-10 * scale


def test_plane_tile_grid_independence(F, torch_dev):
    """Per-tile partial sums: the result does not depend on the launch grid,
    bit for bit, and repeats bit for bit."""
    case = _case(F, (256, 18, 13), TANK)
    _say("case plane tiles grids")
    p1, s1 = _solve(torch_dev, case, grid_blocks=8)
    p2, s2 = _solve(torch_dev, case, grid_blocks=1024)
    p3, s3 = _solve(torch_dev, case, grid_blocks=1024)
    assert s1["iters"] == s2["iters"] == s3["iters"]
    assert np.array_equal(p1, p2) and np.array_equal(p2, p3)


def test_plane_tiles_in_a_batch(F, torch_dev):
    """A batch mixing a plane-tile solve (rows of 128) with consecutive-cell
    ones gives each the result of its solo run, bit for bit."""
    import torch
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import Batch
    torch_, dev = torch_dev
    cases = [_case(F, (128, 12, 10), TANK, s1=41, s2=42),
             _case(F, (37, 29, 23), TANK, s1=43, s2=44),
             _case(F, (64, 30, 20), (1, 0, 0, 1, 0, 1), s1=45, s2=46)]

    def run(members):
        b = Batch(1 << 28, len(members), precision=L.PREC_FP64)
        try:
            outs = []
            for c in members:
                p = torch.empty(c.shape, dtype=torch.float64, device=dev)
                code, slot = b.admit(_to(torch_, dev, c.rho), _to(torch_, dev, c.mask), c.bc,
                                     c.h, _to(torch_, dev, c.rhs), p, tol=1e-8,
                                     flags=PLANE | TWO)
                assert code == L.OK, code
                outs.append((slot, p))
            while b.step(1):
                pass
            res = [(b.poll(s)[1], p.cpu().numpy()) for s, p in outs]
        finally:
            b.close()
        return res

    _say("case plane tiles in a batch")
    mixed = run(cases)
    for i, c in enumerate(cases):
        (st1, p1), = run([c])
        assert mixed[i][0]["status"] == 0 and st1["status"] == 0
        assert mixed[i][0]["iters"] == st1["iters"], i
        assert np.array_equal(mixed[i][1], p1), i


def test_tile_form_reported(F, torch_dev):
    """pcg_tile_form names the tile form each context took and its sweeps
    per iteration."""
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Solver
    t = lambda a: _to(torch, dev, a)
    for shape, bc, flags, prec, want in [
            ((128, 8, 6), TANK, PLANE, 0, (128, 4, 1)),
            ((128, 8, 6), TANK, PLANE | TWO, 0, (128, 4, 2)),
            ((256, 8, 6), TANK, PLANE, 1, (256, 4, 1)),
            ((256, 8, 6), TANK, PLANE | TWO, 1, (256, 4, 2)),
            ((128, 8, 6), TANK, PLANE | FLAT_TILES, 0, (0, 0, 2)),
            ((128, 8, 6), TANK, 0, 0, (128, 4, 1)),            # FP64: plane tiles at any size
            ((256, 8, 6), TANK, 0, 1, (256, 4, 1)),            # FP32: plane tiles at any size
            ((128, 13, 6), (0, 0, P, P, 0, 1), PLANE, 0, (0, 0, 2)),   # ragged periodic y
            ((200, 8, 6), TANK, 0, 0, (128, 4, 1)),            # ragged columns: 78% of the lanes
            ((200, 8, 6), TANK, 0, 1, (256, 4, 1)),
            ((160, 64, 32), TANK, 0, 0, (0, 0, 2)),            # FP64 with 62% of the lanes: flat
            ((160, 8, 6), TANK, 0, 0, (64, 4, 1)),             # at most 2^18 cells: narrow
            ((160, 8, 6), TANK, PLANE, 0, (128, 4, 1)),        # wide when asked for
            ((136, 8, 6), TANK, 0, 1, (256, 4, 1)),            # FP32 with 53% of the lanes
            ((120, 64, 48), TANK, 0, 1, (0, 0, 2)),            # FP32 with 47%: flat
            ((120, 8, 6), TANK, 0, 1, (64, 4, 1)),             # at most 2^18 cells: narrow
            ((130, 8, 6), (P, P, 0, 0, 0, 1), PLANE, 0, (0, 0, 2)),   # ragged periodic x
            ((97, 64, 48), TANK, PLANE, 0, (64, 4, 1)),        # odd rows: narrow at any size
            ((80, 64, 64), TANK, 0, 0, (0, 0, 2)),             # rows of pairs past 2^18: flat
            ((97, 8, 6), TANK, PLANE, 0, (64, 4, 1)),          # at most 2^18 cells: narrow
            ((80, 64, 64), TANK, NARROW, 0, (64, 4, 1)),       # narrow when asked for
            ((97, 8, 6), TANK, TWO, 0, (0, 0, 2)),             # two sweeps: no narrow tiles
            ((98, 8, 6), TANK, PLANE, 1, (64, 4, 1))]:         # FP32: rows not of quads
        case = _case(F, shape, bc, wedge=False)
        s = Solver(t(case.rho), t(case.mask), case.bc, case.h, precision=prec, flags=flags)
        try:
            assert s.tile_form_ex() == want, (shape, bc, flags, prec)
            assert s.tile_form() == want[:2]
        finally:
            s.close()
