"""Seeded random grids through every tile form the library picks by itself
(wide plane tiles whole or ragged, narrow plane tiles, consecutive cells),
in FP64 and FP32+IR: each solve meets the oracle's residual at its
tolerance, and the consecutive-cell tiles (two passes, another summation
order) give the same answer to the error that tolerance allows.

Edges are drawn from 1..300 x 1..24 x 1..12 (three in ten row lengths from
whole or ragged wide tiles), walls from four families (the
tank, random Dirichlet walls, periodic x, and singular boxes with no
Dirichlet wall), with a wedge hull on grids of at least 8 cells a side in
the first two families.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = 2
FLAT_TILES = 16
N_CASES = 24


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cases():
    rng = np.random.default_rng(2026)
    out = []
    for i in range(N_CASES):
        if rng.random() < 0.3:       # rows of whole or ragged wide tiles
            nx = int(rng.choice([128, 256, 200, 160, 260, 96, 384]))
        else:
            nx = int(rng.integers(1, 301))
        ny, nz = int(rng.integers(1, 25)), int(rng.integers(1, 13))
        kind = int(rng.integers(0, 4))
        big = min(nx, ny, nz) >= 8
        if kind == 0:
            bc, wedge = (0, 0, 0, 0, 0, 1), big and bool(rng.integers(0, 2))
        elif kind == 1:
            bc = tuple(int(v) for v in rng.integers(0, 2, size=5)) + (1,)
            wedge = big and bool(rng.integers(0, 2))
        elif kind == 2:
            y = (P, P) if rng.integers(0, 2) else (0, 0)
            bc, wedge = (P, P) + y + (0, 1), False
        else:
            bc, wedge = ((P, P) if rng.integers(0, 2) else (0, 0)) + (0, 0, 0, 0), False
        out.append(((nx, ny, nz), bc, wedge, i % 2, 700 + i))
    return out


CASES = _cases()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


def _solve(torch_dev, case, precision, flags):
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Solver
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    s = Solver(t(case.rho), t(case.mask), case.bc, case.h, precision=precision, flags=flags)
    try:
        form = s.tile_form_ex()
        p, st = s.solve(t(case.rhs), tol=1e-8, raise_on_error=False)
        torch.cuda.synchronize()
    finally:
        s.close()
    return p.cpu().numpy(), st, form


def _make(F, shape, bc, wedge, seed):
    nx, ny, nz = shape
    return F.make_two_phase(nx, ny, nz, surface_seed=seed, velocity_seed=seed + 1,
                            wedge=F.Wedge() if wedge else None, bc=bc)


@pytest.mark.parametrize("shape,bc,wedge,precision,seed", CASES, ids=lambda v: str(v))
def test_random_grid_tile_forms(orc, F, torch_dev, shape, bc, wedge, precision, seed):
    case = _make(F, shape, bc, wedge, seed)
    _say(f"case random {shape} bc={bc} wedge={wedge} prec={precision}")
    p, st, form = _solve(torch_dev, case, precision, 0)
    assert st["status"] == 0, (st, form)
    rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, p)
    assert rr <= 1e-8, (rr, st, form)
    pf, stf, formf = _solve(torch_dev, case, precision, FLAT_TILES)
    assert formf == (0, 0, 2)
    assert stf["status"] == 0, stf
    scale = max(np.abs(pf).max(), 1e-300)
    assert np.abs(p - pf).max() <= 1e-6 * scale, (form, np.abs(p - pf).max() / scale)


def test_random_grids_span_the_tile_forms(F, torch_dev):
    """The seeded cases reach every form: wide plane tiles (128 or 256
    columns), narrow ones (64) and consecutive cells."""
    forms = set()
    for shape, bc, wedge, precision, seed in CASES:
        case = _make(F, shape, bc, wedge, seed)
        forms.add(_solve(torch_dev, case, precision, 0)[2][0])
    assert {64, 0} <= forms and (128 in forms or 256 in forms), forms
