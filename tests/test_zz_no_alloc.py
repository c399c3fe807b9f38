"""The allocation-free entry point (pcg_solve_static) against the existing
one (pcg_setup + pcg_solve on a caller workspace), through the C ABI: calls
in a row on the library's fixed device array, each on a smaller grid than
the one before (plane tiles with one sweep per iteration on rows that leave
the last tile partly empty, on rows of whole tiles, narrow plane tiles of
one cell a thread on rows of an odd length, and wide plane tiles again),
each equal to the
workspace path's result (the same kernels in the same order, so bit for
bit) and within tolerance by the oracle's residual; and a grid too large
for the array is refused."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _to(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "ir"])
def test_static_entry_point_matches_workspace_path(orc, F, precision):
    import torch
    from paper_1410_1942_amd.solver import Solver, solve_static
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    # each call smaller than the one before; each leaves its contents in the
    # array; plane tiles keep the second z of the one-sweep form in it too
    wide = 128 if precision == 0 else 256     # one tile across
    rows = 2560 // wide
    cases = [F.make_two_phase(200, 24, 30, surface_seed=51, velocity_seed=52, wedge=F.Wedge()),
             F.make_two_phase(wide, rows, 17, surface_seed=55, velocity_seed=56, wedge=F.Wedge()),
             F.make_two_phase(37, 29, 23, surface_seed=53, velocity_seed=54, wedge=F.Wedge()),
             F.make_two_phase(wide, 1024 // wide, 9, surface_seed=57, velocity_seed=58,
                              wedge=F.Wedge())]
    sizes = [c.rho.size for c in cases]
    assert sizes == sorted(sizes, reverse=True) and len(set(sizes)) == len(sizes), sizes
    forms = [(wide, 4, 1), (wide, 4, 1), (64, 4, 1), (wide, 4, 1)]
    for case, form in zip(cases, forms):
        _say(f"case static {case.shape} prec={precision}")
        rho, mask, rhs = (_to(torch, dev, a) for a in (case.rho, case.mask, case.rhs))
        out = torch.full_like(rhs, np.nan)
        p_s, st_s = solve_static(rho, mask, case.bc, case.h, rhs, p=out, tol=1e-8,
                                 precision=precision)
        s = Solver(rho, mask, case.bc, case.h, precision=precision)
        try:
            assert s.tile_form_ex() == form
            p_w, st_w = s.solve(rhs, tol=1e-8)
        finally:
            s.close()
        torch.cuda.synchronize()
        assert p_s.data_ptr() == out.data_ptr()
        assert st_s["status"] == 0 and st_w["status"] == 0, (st_s, st_w)
        assert st_s["iters"] == st_w["iters"], (st_s, st_w)
        assert torch.equal(p_s, p_w)
        pn = p_s.cpu().numpy()
        rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, pn)
        assert rr <= 1e-8, rr
        ref = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=1e-12)
        assert np.abs(pn - ref.p).max() <= 1e-6 * np.abs(ref.p).max()


def test_static_entry_point_refuses_large_grids(F):
    import torch
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import solve_static
    dev = torch.device("cuda:0")
    n = (160, 160, 160)     # about 41 B per cell: beyond the 64 MiB array
    rho = torch.ones(n, dtype=torch.float64, device=dev)
    rhs = torch.zeros(n, dtype=torch.float64, device=dev)
    with pytest.raises(L.PCGError) as e:
        solve_static(rho, None, (0, 0, 0, 0, 0, 1), 1.0 / 160, rhs, tol=1e-8)
    assert e.value.code == L.ENOMEM
    assert "static scratch" in L.last_hip_error()
