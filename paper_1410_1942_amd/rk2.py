"""Pressure half of one two-stage Runge-Kutta step (Section 2.1).

With the remaining momentum terms R set to zero, one step takes two pressure
solves on the same grid and hull:

1. P* from div((1/rho(phi^k)) grad P*) = div(u^k)/dt          (pcg_rhs, pcg_solve_ex)
2. u* = u^k - dt (1/rho(phi^k)) grad P*                         (pcg_project_ex)
3. coefficients rebuilt for rho(phi*)                            (pcg_update_density)
4. P^{k+1} from div((1/rho(phi*)) grad P^{k+1}) = div(u* + u^k)/dt,
   warm-started from P* in the same array                        (pcg_rhs, pcg_solve_ex)
5. u^{k+1} = (u* + u^k - dt (1/rho(phi*)) grad P^{k+1}) / 2      (pcg_project_ex)

This module only orders those library calls; every step runs in the HIP
kernels behind include/pcg.h.  The volume-fraction advance that produces
phi* is not part of the package: the caller supplies rho(phi*).
"""
from __future__ import annotations

import time
from typing import Optional, Sequence

import torch

from . import _lib as L
from .solver import Solver


def _faces_like(u, v, w):
    return torch.empty_like(u), torch.empty_like(v), torch.empty_like(w)


def pressure_pair(solver: Solver, rho_k: Optional[torch.Tensor], rho_star: torch.Tensor,
                  mask: Optional[torch.Tensor], uk: Sequence[torch.Tensor], dt: float,
                  tol: float = 1e-8, maxit: int = 1000000, p: Optional[torch.Tensor] = None,
                  warm_first: bool = False, warm_second: bool = True,
                  u_out: Optional[Sequence[torch.Tensor]] = None,
                  update_flags: int = L.SKIP_CONNECTIVITY_CHECK, rhs=None,
                  timed: bool = False):
    """Run steps 1-5.  ``rho_k`` None means the solver already holds
    rho(phi^k).  ``p`` holds P* and then P^{k+1} (warm-started from P* unless
    ``warm_second`` is False); with ``warm_first`` it is also the first
    stage's initial guess (the previous step's pressure).  ``u_out`` receives
    u* and then u^{k+1} (allocated when None).  ``update_flags`` apply to both
    coefficient rebuilds; the default skips the host connectivity check
    because the hull is the one the solver was set up with.

    Returns (p, u_next, info) with the two solves' stats and, if ``timed``,
    per-step milliseconds (host clock around stream-synchronised steps)."""
    u, v, w = uk
    if p is None:
        if warm_first:
            raise ValueError("a warm first stage needs p")
        p = torch.empty(solver.shape, dtype=torch.float64, device=u.device)
    us = tuple(u_out) if u_out is not None else _faces_like(u, v, w)
    if rhs is None:
        rhs = torch.empty(solver.shape, dtype=torch.float64, device=u.device)
    ms = {}
    t = [time.perf_counter()]

    def mark(name):
        if timed:
            torch.cuda.synchronize()
            now = time.perf_counter()
            ms[name] = (now - t[0]) * 1e3
            t[0] = now

    if rho_k is not None:
        solver.update_density(rho_k, mask, update_flags)
        mark("rebuild_k")
    solver.rhs(dt, u, v, w, out=rhs)
    _, st1 = solver.solve(rhs, p=p, tol=tol, maxit=maxit, warm=warm_first)
    mark("stage1_solve")
    solver.project(p, dt, u, v, w, out=us)
    mark("stage1_project")
    solver.update_density(rho_star, mask, update_flags)
    mark("rebuild_star")
    solver.rhs(dt, *us, add=(u, v, w), out=rhs)
    _, st2 = solver.solve(rhs, p=p, tol=tol, maxit=maxit, warm=warm_second)
    mark("stage2_solve")
    solver.project(p, dt, *us, add=(u, v, w), weight=0.5, out=us)
    mark("stage2_project")
    info = {"stage1": st1, "stage2": st2}
    if timed:
        info["ms"] = ms
    return p, us, info
