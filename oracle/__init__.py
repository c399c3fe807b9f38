"""Plain FP64 CPU reference of the pressure-projection solve (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the bench's
CPU-baseline leg are the only callers.  The product library never imports
this package and this package never imports the product library.

All arrays are NumPy, C-ordered ``[nz, ny, nx]`` (x fastest).  Sign convention
follows Eq. (pois): ``apply`` returns ``L p = div((1/rho) grad p)`` and
``pcg`` solves ``L p = rhs``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, MAXIT = 0, 1
EINVAL, EDOMAIN, ESINGULAR, EBREAKDOWN, ENOMEM, EUNSUPPORTED = -1, -2, -3, -4, -5, -8

_lib = None


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wno-unknown-pragmas", "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def load(path: Optional[str] = None):
    """Load the built oracle, building it first if nothing is built."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _LIB
    if not os.path.exists(p):
        build(out=p)
    lib = ctypes.CDLL(p)
    dp = ctypes.POINTER(ctypes.c_double)
    up = ctypes.POINTER(ctypes.c_uint8)
    ip = ctypes.POINTER(ctypes.c_int)
    i, d = ctypes.c_int, ctypes.c_double
    fr = [dp, dp, dp, dp]   # optional area/volume fractions
    lib.oracle_apply.argtypes = [i, i, i, d, dp, up, ip, dp, dp] + fr
    lib.oracle_apply.restype = i
    lib.oracle_relres.argtypes = [i, i, i, d, dp, up, ip, dp, dp] + fr
    lib.oracle_relres.restype = d
    lib.oracle_pcg.argtypes = [i, i, i, d, dp, up, ip, dp, d, i, dp, ip, dp, dp] + fr
    lib.oracle_pcg.restype = i
    lib.oracle_project.argtypes = [i, i, i, d, dp, up, ip, d, dp, dp, dp, dp]
    lib.oracle_project.restype = i
    lib.oracle_divergence.argtypes = [i, i, i, d, dp, dp, dp, dp] + fr
    lib.oracle_divergence.restype = None
    lib.oracle_connected.argtypes = [i, i, i, up, ip]
    lib.oracle_connected.restype = i
    lib.oracle_components.argtypes = [i, i, i, up, ip, ctypes.POINTER(ctypes.c_int)]
    lib.oracle_components.restype = i
    lib.oracle_set_threads.argtypes = [i]
    lib.oracle_set_threads.restype = None
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = i
    lib.oracle_host_triad.argtypes = [ctypes.c_long, i]
    lib.oracle_host_triad.restype = d
    if path is None:
        _lib = lib
    return lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _bc(bc):
    arr = (ctypes.c_int * 6)(*[int(b) for b in bc])
    return arr


def _dims(rho):
    nz, ny, nx = rho.shape
    return nx, ny, nz


def _frac(frac):
    """(ax, ay, az, vol) area and volume fractions, or None: returns the
    kept arrays and the four pointers (NULL without fractions)."""
    if frac is None:
        return (), [None] * 4
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in frac]
    return arrs, [a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs]


def apply(rho, mask, bc, h, p, lib=None, frac=None):
    """L p per Eq. (pois) with the face rules of the module docstring."""
    lib = lib or load()
    rho, rp = _f64(rho)
    mask, mp = _u8(mask)
    p, pp = _f64(p)
    out = np.empty_like(rho)
    nx, ny, nz = _dims(rho)
    keep, fp = _frac(frac)
    st = lib.oracle_apply(nx, ny, nz, float(h), rp, mp, _bc(bc), pp,
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), *fp)
    if st != OK:
        raise ValueError(f"oracle_apply status {st}")
    return out


def relres(rho, mask, bc, h, rhs, p, lib=None, frac=None) -> float:
    """||rhs - L p||_2 / ||rhs||_2 over fluid cells (with fractions, the
    volume-weighted norms of the scaled system).  In a singular problem (one
    fluid region, no Dirichlet wall) the source is measured with its fluid
    mean removed, the source ``pcg`` solves for."""
    lib = lib or load()
    rho, rp = _f64(rho)
    mask, mp = _u8(mask)
    rhs, bp = _f64(rhs)
    p, pp = _f64(p)
    nx, ny, nz = _dims(rho)
    keep, fp = _frac(frac)
    return float(lib.oracle_relres(nx, ny, nz, float(h), rp, mp, _bc(bc), bp, pp, *fp))


class PCGResult:
    def __init__(self, p, status, iters, relres, hist):
        self.p, self.status, self.iters, self.relres, self.hist = \
            p, status, iters, relres, hist

    def __repr__(self):
        return (f"PCGResult(status={self.status}, iters={self.iters}, "
                f"relres={self.relres:.3e})")


def pcg(rho, mask, bc, h, rhs, tol=1e-8, maxit=100000, history=False,
        lib=None, frac=None) -> PCGResult:
    """Jacobi-PCG solve of L p = rhs (cold start); see oracle.c."""
    lib = lib or load()
    rho, rp = _f64(rho)
    mask, mp = _u8(mask)
    rhs, bp = _f64(rhs)
    nx, ny, nz = _dims(rho)
    p = np.zeros_like(rho)
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1) if history else None
    hp = (hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
          if history else None)
    keep, fp = _frac(frac)
    st = lib.oracle_pcg(nx, ny, nz, float(h), rp, mp, _bc(bc), bp, float(tol),
                        int(maxit),
                        p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        ctypes.byref(it), ctypes.byref(rr), hp, *fp)
    if history:
        hist = hist[: it.value + 1]
    return PCGResult(p, st, it.value, rr.value, hist)


def project(rho, mask, bc, h, dt, p, u, v, w, lib=None):
    """Return projected copies of the face velocities (Section 2.1)."""
    lib = lib or load()
    rho, rp = _f64(rho)
    mask, mp = _u8(mask)
    p, pp = _f64(p)
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    v = np.array(v, dtype=np.float64, copy=True, order="C")
    w = np.array(w, dtype=np.float64, copy=True, order="C")
    nx, ny, nz = _dims(rho)
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.oracle_project(nx, ny, nz, float(h), rp, mp, _bc(bc), float(dt), pp,
                            u.ctypes.data_as(dp), v.ctypes.data_as(dp),
                            w.ctypes.data_as(dp))
    if st != OK:
        raise ValueError(f"oracle_project status {st}")
    return u, v, w


def divergence(u, v, w, h, lib=None, frac=None):
    """Face-difference divergence of MAC velocities (with fractions, area-
    weighted and divided by the volume fraction)."""
    lib = lib or load()
    nz, ny, nx1 = u.shape
    nx = nx1 - 1
    u, up_ = _f64(u)
    v, vp = _f64(v)
    w, wp = _f64(w)
    out = np.empty((nz, ny, nx))
    keep, fp = _frac(frac)
    lib.oracle_divergence(nx, ny, nz, float(h), up_, vp, wp,
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), *fp)
    return out


def source(u, v, w, h, dt, mask, lib=None, frac=None):
    """Right-hand side of either stage's pressure equation (Section 2.1, R
    set to zero): div(u)/dt on fluid cells, 0 on hull cells."""
    rhs = divergence(u, v, w, h, lib, frac) / dt
    rhs[np.asarray(mask, dtype=bool)] = 0.0
    return rhs


def rk2_pair(rho_k, rho_star, mask, bc, h, dt, u, v, w, tol=1e-12, maxit=100000,
             lib=None):
    """Pressure half of one two-stage Runge-Kutta step (Section 2.1, R = 0),
    each solve cold-started and taken to ``tol``:

    1. P*  solves div((1/rho(phi^k)) grad P*) = div(u^k)/dt;
    2. u*  = u^k - dt (1/rho(phi^k)) grad P*;
    3. P^{k+1} solves div((1/rho(phi*)) grad P^{k+1}) = div(u* + u^k)/dt;
    4. u^{k+1} = (u* + u^k - dt (1/rho(phi*)) grad P^{k+1}) / 2.

    Returns a dict with p_star, u_star (triple), p_next, u_next (triple) and
    the two iteration counts."""
    lib = lib or load()
    r1 = pcg(rho_k, mask, bc, h, source(u, v, w, h, dt, mask, lib), tol, maxit, lib=lib)
    if r1.status != OK:
        raise ValueError(f"first-stage solve status {r1.status}")
    us = project(rho_k, mask, bc, h, dt, r1.p, u, v, w, lib)
    s = tuple(a + b for a, b in zip(us, (u, v, w)))
    r2 = pcg(rho_star, mask, bc, h, source(*s, h, dt, mask, lib), tol, maxit, lib=lib)
    if r2.status != OK:
        raise ValueError(f"second-stage solve status {r2.status}")
    un = project(rho_star, mask, bc, h, dt, r2.p, *s, lib)
    un = tuple(0.5 * a for a in un)
    return {"p_star": r1.p, "u_star": us, "p_next": r2.p, "u_next": un,
            "iters": (r1.iters, r2.iters)}


def components(mask, bc, lib=None):
    """(fluid regions, regions without a Dirichlet face); periodic faces join
    the cells they connect."""
    lib = lib or load()
    mask, mp = _u8(mask)
    nz, ny, nx = mask.shape
    loose = ctypes.c_int(0)
    n = lib.oracle_components(nx, ny, nz, mp, _bc(bc), ctypes.byref(loose))
    if n < 0:
        raise MemoryError("oracle_components")
    return int(n), int(loose.value)


def connected(mask, bc, lib=None) -> bool:
    lib = lib or load()
    mask, mp = _u8(mask)
    nz, ny, nx = mask.shape
    return bool(lib.oracle_connected(nx, ny, nz, mp, _bc(bc)))


def set_threads(n: int, lib=None) -> None:
    """Threads of the oracle's loops started from the calling thread."""
    lib = lib or load()
    lib.oracle_set_threads(int(n))


def threads(lib=None) -> int:
    lib = lib or load()
    return int(lib.oracle_threads())


def host_triad(n: int = 1 << 26, reps: int = 5, lib=None) -> float:
    """Host STREAM-triad bandwidth (GB/s) on the oracle's threads: context
    for the oracle's timing, not part of the method."""
    lib = lib or load()
    return float(lib.oracle_host_triad(int(n), int(reps)))
