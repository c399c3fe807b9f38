"""Python front end of the HIP pressure solver.

PyTorch supplies device memory and the HIP stream; every step of the solve
runs in the library behind include/pcg.h (see _lib).  There is no CPU path:
constructing a Solver or Batch without the built library or without a GPU
raises.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib as L


def _grid(shape_zyx, h) -> L.Grid:
    nz, ny, nx = shape_zyx
    return L.Grid(int(nx), int(ny), int(nz), float(h))


def _bc(bc: Sequence[int]) -> L.BC:
    b = L.BC()
    for f in range(6):
        b.kind[f] = int(bc[f])
    return b


def make_opts(precision: int = L.PREC_FP64, check_every: int = 0,
              flags: int = 0, inner_maxit: int = 0, inner_tol: float = 0.0,
              tz: int = 0, grid_blocks: int = 0) -> L.Opts:
    return L.Opts(int(precision), int(check_every), int(flags),
                  int(inner_maxit), float(inner_tol), int(tz), int(grid_blocks))


def _stream_handle(stream: Optional[torch.cuda.Stream]):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check(t: Optional[torch.Tensor], shape, dtype, name: str, device=None,
           optional: bool = False):
    """The library reads and writes exactly the grid's extent through raw
    pointers: refuse anything that is not a contiguous device tensor of the
    expected dtype, shape and device before it gets there."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name}: a device tensor is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: must be a contiguous device tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: must be {dtype} of shape {tuple(shape)}, "
                         f"got {t.dtype} of shape {tuple(t.shape)}")
    if device is not None and t.device != device:
        raise ValueError(f"{name}: must be on {device}, got {t.device}")


def _field_shape(rho: torch.Tensor):
    if not isinstance(rho, torch.Tensor) or rho.dim() != 3:
        raise ValueError("rho: a 3-D [nz, ny, nx] tensor")
    return tuple(rho.shape)


def solve_static(rho: torch.Tensor, mask: Optional[torch.Tensor], bc, h: float,
                 rhs: torch.Tensor, p: Optional[torch.Tensor] = None, tol: float = 1e-8,
                 maxit: int = 1000000, precision: int = L.PREC_FP64, flags: int = 0,
                 stream: Optional[torch.cuda.Stream] = None, raise_on_error=True, **opt_kw):
    """One solve through pcg_solve_static: the library's fixed device
    array serves as workspace, so nothing is allocated (p, when given, is
    the caller's output tensor).  Returns (p, stats dict)."""
    lib = L.load()
    shape = _field_shape(rho)
    _check(rho, shape, torch.float64, "rho")
    _check(mask, shape, torch.uint8, "mask", rho.device, optional=True)
    _check(rhs, shape, torch.float64, "rhs", rho.device)
    if p is None:
        p = torch.empty_like(rhs)
    _check(p, shape, torch.float64, "p", rho.device)
    opts = make_opts(precision=precision, flags=flags, **opt_kw)
    st = L.Stats()
    code = lib.pcg_solve_static(ctypes.byref(_grid(shape, h)), _ptr(rho), _ptr(mask),
                                ctypes.byref(_bc(bc)), ctypes.byref(opts), _ptr(rhs),
                                _ptr(p), float(tol), int(maxit), ctypes.byref(st),
                                _stream_handle(stream))
    if raise_on_error:
        L.check(code, "pcg_solve_static")
    return p, st.as_dict()


class Solver:
    """One density field, any number of solves (pcg_setup / pcg_solve).

    rho: float64 [nz, ny, nx] device tensor; mask: uint8 (1 = hull) or None;
    bc: six wall kinds (x-, x+, y-, y+, z-, z+), 0 Neumann / 1 Dirichlet.
    """

    def __init__(self, rho: torch.Tensor, mask: Optional[torch.Tensor], bc,
                 h: float, precision: int = L.PREC_FP64, flags: int = 0,
                 stream: Optional[torch.cuda.Stream] = None, **opt_kw):
        lib = L.load()
        from .autotune import ensure_installed
        ensure_installed()
        shape = _field_shape(rho)
        _check(rho, shape, torch.float64, "rho")
        _check(mask, shape, torch.uint8, "mask", rho.device, optional=True)
        self.shape = shape
        self.device = rho.device
        self.grid = _grid(self.shape, h)
        self.opts = make_opts(precision=precision, flags=flags, **opt_kw)
        nbytes = ctypes.c_size_t(0)
        L.check(lib.pcg_workspace_bytes(ctypes.byref(self.grid),
                                        ctypes.byref(self.opts),
                                        ctypes.byref(nbytes)), "workspace")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8,
                                     device=rho.device)
        self._stream = _stream_handle(stream)
        self._ctx = ctypes.c_void_p()
        L.check(lib.pcg_setup(ctypes.byref(self._ctx), ctypes.byref(self.grid),
                              _ptr(rho), _ptr(mask), ctypes.byref(_bc(bc)),
                              ctypes.byref(self.opts), _ptr(self.workspace),
                              nbytes.value, self._stream), "pcg_setup")
        self.lib = lib

    def solve(self, rhs: torch.Tensor, p: Optional[torch.Tensor] = None,
              tol: float = 1e-8, maxit: int = 1000000, raise_on_error=True,
              warm: Optional[bool] = None):
        """Solve L p = rhs.  Returns (p, stats dict).  ``warm`` True starts
        from p's contents, False from zero, None as the setup flags say."""
        _check(rhs, self.shape, torch.float64, "rhs", self.device)
        if p is None:
            if warm:
                raise ValueError("a warm start needs p")
            p = torch.empty_like(rhs)
        _check(p, self.shape, torch.float64, "p", self.device)
        st = L.Stats()
        if warm is None:
            code = self.lib.pcg_solve(self._ctx, _ptr(rhs), _ptr(p), float(tol),
                                      int(maxit), ctypes.byref(st))
        else:
            code = self.lib.pcg_solve_ex(self._ctx, _ptr(rhs), _ptr(p), float(tol),
                                         int(maxit), L.WARM_START if warm else 0,
                                         ctypes.byref(st))
        if raise_on_error:
            L.check(code, "pcg_solve")
        return p, st.as_dict()

    def update_density(self, rho: torch.Tensor, mask: Optional[torch.Tensor] = None,
                       flags: int = 0):
        """New density (and hull) on the same grid and walls
        (pcg_update_density); the next solve may warm-start."""
        _check(rho, self.shape, torch.float64, "rho", self.device)
        _check(mask, self.shape, torch.uint8, "mask", self.device, optional=True)
        L.check(self.lib.pcg_update_density(self._ctx, _ptr(rho), _ptr(mask), int(flags)),
                "pcg_update_density")

    def density_classes(self) -> int:
        """Fluid density classes in use (0: per-cell densities)."""
        n = ctypes.c_int32()
        L.check(self.lib.pcg_density_classes(self._ctx, ctypes.byref(n)), "classes")
        return n.value

    def tile_form(self):
        """(columns, rows) of the context's plane tiles, or (0, 0) for tiles
        of consecutive cells (pcg_tile_form)."""
        return self.tile_form_ex()[:2]

    def tile_form_ex(self):
        """(columns, rows, sweeps per iteration) of the context's tiles
        (pcg_tile_form)."""
        tx, ty, sw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        L.check(self.lib.pcg_tile_form(self._ctx, ctypes.byref(tx), ctypes.byref(ty),
                                       ctypes.byref(sw)), "pcg_tile_form")
        return tx.value, ty.value, sw.value

    def set_fractions(self, ax=None, ay=None, az=None, vol=None):
        """Free-slip cut-cell fractions (pcg_set_fractions): MAC face area
        fractions ax[nz,ny,nx+1], ay[nz,ny+1,nx], az[nz+1,ny,nx] and cell
        volume fractions vol[nz,ny,nx], float64 device tensors; no arguments
        clears them.  Needs a Solver created with flags including FRACTIONS."""
        if ax is None and ay is None and az is None and vol is None:
            L.check(self.lib.pcg_set_fractions(self._ctx, None, None, None, None),
                    "pcg_set_fractions")
            return
        a = self._faces((ax, ay, az), "fractions")
        _check(vol, self.shape, torch.float64, "vol", self.device)
        L.check(self.lib.pcg_set_fractions(self._ctx, *a, _ptr(vol)), "pcg_set_fractions")

    def _faces(self, faces, what):
        nz, ny, nx = self.shape
        if faces is None or len(faces) != 3:
            raise ValueError(f"{what}: three face arrays (u, v, w)")
        for t, shp, c in zip(faces, ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)),
                             "uvw"):
            _check(t, shp, torch.float64, f"{what} {c}", self.device)
        return [_ptr(t) for t in faces]

    def project(self, p: torch.Tensor, dt: float, u: torch.Tensor,
                v: torch.Tensor, w: torch.Tensor, add=None, weight: float = 1.0,
                out=None):
        """Face update out = weight (u [+ add] - dt (1/rho) grad p) on the MAC
        faces (pcg_project_ex); out defaults to (u, v, w), i.e. in place."""
        a = self._faces((u, v, w), "velocity")
        b = self._faces(add, "add") if add is not None else [None, None, None]
        o = self._faces(out, "out") if out is not None else a
        _check(p, self.shape, torch.float64, "p", self.device)
        L.check(self.lib.pcg_project_ex(self._ctx, _ptr(p), float(dt), *a, *b,
                                        float(weight), *o), "pcg_project_ex")

    def rhs(self, dt: float, u, v, w, add=None, out: Optional[torch.Tensor] = None):
        """Source div(u [+ add]) / dt in fluid cells, 0 in hull cells (pcg_rhs)."""
        a = self._faces((u, v, w), "velocity")
        b = self._faces(add, "add") if add is not None else [None, None, None]
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        _check(out, self.shape, torch.float64, "out", self.device)
        L.check(self.lib.pcg_rhs(self._ctx, float(dt), *a, *b, _ptr(out)), "pcg_rhs")
        return out

    def divergence(self, u, v, w):
        """(||D u||_2, max |D u|) over fluid cells (pcg_divergence)."""
        a = self._faces((u, v, w), "velocity")
        out = (ctypes.c_double * 2)()
        L.check(self.lib.pcg_divergence(self._ctx, *a, out), "pcg_divergence")
        return out[0], out[1]

    def inject_failure(self, after_steps: int):
        """Test hook: the after_steps-th polling step of the next solve
        reports a runtime failure (pcg_inject_failure); 0 disarms."""
        L.check(self.lib.pcg_inject_failure(self._ctx, int(after_steps)),
                "pcg_inject_failure")

    def set_timing(self, on: bool = True):
        L.check(self.lib.pcg_set_timing(self._ctx, int(on)), "pcg_set_timing")

    def last_timing(self):
        a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        L.check(self.lib.pcg_last_timing(self._ctx, ctypes.byref(a),
                                         ctypes.byref(b), ctypes.byref(n)),
                "pcg_last_timing")
        return a.value, b.value, n.value

    def close(self):
        if self._ctx:
            self.lib.pcg_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Resident solves advanced together (pcg_batch_*).

    The arena is one device tensor of ``arena_bytes``; admission fails with
    PCG_EBUSY (returned, not raised) when a solve does not fit.
    """

    def __init__(self, arena_bytes: int, max_slots: int,
                 precision: int = L.PREC_FP32_IR, device="cuda",
                 stream: Optional[torch.cuda.Stream] = None, **opt_kw):
        lib = L.load()
        from .autotune import ensure_installed
        ensure_installed()
        self.lib = lib
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8,
                                 device=device)
        self.opts = make_opts(precision=precision, **opt_kw)
        self._b = ctypes.c_void_p()
        L.check(lib.pcg_batch_create(ctypes.byref(self._b), _ptr(self.arena),
                                     int(arena_bytes), int(max_slots),
                                     ctypes.byref(self.opts),
                                     _stream_handle(stream)), "pcg_batch_create")
        self._keep = {}

    def footprint(self, shape_zyx, h=1.0) -> int:
        out = ctypes.c_size_t()
        g = _grid(shape_zyx, h)
        L.check(self.lib.pcg_batch_footprint(self._b, ctypes.byref(g),
                                             ctypes.byref(out)), "footprint")
        return int(out.value)

    def admit(self, rho, mask, bc, h, rhs, p, tol=1e-8, maxit=1000000,
              flags=0):
        """Returns (status, slot).  status PCG_EBUSY means "try later"."""
        shape = _field_shape(rho)
        dev = self.arena.device
        _check(rho, shape, torch.float64, "rho", dev)
        _check(mask, shape, torch.uint8, "mask", dev, optional=True)
        _check(rhs, shape, torch.float64, "rhs", dev)
        _check(p, shape, torch.float64, "p", dev)
        g = _grid(shape, h)
        slot = ctypes.c_int32(-1)
        code = self.lib.pcg_batch_admit(self._b, ctypes.byref(g), _ptr(rho),
                                        _ptr(mask), ctypes.byref(_bc(bc)),
                                        _ptr(rhs), _ptr(p), float(tol),
                                        int(maxit), int(flags),
                                        ctypes.byref(slot))
        if code == L.EBUSY:
            return code, -1
        L.check(code, "pcg_batch_admit")
        self._keep[slot.value] = (rhs, p)
        return code, slot.value

    def step(self, replays: int = 1) -> int:
        active = ctypes.c_int32()
        L.check(self.lib.pcg_batch_step(self._b, int(replays),
                                        ctypes.byref(active)), "pcg_batch_step")
        return active.value

    def poll(self, slot: int):
        st = L.Stats()
        code = self.lib.pcg_batch_poll(self._b, int(slot), ctypes.byref(st))
        return code, st.as_dict()

    def release(self, slot: int):
        L.check(self.lib.pcg_batch_release(self._b, int(slot)), "release")
        self._keep.pop(slot, None)

    def close(self):
        if self._b:
            self.lib.pcg_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def triad_probe(n_doubles: int, reps: int = 10, device="cuda") -> float:
    """Achieved triad bandwidth (GB/s, 24 B per element) of a plain
    a = b + s c kernel on three arrays of n_doubles."""
    lib = L.load()
    b = torch.ones(n_doubles, dtype=torch.float64, device=device)
    c = torch.ones(n_doubles, dtype=torch.float64, device=device)
    a = torch.empty_like(b)
    ms = ctypes.c_double()
    L.check(lib.pcg_triad_probe(_ptr(a), _ptr(b), _ptr(c), n_doubles, 3.0, int(reps),
                                _stream_handle(None), ctypes.byref(ms)), "triad probe")
    del a, b, c
    return 24 * n_doubles / (ms.value * 1e-3) / 1e9


def copy_probe(n_doubles: int, reps: int = 20, device="cuda") -> float:
    """Achieved copy bandwidth (GB/s, read + write) of a plain copy kernel."""
    lib = L.load()
    src = torch.ones(n_doubles, dtype=torch.float64, device=device)
    dst = torch.empty_like(src)
    ms = ctypes.c_double()
    L.check(lib.pcg_copy_probe(_ptr(src), _ptr(dst), n_doubles, int(reps),
                               _stream_handle(None), ctypes.byref(ms)), "probe")
    return 2 * 8 * n_doubles / (ms.value * 1e-3) / 1e9
