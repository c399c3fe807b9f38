"""ctypes binding of the C ABI declared in include/pcg.h.

Argument marshalling only: every step of the solve runs in the HIP library.
If the library is missing this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# PCGMI_LIB selects another build of the same library (e.g. an install path)
LIB_PATH = os.environ.get("PCGMI_LIB", os.path.join(PKG, "libpcgmi.so"))

OK, MAXIT, PENDING, SINGULAR = 0, 1, 2, 3
EINVAL, EDOMAIN, ESINGULAR, EBREAKDOWN, ENOMEM, EBUSY, EHIP, EUNSUPPORTED = \
    -1, -2, -3, -4, -5, -6, -7, -8
BC_NEUMANN, BC_DIRICHLET, BC_PERIODIC = 0, 1, 2
PREC_FP64, PREC_FP32_IR = 0, 1
WARM_START, SKIP_CONNECTIVITY_CHECK, NO_DENSITY_CLASSES, FRACTIONS = 1, 2, 4, 8
FLAT_TILES, PLANE_TILES, TWO_SWEEPS, NARROW_TILES = 16, 32, 64, 128

EXPORTED = [
    "pcg_workspace_bytes", "pcg_setup", "pcg_solve", "pcg_destroy",
    "pcg_strerror", "pcg_last_hip_error", "pcg_batch_create",
    "pcg_batch_footprint", "pcg_batch_admit", "pcg_batch_step",
    "pcg_batch_poll", "pcg_batch_release", "pcg_batch_destroy",
    "pcg_set_timing", "pcg_last_timing", "pcg_copy_probe",
    "pcg_check_connectivity", "pcg_set_tile_rules", "pcg_get_tile_rules",
    "pcg_density_classes", "pcg_project", "pcg_divergence",
    "pcg_solve_ex", "pcg_project_ex", "pcg_rhs", "pcg_update_density",
    "pcg_set_fractions", "pcg_triad_probe", "pcg_inject_failure",
    "pcg_solve_static", "pcg_tile_form",
]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("h", ctypes.c_double)]


class BC(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32 * 6)]


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("inner_maxit", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("tz", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("outer_iters", ctypes.c_int32),
                ("rel_res_true", ctypes.c_double),
                ("rel_res_recursive", ctypes.c_double),
                ("ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class PCGError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = strerror(code)
        if code == EHIP:
            msg += ": " + last_hip_error()
        super().__init__(f"{where}: {msg} ({code})" if where else f"{msg} ({code})")


_lib = None


def load(path: str = LIB_PATH):
    """Load the built library (raises if it is not built)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, sz, i32, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    lib.pcg_workspace_bytes.argtypes = [P(Grid), P(Opts), P(sz)]
    lib.pcg_setup.argtypes = [P(vp), P(Grid), vp, vp, P(BC), P(Opts), vp, sz, vp]
    lib.pcg_solve.argtypes = [vp, vp, vp, dbl, i32, P(Stats)]
    lib.pcg_destroy.argtypes = [vp]
    lib.pcg_strerror.argtypes = [ctypes.c_int]
    lib.pcg_strerror.restype = ctypes.c_char_p
    lib.pcg_last_hip_error.argtypes = []
    lib.pcg_last_hip_error.restype = ctypes.c_char_p
    lib.pcg_batch_create.argtypes = [P(vp), vp, sz, i32, P(Opts), vp]
    lib.pcg_batch_footprint.argtypes = [vp, P(Grid), P(sz)]
    lib.pcg_batch_admit.argtypes = [vp, P(Grid), vp, vp, P(BC), vp, vp, dbl, i32,
                                    i32, P(i32)]
    lib.pcg_batch_step.argtypes = [vp, i32, P(i32)]
    lib.pcg_batch_poll.argtypes = [vp, i32, P(Stats)]
    lib.pcg_batch_release.argtypes = [vp, i32]
    lib.pcg_batch_destroy.argtypes = [vp]
    lib.pcg_set_timing.argtypes = [vp, i32]
    lib.pcg_last_timing.argtypes = [vp, P(dbl), P(dbl), P(i32)]
    lib.pcg_copy_probe.argtypes = [vp, vp, sz, i32, vp, P(dbl)]
    lib.pcg_triad_probe.argtypes = [vp, vp, vp, sz, dbl, i32, vp, P(dbl)]
    lib.pcg_check_connectivity.argtypes = [vp, P(Grid), P(BC)]
    lib.pcg_set_tile_rules.argtypes = [i32, i32, i32, vp, vp, vp]
    lib.pcg_density_classes.argtypes = [vp, P(i32)]
    lib.pcg_tile_form.argtypes = [vp, P(i32), P(i32), P(i32)]
    lib.pcg_project.argtypes = [vp, vp, dbl, vp, vp, vp]
    lib.pcg_divergence.argtypes = [vp, vp, vp, vp, P(dbl)]
    lib.pcg_get_tile_rules.argtypes = [i32, i32, i32, vp, vp, vp, P(i32)]
    lib.pcg_solve_ex.argtypes = [vp, vp, vp, dbl, i32, i32, P(Stats)]
    lib.pcg_project_ex.argtypes = [vp, vp, dbl, vp, vp, vp, vp, vp, vp, dbl, vp, vp, vp]
    lib.pcg_rhs.argtypes = [vp, dbl, vp, vp, vp, vp, vp, vp, vp]
    lib.pcg_update_density.argtypes = [vp, vp, vp, i32]
    lib.pcg_set_fractions.argtypes = [vp, vp, vp, vp, vp]
    lib.pcg_inject_failure.argtypes = [vp, i32]
    lib.pcg_solve_static.argtypes = [P(Grid), vp, vp, P(BC), P(Opts), vp, vp, dbl, i32,
                                     P(Stats), vp]
    for name in EXPORTED:
        if name not in ("pcg_strerror", "pcg_last_hip_error"):
            getattr(lib, name).restype = ctypes.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().pcg_strerror(int(code)).decode()


def last_hip_error() -> str:
    return load().pcg_last_hip_error().decode()


def check(code: int, where: str = "") -> int:
    if code < 0:
        raise PCGError(code, where)
    return code
