"""Tile-shape autotuner.

For each size class the tuner times short fixed-iteration solves (graph mode,
as served) on a synthetic two-phase + wedge field of that size, for every
candidate tile height tz and (single-solve) workgroup count, and keeps the
fastest per iteration.  The result is a JSON table keyed by GPU architecture:

    {"gfx950": {"fp64":    [[max_cells, tz, grid], ...],
                "fp32_ir": [[max_cells, tz, grid], ...],
                "fp64_batch": [...], "fp32_ir_batch": [...],
                "fp64_plane": [...], "fp32_ir_plane": [...],
                "fp64_narrow": [...], "fp32_ir_narrow": [...],
                "measured": {...}}}

Single-solve rules are tuned on one solve at a time, on tiles of consecutive
cells ("fp64", "fp32_ir"), on wide 2-D plane tiles ("*_plane", grids whose
rows take them) and on narrow ones ("*_narrow", 64 x 4 tiles of one cell a
thread, on rows of odd lengths); plane tiles run one sweep per iteration; batch
rules on a resident batch of several solves of the class size (their tiles
share every launch, so longer tiles usually win).

``install()`` hands a table to the library (pcg_set_tile_rules); the binding
calls it once per process with the table shipped in the package
(``tile_table.json``) unless PCGMI_TILE_TABLE names another file or "none".
Tile height depends only on a solve's own cell count, so a tuned table never
makes a solve's result depend on the other solves it is batched with.

    python -m paper_1410_1942_amd.autotune [--out FILE] [--quick] [--plane-only]
        [--narrow-only]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

from . import _lib as L

PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(PKG, "tile_table.json")
PREC_KEYS = {L.PREC_FP64: "fp64", L.PREC_FP32_IR: "fp32_ir"}

CLASSES = [16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512]
BATCH_CLASSES = [16, 24, 32, 48, 64, 96, 128, 192]
# plane-tile classes as grid shapes (nx, ny, nz), sorted by cell count:
# rows of whole tiles and of partly empty ones (96 and 192 cells: three
# quarters of a tile's lanes busy; FP32 128 and 192: a half and three
# quarters), small grids, where the chain of planes a tile walks sets the
# time, and for FP64 a 256 x 256 x 128 grid, whose tile count per plane and
# height are those of the 512 x 128 x 128 strut tank
PLANE_CLASSES = {L.PREC_FP64: [(128, 64, 64), (96, 96, 96), (128, 128, 128), (192, 192, 192),
                               (256, 256, 128), (256, 256, 256), (384, 384, 384),
                               (512, 512, 512)],
                 L.PREC_FP32_IR: [(128, 64, 64), (128, 128, 128), (192, 192, 192),
                                  (256, 256, 256), (512, 256, 256), (512, 512, 512)]}
# tile heights tried on plane tiles: a tile count just above the resident
# workgroups costs a second round, so heights between the powers of two too
PLANE_TZS = [2, 4, 8, 16, 24, 32, 48, 64, 96, 128, 256]
# narrow-tile classes: rows of odd lengths (narrow tiles are what such rows
# run), sorted by cell count
NARROW_CLASSES = {p: [(33, 33, 33), (65, 65, 65), (99, 99, 99), (127, 127, 127),
                      (161, 120, 100), (191, 191, 191), (255, 255, 255), (383, 383, 383)]
                  for p in (L.PREC_FP64, L.PREC_FP32_IR)}
NARROW_TZS = [4, 8, 16, 24, 32, 48, 64, 96, 128]
# pcg_set_tile_rules table kinds
SINGLE, BATCH, PLANE, NARROW = 0, 1, 2, 3
TZS = [2, 4, 8, 16, 32, 64, 128, 256]
GRIDS = [256, 512, 768, 1024, 2048]

_installed = False


def _kind(for_batches, table):
    return int(table) if table is not None else (BATCH if for_batches else SINGLE)


def get_rules(precision: int, for_batches: bool = False, table=None):
    """Rules of one table: single solves (default), batches, or single
    solves on wide (table = PLANE) or narrow (table = NARROW) plane tiles."""
    lib = L.load()
    cap = 64
    mc = (ctypes.c_int64 * cap)()
    tz = (ctypes.c_int32 * cap)()
    gr = (ctypes.c_int32 * cap)()
    n = ctypes.c_int32()
    L.check(lib.pcg_get_tile_rules(int(precision), _kind(for_batches, table), cap, mc, tz, gr,
                                   ctypes.byref(n)), "pcg_get_tile_rules")
    return [[int(mc[i]), int(tz[i]), int(gr[i])] for i in range(n.value)]


def set_rules(precision: int, rules, for_batches: bool = False, table=None):
    lib = L.load()
    n = len(rules)
    mc = (ctypes.c_int64 * n)(*[int(r[0]) for r in rules])
    tz = (ctypes.c_int32 * n)(*[int(r[1]) for r in rules])
    gr = (ctypes.c_int32 * n)(*[int(r[2]) if len(r) > 2 else 0 for r in rules])
    L.check(lib.pcg_set_tile_rules(int(precision), _kind(for_batches, table), n, mc, tz, gr),
            "pcg_set_tile_rules")


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def install(path: str = None, arch: str = None) -> bool:
    """Install the table for this GPU from `path` (default: the shipped one).
    Returns False when the file has no entry for the architecture."""
    path = path or TABLE
    if not os.path.exists(path):
        return False
    table = json.load(open(path))
    arch = arch or device_arch()
    if arch not in table:
        return False
    for prec, key in PREC_KEYS.items():
        if key in table[arch]:
            set_rules(prec, table[arch][key])
        if key + "_batch" in table[arch]:
            set_rules(prec, table[arch][key + "_batch"], for_batches=True)
        if key + "_plane" in table[arch]:
            set_rules(prec, table[arch][key + "_plane"], table=PLANE)
        if key + "_narrow" in table[arch]:
            set_rules(prec, table[arch][key + "_narrow"], table=NARROW)
    return True


def ensure_installed():
    """Called by the binding before creating solvers (once per process)."""
    global _installed
    if _installed:
        return
    _installed = True
    path = os.environ.get("PCGMI_TILE_TABLE", TABLE)
    if path.lower() == "none":
        return
    try:
        install(path)
    except Exception as e:                       # a broken table must not stop solves
        print(f"tile table not installed: {e}", file=sys.stderr)


def _time_per_iter(dev_case, precision, tz, grid, target_ms=25.0, flags=L.FLAT_TILES):
    import torch
    from .solver import Solver
    rho, mask, rhs, bc, h = dev_case
    s = Solver(rho, mask, bc, h, precision=precision, tz=tz, grid_blocks=grid,
               flags=L.SKIP_CONNECTIVITY_CHECK | flags, check_every=16)
    p = torch.empty_like(rhs)
    s.solve(rhs, p=p, tol=1e-30, maxit=16, raise_on_error=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.solve(rhs, p=p, tol=1e-30, maxit=16, raise_on_error=False)
    torch.cuda.synchronize()
    est = (time.perf_counter() - t) / 16
    iters = int(min(2000, max(32, math.ceil(target_ms * 1e-3 / max(est, 1e-6)))))
    iters = (iters + 15) // 16 * 16
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.solve(rhs, p=p, tol=1e-30, maxit=iters, raise_on_error=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / iters
    s.close()
    return dt * 1e3


def _time_batch_per_iter(dev_case, precision, tz, copies, iters=64):
    """Per-iteration time of `copies` resident copies of one case."""
    import torch
    from .solver import Batch
    rho, mask, rhs, bc, h = dev_case
    b = Batch(1 << 20, 1, precision=precision)
    fp = b.footprint(tuple(rho.shape), h)
    b.close()
    ps = [torch.empty_like(rhs) for _ in range(copies)]

    def run():
        bb = Batch(copies * fp + (4 << 20), copies, precision=precision, tz=tz,
                   check_every=16)
        for p in ps:
            code, _ = bb.admit(rho, mask, bc, h, rhs, p, tol=1e-30, maxit=iters,
                               flags=L.SKIP_CONNECTIVITY_CHECK)
            L.check(code, "admit")
        torch.cuda.synchronize()
        t = time.perf_counter()
        while bb.step(1):
            pass
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        bb.close()
        return dt

    run()
    return run() / iters * 1e3


def tune_batches(classes=BATCH_CLASSES, precisions=(L.PREC_FP64, L.PREC_FP32_IR),
                 tzs=TZS, log=print):
    import torch
    from . import fields as F
    dev = torch.device("cuda:0")
    best = {prec: [] for prec in precisions}
    measured = {}
    for n in classes:
        case = F.make_two_phase(n, n, n, surface_seed=1, velocity_seed=2,
                                wedge=F.Wedge(), keep_velocity=False)
        dev_case = (torch.from_numpy(case.rho).to(dev),
                    torch.from_numpy(case.mask).to(dev),
                    torch.from_numpy(case.rhs).to(dev), case.bc, case.h)
        copies = int(min(64, max(2, (4 << 20) // n ** 3)))
        for prec in precisions:
            key = PREC_KEYS[prec] + "_batch"
            results = sorted((_time_batch_per_iter(dev_case, prec, tz, copies), tz)
                             for tz in tzs if tz <= n)
            ms, tz = results[0]
            measured[f"{key}/{n}x{copies}"] = [[round(m, 5), t] for m, t in results]
            log(f"{key} n={n} x{copies}: best tz={tz} {ms*1e3:.1f} us/iter "
                f"({copies * n**3 / (ms * 1e-3) / 1e9:.2f} Gcell-iter/s)", flush=True)
            best[prec].append((n ** 3, tz))
        del dev_case
        torch.cuda.empty_cache()
    out = {}
    for prec in precisions:
        b = best[prec]
        out[PREC_KEYS[prec] + "_batch"] = [
            [int(math.sqrt(cells * b[i + 1][0])) if i + 1 < len(b) else 2 ** 62, tz, 0]
            for i, (cells, tz) in enumerate(b)]
    out["measured_batch"] = measured
    return out


def tune(classes=CLASSES, precisions=(L.PREC_FP64, L.PREC_FP32_IR), tzs=TZS,
         grids=GRIDS, log=print):
    import torch
    from . import fields as F
    dev = torch.device("cuda:0")
    best = {prec: [] for prec in precisions}
    measured = {}
    for n in classes:
        case = F.make_two_phase(n, n, n, surface_seed=1, velocity_seed=2,
                                wedge=F.Wedge(), keep_velocity=False)
        dev_case = (torch.from_numpy(case.rho).to(dev),
                    torch.from_numpy(case.mask).to(dev),
                    torch.from_numpy(case.rhs).to(dev), case.bc, case.h)
        for prec in precisions:
            key = PREC_KEYS[prec]
            results = []
            for tz in tzs:
                if tz > n:
                    continue
                for g in grids:
                    results.append((_time_per_iter(dev_case, prec, tz, g), tz, g))
            results.sort()
            ms, tz, g = results[0]
            measured[f"{key}/{n}"] = [[round(m, 5), t, gg] for m, t, gg in results[:5]]
            log(f"{key} n={n}: best tz={tz} grid={g} {ms*1e3:.1f} us/iter "
                f"({n**3 / (ms * 1e-3) / 1e9:.2f} Gcell-iter/s)", flush=True)
            best[prec].append((n ** 3, tz, g))
        del dev_case
        torch.cuda.empty_cache()
    out = {}
    for prec in precisions:
        b = best[prec]
        rules = []
        for i, (cells, tz, g) in enumerate(b):
            hi = int(math.sqrt(cells * b[i + 1][0])) if i + 1 < len(b) else 2 ** 62
            rules.append([hi, tz, g])
        out[PREC_KEYS[prec]] = rules
    out["measured"] = measured
    return out


def tune_plane(classes=PLANE_CLASSES, tzs=PLANE_TZS, grids=(512, 768, 1024), log=print,
               form="plane"):
    """Single solves on wide (form "plane") or narrow (form "narrow") plane
    tiles, per grid shape; rules split at the geometric means of the shapes'
    cell counts."""
    flags = L.PLANE_TILES if form == "plane" else L.NARROW_TILES
    import torch
    from . import fields as F
    dev = torch.device("cuda:0")
    out, measured = {}, {}
    for prec, shapes in classes.items():
        key = PREC_KEYS[prec] + "_" + form
        best = []
        for nx, ny, nz in shapes:
            case = F.make_two_phase(nx, ny, nz, surface_seed=1, velocity_seed=2,
                                    wedge=F.Wedge(), keep_velocity=False)
            dev_case = (torch.from_numpy(case.rho).to(dev),
                        torch.from_numpy(case.mask).to(dev),
                        torch.from_numpy(case.rhs).to(dev), case.bc, case.h)
            results = sorted((_time_per_iter(dev_case, prec, tz, g, flags=flags), tz, g)
                             for tz in tzs if tz <= nz for g in grids)
            ms, tz, g = results[0]
            measured[f"{key}/{nx}x{ny}x{nz}"] = [[round(m, 5), t, gg] for m, t, gg in results[:5]]
            cells = nx * ny * nz
            log(f"{key} {nx}x{ny}x{nz}: best tz={tz} grid={g} {ms*1e3:.1f} us/iter "
                f"({cells / (ms * 1e-3) / 1e9:.2f} Gcell-iter/s)", flush=True)
            best.append((cells, tz, g))
            del dev_case
            torch.cuda.empty_cache()
        out[key] = [[int(math.sqrt(c * best[i + 1][0])) if i + 1 < len(best) else 2 ** 62, t, g]
                    for i, (c, t, g) in enumerate(best)]
    out["measured_" + form] = measured
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--quick", action="store_true",
                    help="fewer classes and candidates")
    ap.add_argument("--batches-only", action="store_true",
                    help="tune only the batch tables, keep the others")
    ap.add_argument("--plane-only", action="store_true",
                    help="tune only the wide plane-tile tables, keep the others")
    ap.add_argument("--narrow-only", action="store_true",
                    help="tune only the narrow plane-tile tables, keep the others")
    a = ap.parse_args(argv)
    os.environ["PCGMI_TILE_TABLE"] = "none"
    arch = device_arch()
    full = json.load(open(a.out)) if os.path.exists(a.out) else {}
    table = dict(full.get(arch, {}))
    only = a.batches_only or a.plane_only or a.narrow_only
    if not only:
        kw = dict(classes=[24, 64, 160], tzs=[4, 16, 32], grids=[512, 1024]) if a.quick else {}
        table.update(tune(**kw))
    if not only or a.plane_only:
        kwp = dict(classes={L.PREC_FP64: [(128, 64, 64)]}, tzs=[8, 32]) if a.quick else {}
        table.update(tune_plane(**kwp))
    if not only or a.narrow_only:
        kwn = dict(classes={L.PREC_FP64: [(65, 64, 64)]}, tzs=[8, 32]) if a.quick else {}
        table.update(tune_plane(**dict(dict(classes=NARROW_CLASSES, tzs=NARROW_TZS), **kwn),
                                form="narrow"))
    if not only or a.batches_only:
        kwb = dict(classes=[24, 64], tzs=[4, 16]) if a.quick else {}
        table.update(tune_batches(**kwb))
    full[arch] = table
    with open(a.out, "w") as f:
        json.dump(full, f, indent=1)
    print(f"wrote {a.out} [{arch}]")


if __name__ == "__main__":
    sys.exit(main())
