#!/usr/bin/env python3
"""Throughput of the MI355X pressure solve (one JSON line on stdout).

Workload: 512^3 two-phase tank (water 1000 below an eight-mode free surface,
air 1.2 above), vertical wedge hull (half-angle 15 deg, draft 0.2), Neumann
on five walls and p = 0 on top, source = div(u)/dt of seeded face
velocities, tolerance 1e-8 on the relative residual.

A step is the whole hot path on that input: density encoding and validation
(setup) plus the FP64 Jacobi-PCG solve to 1e-8, inputs resident in HBM.
The metric is cell-iterations per second, nx*ny*nz*iterations / step time.
Beside it: the FP32-stencil form with FP64 iterative refinement on the same
input, the roofline of the dominant kernel (hipEvent-timed on the solver's
stream), the copy bandwidth achieved on this device, and the CPU reference
timed on the host cores for a bounded number of iterations.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell of the two iteration kernels, by precision and
# coefficient source (a one-byte density class, or the density itself)
#   pass A: read p_old, z, coefficient key; write p
#   pass B: read p, z, coefficient key (+ x or d, p_prev, p_prev2); write z (+ x or d)
BYTES_K1 = {("fp64", "classes"): 25, ("fp64", "density"): 32,
            ("fp32", "classes"): 13, ("fp32", "density"): 16}
# pass B reads and writes x (FP64) or the inner correction d (FP32) every
# third launch only, together with the two previous directions (FP64 25, 25,
# 57 B/cell with classes, 32, 32, 64 with densities; FP32 13, 13, 29 and 16,
# 16, 32): the per-launch average
BYTES_K2 = {("fp64", "classes"): 107 / 3, ("fp64", "density"): 128 / 3,
            ("fp32", "classes"): 55 / 3, ("fp32", "density"): 64 / 3}
# the one-sweep FP64 iteration on plane tiles (its only kernel with work):
# read z, p_old, coefficient key; write p, z' (33 B/cell with classes, 40
# with densities); every third launch also x (read and write) and the
# direction two back: 57 and 64 B/cell; the per-launch average
BYTES_SWEEP = {("fp64", "classes"): 123 / 3, ("fp64", "density"): 144 / 3}


def iteration_bytes(mode, sweeps):
    """(first-half, second-half) kernel bytes per cell of an FP64 iteration."""
    if sweeps == 1:
        return 0.0, BYTES_SWEEP[("fp64", mode)]
    return BYTES_K1[("fp64", mode)], BYTES_K2[("fp64", mode)]


# Timings the paper reports (Section 3), as context only: whole time steps of
# the full flow solver (two pressure solves plus advection, interface
# capturing and the rest), on its machines; no Poisson-level number is
# given, so no ratio to them is formed.
PAPER_CONTEXT = [
    {"case": "NACA 0024 strut, 512x128x128 cells", "seconds_per_time_step": 60,
     "hardware": "512 Cray T3E processors"},
    {"case": "DDG 5415, 2,097,152 cells", "seconds_per_time_step": 376,
     "hardware": "32 IBM processors"},
    {"case": "DDG 5415 with AMR, 5,324,800 cells", "seconds_per_time_step": 1300,
     "hardware": "32 IBM processors"},
    {"case": "DDG 5415 with AMR, 17,940,480 cells", "seconds_per_time_step": 3000,
     "hardware": "64 IBM processors"},
]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="grid edge")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-ir", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=40,
                    help="oracle iterations timed on the full-size input")
    ap.add_argument("--cpu-iters-256", type=int, default=100,
                    help="oracle iterations timed on the 256^3 wedge input")
    ap.add_argument("--no-project", action="store_true")
    ap.add_argument("--no-rk2", action="store_true")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the 256^3 wedge and strut single-solve legs")
    ap.add_argument("--no-tight", action="store_true",
                    help="skip the solves at the tolerance that meets the 1e-6 error bar")
    ap.add_argument("--tight-tol", type=float, default=1e-9)
    ap.add_argument("--no-density", action="store_true",
                    help="skip the mollified-interface (per-cell density) leg")
    ap.add_argument("--rk2-shift", type=float, default=0.025,
                    help="surface phase advance (rad) that gives rho(phi*); "
                         "0.025 moves the 512^3 surface by at most about one cell")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--batch-n", type=int, default=64)
    ap.add_argument("--serve-n", type=int, default=1000,
                    help="reported requests of the served stream")
    ap.add_argument("--serve-warmup", type=int, default=100,
                    help="warm-up requests served before the reported ones")
    ap.add_argument("--profile-iters", type=int, default=0,
                    help="short run for counter collection: copy probe of "
                         "1 GiB, then FP64 and FP32+IR solves capped at this "
                         "many iterations; prints a summary and exits")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles",
                                                      "traffic_wedge512.txt"))
    return ap.parse_args()


def read_traffic(path):
    """key = value lines of a committed counter summary (or None)."""
    if not os.path.exists(path):
        return None
    out = {}
    for line in open(path):
        line = line.strip()
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            out[k.strip()] = v.strip()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solve is not sharded "
              "across GPUs in this build (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd import fields as F
    from paper_1410_1942_amd.solver import Solver, copy_probe, triad_probe

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    n = args.n
    log(f"generating wedge{n} input")
    t = time.time()
    case = F.config_wedge(n, keep_velocity=not args.no_project and not args.profile_iters)
    log(f"  {time.time() - t:.1f} s")
    rho = torch.from_numpy(case.rho).to(dev)
    mask = torch.from_numpy(case.mask).to(dev)
    rhs = torch.from_numpy(case.rhs).to(dev)
    cells = case.ncells
    torch.cuda.synchronize()

    if args.profile_iters:
        copy_gbs = copy_probe(1 << 27, reps=3)
        res = {"copy_bytes": (1 << 27) * 8, "copy_GBps": copy_gbs, "cells": cells}
        for prec, name in ((L.PREC_FP64, "fp64"), (L.PREC_FP32_IR, "ir")):
            s = Solver(rho, mask, case.bc, case.h, precision=prec)
            _, st = s.solve(rhs, tol=1e-30, maxit=args.profile_iters,
                            raise_on_error=False)
            s.close()
            res[name] = st
        print(json.dumps(res), flush=True)
        return

    coef, form = {}, {}

    def step(precision=L.PREC_FP64, p=None, timing=False):
        s = Solver(rho, mask, case.bc, case.h, precision=precision)
        coef[precision] = "classes" if s.density_classes() else "density"
        form[precision] = s.tile_form_ex()
        if timing:
            s.set_timing(True)
        p, st = s.solve(rhs, p=p, tol=args.tol)
        tm = s.last_timing() if timing else None
        s.close()
        return p, st, tm

    # achievable bandwidth: plain copy of 4 GiB, STREAM triad on 3 x 4 GiB
    log("copy and triad probes")
    copy_gbs = copy_probe(1 << 29, reps=10)
    triad_gbs = triad_probe(1 << 29, reps=10)
    torch.cuda.empty_cache()
    log(f"  copy {copy_gbs:.0f} GB/s, triad {triad_gbs:.0f} GB/s")

    # setup alone (density encoding + host connectivity check)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s0 = Solver(rho, mask, case.bc, case.h)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t) * 1e3
    s0.close()
    del s0

    p64 = torch.empty_like(rhs)
    for w in range(args.warmup):
        log(f"warmup {w}")
        _, st, _ = step(p=p64)
        log(f"  iters {st['iters']} relres {st['rel_res_true']:.3e}")
    torch.cuda.synchronize()
    log(f"timed {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st64, _ = step(p=p64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    iters = st64["iters"]
    value = cells * iters / (ms_step * 1e-3) / 1e9
    log(f"  {ms_step:.1f} ms/step, {iters} iters, {value:.2f} Gcell-iter/s")

    out = {
        "metric": "PCG Gcell-iter/s & %HBM roofline at 1e-8 rel-res",
        "value": round(value, 3),
        "unit": "Gcell-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"wedge{n}_fp64: {n}^3 two-phase tank + wedge hull, "
                        f"FP64 Jacobi-PCG to rel-res {args.tol:g}",
            "grid": [n, n, n], "cells": cells, "tol": args.tol,
            "rho_water": F.RHO_WATER, "rho_air": F.RHO_AIR,
            "surface": "8 modes, amp 0.01, k 2-16, seed 1", "velocity_seed": 2,
            "hull": "wedge half-angle 15 deg, draft 0.2",
            "bc": "Neumann x,y,z-; Dirichlet z+",
        },
        "iters": iters,
        "rel_res_true": st64["rel_res_true"],
        "setup_ms": round(setup_ms, 2),
        "copy_GBps": round(copy_gbs, 1),
        "triad_GBps": round(triad_gbs, 1),
    }

    # roofline of the dominant kernel, hipEvent-timed on the solver's stream
    if not args.no_roofline:
        log("event-timed solve")
        _, stt, (k1_ms, k2_ms, nlaunch) = step(p=p64, timing=True)
        mode = coef[L.PREC_FP64]
        tx, ty, sweeps = form[L.PREC_FP64]
        b1, b2 = iteration_bytes(mode, sweeps)
        # kernel template argument of the coefficient mode (plane tiles: 3, 4)
        plane = tx > 0
        kmode = (3 if mode == "classes" else 4) if plane else (1 if mode == "classes" else 0)
        tiles = (f"{tx}x{ty} plane tiles, LDS-staged" if plane else "tiles of consecutive cells")
        a2 = b2 * cells / (k2_ms * 1e-3) / 1e9
        a1 = b1 * cells / (k1_ms * 1e-3) / 1e9
        traffic = None
        tr = read_traffic(args.traffic)
        if tr and tr.get("kernel_source_sha") == kernel_sha():
            key = f"bytes[k_iter<0, 2, {kmode}>]"
            try:
                traffic = float(tr[key])
            except (KeyError, ValueError):
                traffic = None
        out["roofline"] = {
            "bound": "hbm", "achieved": round(a2, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(a2 / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": (f"k_iter<0,2,{kmode}> (FP64 one-sweep iteration, {mode}, {tiles}): "
                       f"p update + operator apply + z update + r.z, r.r, z.Az, x updated "
                       f"every third launch ({b2:.2f} B/cell per launch on average)"
                       if sweeps == 1 else
                       f"k_iter<0,2,{kmode}> (FP64 pass B, {mode}, {tiles}): operator apply + "
                       f"z update + r.z, r.r, x updated every third launch "
                       f"({b2:.2f} B/cell per launch on average)"),
            "sweeps_per_iteration": sweeps,
            "avg_ms": round(k2_ms, 4), "launches": nlaunch,
            "frac_of_copy": round(a2 / copy_gbs, 4),
            "frac_of_triad": round(a2 / triad_gbs, 4),
            # counted HBM bytes per launch over the same event-timed duration
            "traffic_GBps": (round(traffic / (k2_ms * 1e-3) / 1e9, 1)
                             if traffic is not None else None),
        }
        if sweeps == 1:
            out["kernel_k1"] = {
                "kernel": f"k_iter<0,3,{kmode}> (FP64 first-half launch: passes the one-sweep "
                          f"solve by, except for its set-up, first pass A and residual checks)",
                "avg_ms": round(k1_ms, 4), "achieved_GBps": None, "frac": None,
            }
        else:
            out["kernel_k1"] = {
                "kernel": f"k_iter<0,3,{kmode}> (FP64 pass A, {mode}, {tiles}): p update + "
                          f"p.Ap, and the rare set-up and residual actions ({b1} B/cell)",
                "avg_ms": round(k1_ms, 4), "achieved_GBps": round(a1, 1),
                "frac": round(a1 / HBM_PEAK_GBS, 4),
            }
        per_iter_ms = k1_ms + k2_ms
        out["iteration_GBps"] = round((b1 + b2) * cells / (per_iter_ms * 1e-3) / 1e9, 1)
        out["coefficients"] = mode
        log(f"  K1 {k1_ms:.3f} ms ({a1:.0f} GB/s)  K2 {k2_ms:.3f} ms ({a2:.0f} GB/s)")

    # mixed precision: FP32 stencil, FP64 refinement, same input and tolerance
    if not args.no_ir:
        log("FP32+IR solve")
        pir = torch.empty_like(rhs)
        step(precision=L.PREC_FP32_IR, p=pir)   # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, stir, _ = step(precision=L.PREC_FP32_IR, p=pir)
        torch.cuda.synchronize()
        ir_ms = (time.perf_counter() - t) * 1e3
        err = (pir - p64).abs().max().item() / p64.abs().max().item()
        out["ir"] = {
            "tol": args.tol,
            "ms_per_step": round(ir_ms, 2),
            "inner_iters": stir["iters"], "outer_iters": stir["outer_iters"],
            "rel_res_true": stir["rel_res_true"],
            "Gcell_iter_per_s": round(cells * stir["iters"] / (ir_ms * 1e-3) / 1e9, 3),
            "speedup_vs_fp64": round(ms_step / ir_ms, 3),
            "max_err_vs_fp64": err,
        }
        log(f"  {ir_ms:.1f} ms, {stir['iters']} inner / {stir['outer_iters']} outer, "
            f"err vs fp64 {err:.2e}")

    # error against the oracle's own 1e-12 solution, read at its stored
    # strided sample (written by tests/golden/make_fullsize_golden.py)
    gold = golden_reference(n, case)
    if gold is not None:
        meta, ref = gold
        out["max_err_vs_oracle"] = err_vs_golden(p64, meta, ref)
        if "ir" in out:
            out["ir"]["max_err_vs_oracle"] = err_vs_golden(pir, meta, ref)
        out["oracle_reference"] = {"tol": meta["tol"], "iters": meta["iters"],
                                   "relres": meta["relres"],
                                   "sample": f"every {meta['stride']}th cell per axis"}
        log(f"  max err vs oracle: fp64 {out['max_err_vs_oracle']:.2e}"
            + (f", ir {out['ir']['max_err_vs_oracle']:.2e}" if "ir" in out else ""))
        if not args.no_tight:
            out["tight_tol"] = bench_tight(rho, mask, rhs, case, args.tight_tol, meta, ref,
                                           not args.no_ir)
    out["paper_context"] = PAPER_CONTEXT

    # CPU reference on the host cores: a bounded number of iterations
    if not args.no_cpu:
        import oracle
        log("cpu baseline")

        def cpu_rate(c, k):
            t = time.perf_counter()
            oracle.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-30, maxit=1)
            ta = time.perf_counter() - t
            t = time.perf_counter()
            oracle.pcg(c.rho, c.mask, c.bc, c.h, c.rhs, tol=1e-30, maxit=1 + k)
            tb = time.perf_counter() - t
            return c.ncells * k / max(tb - ta, 1e-9) / 1e9, ta

        k = args.cpu_iters
        cpu_val, ta = cpu_rate(case, k)
        out["cpu_baseline"] = {
            "value": round(cpu_val, 5), "unit": "Gcell-iter/s",
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"wedge{n} input, {k} PCG iterations timed as the "
                      f"difference of a {1 + k}- and a 1-iteration run "
                      f"(setup {ta:.1f} s excluded)",
            "cpu_model": host_cpu_model(),
            "host_cpus": len(os.sched_getaffinity(0)),
            "host_triad_GBps": round(oracle.host_triad(), 1),
        }
        if args.cpu_iters_256 > 0:
            c2 = F.config_wedge(256, keep_velocity=False)
            v2, _ = cpu_rate(c2, args.cpu_iters_256)
            out["cpu_baseline"]["wedge256_Gcell_iter_per_s"] = round(v2, 5)
            out["cpu_baseline"]["wedge256_sample"] = (
                f"{args.cpu_iters_256} PCG iterations on the 256^3 wedge input")
            del c2
        # relative residual of the GPU solutions recomputed by the reference
        out["rel_res_oracle"] = oracle.relres(case.rho, case.mask, case.bc, case.h,
                                              case.rhs, p64.cpu().numpy())
        if not args.no_ir:
            out["ir"]["rel_res_oracle"] = oracle.relres(
                case.rho, case.mask, case.bc, case.h, case.rhs, pir.cpu().numpy())
        log(f"  {cpu_val:.4f} Gcell-iter/s on {oracle.threads()} threads")

    if not args.no_side:
        # the 32^3 parity case: launch-bound on the GPU; the oracle's full
        # solve of it timed on the host beside it
        c1 = F.config1(32, keep_velocity=False)
        out["flat32"] = bench_single(c1, args.tol, dev, "32^3 flat two-phase tank, FP64")
        if not args.no_cpu:
            import oracle
            t = time.perf_counter()
            ref = oracle.pcg(c1.rho, c1.mask, c1.bc, c1.h, c1.rhs, tol=args.tol)
            out["flat32"]["oracle_solve_ms"] = round((time.perf_counter() - t) * 1e3, 2)
            out["flat32"]["oracle_iters"] = int(ref.iters)
        c256 = F.config_wedge(256, keep_velocity=False)
        out["wedge256"], p256 = bench_single(c256, args.tol, dev,
                                             "256^3 two-phase tank + wedge hull, FP64",
                                             want_p=True)
        g256 = golden_reference(256, c256)
        if g256 is not None:
            out["wedge256"]["max_err_vs_oracle"] = err_vs_golden(p256, *g256)
        del c256, p256
        out["strut"] = bench_single(F.config_strut(keep_velocity=False), args.tol, dev,
                                    "strut tank 512x128x128 (NACA 0024, periodic x, "
                                    "no-flux walls: singular), FP64")
        out["cut_cells256"] = bench_single(
            F.make_two_phase(256, 256, 256, surface_seed=1, velocity_seed=2, wedge=F.Wedge(),
                             keep_velocity=False, fractions=True), args.tol, dev,
            "256^3 two-phase tank + wedge as free-slip cut cells (area/volume fractions), FP64")
    if not args.no_density:
        out["density512"] = bench_density(n, args.tol, dev, not args.no_ir)
    if not args.no_project:
        out["projection"] = bench_project(case, rho, mask, p64, dev)
        if not args.no_rk2:
            out["rk2_pair"] = bench_rk2(case, rho, mask, dev, args.tol, args.rk2_shift)
        case.u = case.v = case.w = None
    if not args.no_batch:
        out["batch"] = bench_batch(args.batch_n)
    if not args.no_serve:
        out["served"] = bench_serve(args.serve_n, args.serve_warmup)

    print(json.dumps(out), flush=True)


def bench_single(case, tol, dev, what, want_p=False):
    """One more single solve (set-up excluded, timed on the host around a
    synchronised solve after a warm-up solve), its iteration count and the
    oracle's recomputed residual of the answer."""
    import numpy as np
    import torch
    import oracle
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import Solver
    log(what)
    rho = torch.from_numpy(case.rho).to(dev)
    mask = torch.from_numpy(case.mask).to(dev)
    rhs = torch.from_numpy(case.rhs).to(dev)
    frac = case.frac
    s = Solver(rho, mask, case.bc, case.h, flags=L.FRACTIONS if frac is not None else 0)
    if frac is not None:
        s.set_fractions(*(torch.from_numpy(a).to(dev) for a in frac))
    p, st = s.solve(rhs, tol=tol)
    torch.cuda.synchronize()
    t = time.perf_counter()
    p, st = s.solve(rhs, p=p, tol=tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    classes = s.density_classes()
    s.close()
    pn = p.cpu().numpy()
    fluid = case.mask == 0
    singular = 1 not in case.bc
    rr = oracle.relres(case.rho, case.mask, case.bc, case.h, case.rhs, pn, frac=frac)
    g = case.ncells * st["iters"] / dt / 1e9
    log(f"  {st['iters']} iters, {dt*1e3:.1f} ms, {g:.2f} Gcell-iter/s, oracle relres {rr:.3e}")
    out = {"workload": what, "grid": [case.nx, case.ny, case.nz], "cells": case.ncells,
           "iters": st["iters"], "ms": round(dt * 1e3, 2), "Gcell_iter_per_s": round(g, 3),
           "rel_res_oracle": rr, "density_classes": classes}
    if singular:
        out["fluid_mean_of_p"] = float(pn[fluid].mean())
    return (out, pn) if want_p else out


def golden_reference(n, case):
    """(metadata, sample) of the oracle's stored 1e-12 solution of the n^3
    wedge tank, or None when none is stored or its inputs differ from
    `case` (checked by digest)."""
    import hashlib
    import numpy as np
    base = os.path.join(ROOT, "tests", "golden", f"wedge{n}_oracle")
    if not (os.path.exists(base + ".json") and os.path.exists(base + ".npy")):
        return None
    meta = json.load(open(base + ".json"))
    if case is not None:
        h = hashlib.sha256()
        for a in (case.rho, case.mask, case.rhs):
            h.update(np.ascontiguousarray(a).tobytes())
        if h.hexdigest() != meta["input_sha256"]:
            return None
    return meta, np.load(base + ".npy")


def err_vs_golden(p, meta, ref):
    """max |p - p_oracle| / max |p_oracle| over the stored sample cells."""
    import numpy as np
    import torch
    o, st = meta["offset"], meta["stride"]
    if isinstance(p, torch.Tensor):
        p = p[o::st, o::st, o::st].cpu().numpy()
    else:
        p = p[o::st, o::st, o::st]
    return float(np.abs(p - ref).max() / meta["p_max_abs"])


def bench_tight(rho, mask, rhs, case, tol, meta, ref, with_ir):
    """Both forms at the tighter tolerance that meets the 1e-6 error bar at
    this size (1e-8 does not bound the max-norm error that far here)."""
    import torch
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import Solver
    log(f"tolerance {tol:g}")
    out = {"tol": tol}
    for prec, name in ((L.PREC_FP64, "fp64"), (L.PREC_FP32_IR, "ir")):
        if prec == L.PREC_FP32_IR and not with_ir:
            continue
        s = Solver(rho, mask, case.bc, case.h, precision=prec)
        p = torch.empty_like(rhs)
        s.solve(rhs, p=p, tol=tol)                       # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = s.solve(rhs, p=p, tol=tol)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
        s.close()
        e = err_vs_golden(p, meta, ref)
        out[name] = {"ms": round(ms, 2), "iters": st["iters"], "outer_iters": st["outer_iters"],
                     "rel_res_true": st["rel_res_true"], "max_err_vs_oracle": e,
                     "Gcell_iter_per_s": round(case.ncells * st["iters"] / (ms * 1e-3) / 1e9, 3)}
        log(f"  {name}: {st['iters']} iters, {ms:.0f} ms, err vs oracle {e:.2e}")
        del p
    return out


def bench_density(n, tol, dev, with_ir):
    """The same tank with the interface smoothed over about 1.5 cells (the
    paper's mollified step): more distinct densities than classes, so every
    pass reads the FP64 (FP32) density per cell.  Whole solves plus the
    event-timed passes and their roofline."""
    import torch
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd import fields as F
    from paper_1410_1942_amd.solver import Solver
    log(f"mollified interface {n}^3")
    case = F.make_two_phase(n, n, n, surface_seed=1, velocity_seed=2, wedge=F.Wedge(),
                            mollify=1.5, keep_velocity=False)
    rho = torch.from_numpy(case.rho).to(dev)
    mask = torch.from_numpy(case.mask).to(dev)
    rhs = torch.from_numpy(case.rhs).to(dev)
    out = {"workload": f"{n}^3 two-phase tank + wedge, interface smoothed over 1.5 cells",
           "distinct_densities": int(len(torch.unique(rho)))}
    for prec, name in ((L.PREC_FP64, "fp64"), (L.PREC_FP32_IR, "ir")):
        if prec == L.PREC_FP32_IR and not with_ir:
            continue
        s = Solver(rho, mask, case.bc, case.h, precision=prec)
        p = torch.empty_like(rhs)
        s.solve(rhs, p=p, tol=tol)                       # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = s.solve(rhs, p=p, tol=tol)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
        d = {"ms": round(ms, 2), "iters": st["iters"], "outer_iters": st["outer_iters"],
             "rel_res_true": st["rel_res_true"], "coefficients":
             "classes" if s.density_classes() else "density",
             "Gcell_iter_per_s": round(case.ncells * st["iters"] / (ms * 1e-3) / 1e9, 3)}
        if prec == L.PREC_FP64:
            s.set_timing(True)
            s.solve(rhs, p=p, tol=tol, maxit=300)
            k1, k2, _ = s.last_timing()
            mode = d["coefficients"]
            sweeps = s.tile_form_ex()[2]
            b1, b2 = iteration_bytes(mode, sweeps)
            d["sweeps_per_iteration"] = sweeps
            d["kernel_k1"] = {"avg_ms": round(k1, 4),
                              "achieved_GBps": (round(b1 * case.ncells / (k1 * 1e-3) / 1e9, 1)
                                                if b1 else None)}
            d["kernel_k2"] = {"avg_ms": round(k2, 4),
                              "achieved_GBps": round(b2 * case.ncells / (k2 * 1e-3) / 1e9, 1)}
            d["frac_k2"] = round(d["kernel_k2"]["achieved_GBps"] / HBM_PEAK_GBS, 4)
        s.close()
        out[name] = d
        log(f"  {name}: {st['iters']} iters, {ms:.0f} ms, {d['Gcell_iter_per_s']:.1f} Gcell-iter/s")
        del p
    return out


def bench_project(case, rho, mask, p64, dev):
    """The projection after the solve: u -= dt (1/rho) grad p on the faces
    of the same 512^3 field, then the divergence norm of the result."""
    import torch
    from paper_1410_1942_amd.solver import Solver
    log("projection")
    s = Solver(rho, mask, case.bc, case.h)
    u0 = torch.from_numpy(case.u).to(dev)
    v0 = torch.from_numpy(case.v).to(dev)
    w0 = torch.from_numpy(case.w).to(dev)
    u, v, w = u0.clone(), v0.clone(), w0.clone()
    d0 = s.divergence(u, v, w)
    s.project(p64, case.dt, u, v, w)            # warm
    u.copy_(u0); v.copy_(v0); w.copy_(w0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.project(p64, case.dt, u, v, w)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    t = time.perf_counter()
    d1 = s.divergence(u, v, w)
    td = time.perf_counter() - t
    s.close()
    cells = case.ncells
    # algorithmic bytes: project reads p, the class byte and the three face
    # arrays and writes them back; divergence reads the faces and the density
    bp, bd = (8 + 1 + 24 + 24) * cells, (24 + 8) * cells
    log(f"  project {tp*1e3:.2f} ms ({bp/tp/1e9:.0f} GB/s), divergence {td*1e3:.2f} ms, "
        f"ratio {d1[0]/d0[0]:.3e}")
    return {"project_ms": round(tp * 1e3, 3), "project_GBps": round(bp / tp / 1e9, 1),
            "divergence_ms": round(td * 1e3, 3), "divergence_GBps": round(bd / td / 1e9, 1),
            "div_l2_before": d0[0], "div_l2_after": d1[0],
            "div_ratio": d1[0] / d0[0], "div_max_after": d1[1]}


def bench_rk2(case, rho, mask, dev, tol, shift):
    """Pressure half of one two-stage Runge-Kutta step on the same field:
    P* from rho(phi^k), u*, coefficients rebuilt for rho(phi*) (the surface
    modes advanced by `shift` rad), P^{k+1} warm-started from P*, u^{k+1}.
    The second stage is repeated cold to show what the warm start saves."""
    import torch
    from paper_1410_1942_amd import fields as F
    from paper_1410_1942_amd import rk2
    from paper_1410_1942_amd.solver import Solver
    log("rk2 stage pair")
    rho_s = torch.from_numpy(F.stage_density(case.nx, case.ny, case.nz, surface_seed=1,
                                             velocity_seed=2, phase_shift=shift)).to(dev)
    uk = [torch.from_numpy(a).to(dev) for a in (case.u, case.v, case.w)]
    s = Solver(rho, mask, case.bc, case.h)
    rhs = torch.empty_like(rho)
    torch.cuda.synchronize()
    t = time.perf_counter()
    p, un, info = rk2.pressure_pair(s, None, rho_s, mask, uk, case.dt, tol=tol, rhs=rhs,
                                    timed=True)
    torch.cuda.synchronize()
    total = (time.perf_counter() - t) * 1e3
    d0, _ = s.divergence(*uk)
    d1, _ = s.divergence(*un)
    # the same second-stage equation from x0 = 0
    pc = torch.empty_like(p)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, stc = s.solve(rhs, p=pc, tol=tol, warm=False)
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - t) * 1e3
    s.close()
    st1, st2, ms = info["stage1"], info["stage2"], info["ms"]
    log(f"  stage 1 {st1['iters']} iters {ms['stage1_solve']:.0f} ms; rebuild "
        f"{ms['rebuild_star']:.1f} ms; stage 2 warm {st2['iters']} iters "
        f"{ms['stage2_solve']:.0f} ms (cold {stc['iters']} iters {cold_ms:.0f} ms); "
        f"pair {total:.0f} ms, div ratio {d1 / d0:.2e}")
    return {"phase_shift": shift, "changed_cells": int((rho_s != rho).sum().item()),
            "stage1_iters": st1["iters"], "stage2_iters_warm": st2["iters"],
            "stage2_iters_cold": stc["iters"],
            "ms": {k: round(v, 2) for k, v in ms.items()}, "pair_ms": round(total, 1),
            "stage2_cold_ms": round(cold_ms, 1),
            "warm_saving": round(1.0 - st2["iters"] / max(stc["iters"], 1), 3),
            "div_ratio_final": d1 / d0}


def bench_batch(nsolves):
    """64 independent solves of uneven sizes (edges log-uniform in [16,128],
    own surface, ratio 1000/1.2, FP32+IR to 1e-8) resident in one batch:
    every launch covers all of them.  Compared with the same solves run one
    after another through single-solve contexts."""
    import torch
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd import fields as F
    from paper_1410_1942_amd import serve
    from paper_1410_1942_amd.solver import Batch, Solver
    log(f"batch of {nsolves}")
    cases = [(F.batch_member(i, keep_velocity=False), 1e-8) for i in range(nsolves)]
    reqs = serve.make_requests(cases, [0.0] * nsolves)
    cells = sum(r.cells for r in reqs)
    probe = Batch(1 << 20, 1, precision=L.PREC_FP32_IR)
    need = sum(probe.footprint(tuple(r.rho.shape), r.h) for r in reqs) + (8 << 20)
    probe.close()

    def run_batch():
        b = Batch(need, nsolves, precision=L.PREC_FP32_IR, check_every=16)
        slots = []
        for r in reqs:
            r.p = torch.empty_like(r.rhs)
            code, sl = b.admit(r.rho, r.mask, r.bc, r.h, r.rhs, r.p, tol=r.tol)
            assert code == L.OK
            slots.append(sl)
        while b.step(1):
            pass
        sts = [b.poll(sl)[1] for sl in slots]
        b.close()
        return sts

    run_batch()                                   # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    sts = run_batch()
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    cell_iters = sum(r.cells * st["iters"] for r, st in zip(reqs, sts))
    # the same solves one at a time
    t = time.perf_counter()
    for r in reqs:
        s = Solver(r.rho, r.mask, r.bc, r.h, precision=L.PREC_FP32_IR)
        s.solve(r.rhs, tol=r.tol)
        s.close()
    torch.cuda.synchronize()
    ts = time.perf_counter() - t
    ok = all(st["status"] == 0 and st["rel_res_true"] <= 1e-8 for st in sts)
    log(f"  batch {tb*1e3:.0f} ms, sequential {ts*1e3:.0f} ms, all ok {ok}")
    return {
        "solves": nsolves, "cells": cells, "precision": "fp32+ir", "tol": 1e-8,
        "ms": round(tb * 1e3, 2), "solves_per_s": round(nsolves / tb, 2),
        "Gcell_iter_per_s": round(cell_iters / tb / 1e9, 3),
        "sequential_ms": round(ts * 1e3, 2), "speedup_vs_sequential": round(ts / tb, 3),
        "all_converged": ok,
        "inner_iters_max": max(st["iters"] for st in sts),
    }


def bench_serve(nreq, nwarm):
    """Served stream: requests with edges log-uniform in [24,192], wedge hull
    with p = 0.5, tol 1e-6 or 1e-8, FP32+IR; first a capacity run (all
    waiting at t = 0) on a prefix, then Poisson arrivals at 75 % of that
    capacity: nwarm warm-up requests, then nreq reported ones.  Requests
    are generated one at a time and uploaded at once (host copies dropped)."""
    import torch
    from paper_1410_1942_amd import fields as F
    from paper_1410_1942_amd import serve
    total = nwarm + nreq
    log(f"served stream of {nwarm} + {nreq}")
    reqs = [serve.make_requests([F.served_request(i, keep_velocity=False)], [0.0])[0]
            for i in range(total)]
    torch.cuda.synchronize()
    arena = 24 << 30
    ncap = min(total, 48)
    srv = serve.Server(arena, max_slots=64)
    srv.run([_fresh(r, 0.0) for r in reqs[: min(8, ncap)]], realtime=False)   # warm
    cap = srv.run([_fresh(r, 0.0) for r in reqs[:ncap]], realtime=False)
    rate = 0.75 * cap.solves_per_s
    arrivals = F.arrival_times(total, rate=rate, seed=7)
    reqs = [_fresh(r, float(t)) for r, t in zip(reqs, arrivals)]
    torch.cuda.synchronize()
    rep = srv.run(reqs, realtime=True, warmup=nwarm)
    srv.close()
    log(f"  capacity {cap.solves_per_s:.1f}/s; at {rate:.1f}/s arrivals: "
        f"{rep.solves_per_s:.1f}/s, p50 {rep.p50_ms:.1f} ms, p99 {rep.p99_ms:.1f} ms")
    d = rep.as_dict()
    d.update({"arrival_rate_per_s": round(rate, 2), "warmup_requests": nwarm,
              "capacity_solves_per_s": round(cap.solves_per_s, 2),
              "capacity_requests": ncap, "precision": "fp32+ir",
              "arena_GiB": arena / 2**30})
    return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in d.items()}


def host_cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _fresh(r, arrival):
    """The same request (shared device inputs) with no result yet."""
    import dataclasses
    from paper_1410_1942_amd import _lib as L
    return dataclasses.replace(r, arrival=arrival, p=None, admitted=float("nan"),
                               done=float("nan"), status=L.PENDING, iters=0, outer=0,
                               rel_res=float("nan"))


def kernel_sha():
    """Hash of the device source with comments and blank lines removed, so
    that a counter summary stays matched across comment-only edits."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("kernels.hip", "pcg_types.h"):
        src = open(os.path.join(ROOT, "paper_1410_1942_amd", "csrc", f)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("\n".join(l.strip() for l in src.splitlines() if l.strip()).encode())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
