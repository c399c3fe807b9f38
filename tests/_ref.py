"""Oracle references for the full-size GPU tests.

* Stored samples of the oracle's solution of the large wedge tanks
  (``tests/golden/wedge{256,512}_oracle.*``, written by
  ``tests/golden/make_fullsize_golden.py`` from the oracle alone), with a
  digest of the generator's inputs so a changed generator is noticed.
* Many independent oracle solves at once (a batch's or a server's members):
  a few host threads, each running the oracle with a share of the cores.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import json
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(n: int):
    """(metadata, sample) of the stored oracle solution of the n^3 wedge tank."""
    base = os.path.join(GOLD, f"wedge{n}_oracle")
    with open(base + ".json") as f:
        meta = json.load(f)
    return meta, np.load(base + ".npy")


def input_digest(case) -> str:
    h = hashlib.sha256()
    for a in (case.rho, case.mask, case.rhs):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def sample(p, meta):
    o, s = meta["offset"], meta["stride"]
    return p[o::s, o::s, o::s]


def err_vs_golden(p, meta, ref) -> float:
    """max |p - p_oracle| / max |p_oracle| over the stored sample cells."""
    return float(np.abs(sample(p, meta) - ref).max() / meta["p_max_abs"])


def solve_many(orc, cases, tol=1e-12, workers=4):
    """Oracle solutions of (case, ...) tuples' cases, in order."""
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    per = max(1, min(16, ncpu) // workers)

    def one(case):
        orc.set_threads(per)
        r = orc.pcg(case.rho, case.mask, case.bc, case.h, case.rhs, tol=tol)
        assert r.status == orc.OK, (case.name, r.status)
        return r.p

    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(one, cases))
