"""Served pressure solves: a continuous-batching request loop.

Requests (a density field, optional hull mask, source and tolerance) arrive
at given times.  The loop admits waiting requests first-in first-out while
the batch's arena has room for their footprint and a slot is free
(``pcg_batch_admit`` refuses with PCG_EBUSY otherwise), with a bounded
bypass: requests behind a head that does not fit may go first, a limited
number of times per head (``AdmissionQueue``).  It replays the captured
iterations of every resident solve together (``pcg_batch_step``), and
retires finished solves as soon as their status turns final, recording the
latency from arrival to completion.  The pressure of each request stays a
device tensor.

All solver work runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .solver import Batch


@dataclasses.dataclass
class Request:
    rho: torch.Tensor
    mask: Optional[torch.Tensor]
    rhs: torch.Tensor
    bc: tuple
    h: float
    tol: float
    arrival: float = 0.0          # seconds after the start of the run
    maxit: int = 1000000
    # filled by the server
    p: Optional[torch.Tensor] = None
    admitted: float = float("nan")
    done: float = float("nan")
    status: int = L.PENDING
    iters: int = 0
    outer: int = 0
    rel_res: float = float("nan")

    @property
    def cells(self) -> int:
        return self.rho.numel()

    @property
    def latency(self) -> float:
        return self.done - self.arrival


ADMITTED, BUSY, REFUSED = "admitted", "busy", "refused"


class AdmissionQueue:
    """Waiting requests, admitted first-in first-out with a bounded bypass.

    ``admit(try_admit)`` offers requests to ``try_admit(r)``, which answers
    ADMITTED, BUSY (no room or slot now) or REFUSED (the request is invalid
    and fails alone).  The head is offered first, then the next ones while
    they are admitted or refused.  When the head is BUSY, up to ``lookahead``
    requests behind it are offered and those that fit go first; each one
    that passes counts against the head, and once ``max_bypass`` have passed
    it nothing more is admitted before it, so a large request cannot starve.
    Returns the (request, answer) pairs of the requests that left the queue,
    in the order they left.  Host logic only: no device work."""

    def __init__(self, lookahead: int = 8, max_bypass: int = 16):
        self.q: collections.deque = collections.deque()
        self.lookahead = lookahead
        self.max_bypass = max_bypass
        self.passed = 0          # requests admitted ahead of the current head

    def __len__(self):
        return len(self.q)

    def push(self, r):
        self.q.append(r)

    def admit(self, try_admit):
        out = []
        while self.q:
            ans = try_admit(self.q[0])
            if ans == BUSY:
                break
            out.append((self.q.popleft(), ans))
            self.passed = 0
        i = 1
        while (self.q and i < len(self.q) and i <= self.lookahead
               and self.passed < self.max_bypass):
            ans = try_admit(self.q[i])
            if ans == BUSY:
                i += 1
                continue
            out.append((self.q[i], ans))
            del self.q[i]
            if ans == ADMITTED:
                self.passed += 1
        return out


@dataclasses.dataclass
class ServeReport:
    n: int
    wall_s: float
    solves_per_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    max_resident: int
    cell_iters_per_s: float
    statuses: dict

    def as_dict(self):
        return dataclasses.asdict(self)


class Server:
    def __init__(self, arena_bytes: int, max_slots: int = 64,
                 precision: int = L.PREC_FP32_IR, replays_per_step: int = 1,
                 check_every: int = 16, flags: int = 0, lookahead: int = 8,
                 max_bypass: int = 16, **opt_kw):
        self.batch = Batch(arena_bytes, max_slots, precision=precision,
                           check_every=check_every, **opt_kw)
        self.replays = replays_per_step
        self.flags = flags
        self.lookahead = lookahead
        self.max_bypass = max_bypass

    def close(self):
        self.batch.close()

    def run(self, requests: Sequence[Request], clock=time.perf_counter,
            realtime: bool = True, warmup: int = 0) -> ServeReport:
        """Serve every request; with realtime=False all requests are treated
        as already waiting at t = 0 (capacity measurement).  The first
        `warmup` requests (in arrival order) are served but left out of the
        report, whose window runs from the first reported arrival to the
        last reported completion."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        waiting = AdmissionQueue(self.lookahead, self.max_bypass)
        resident = {}                       # slot -> request
        nxt = 0
        max_res = 0
        t0 = clock()
        now = 0.0
        while nxt < len(reqs) or waiting or resident:
            now = clock() - t0
            while nxt < len(reqs) and (not realtime or reqs[nxt].arrival <= now):
                if not realtime:
                    reqs[nxt].arrival = 0.0
                waiting.push(reqs[nxt])
                nxt += 1

            def try_admit(r):
                if r.p is None:
                    r.p = torch.empty_like(r.rhs)
                try:
                    code, slot = self.batch.admit(r.rho, r.mask, r.bc, r.h, r.rhs,
                                                  r.p, tol=r.tol, maxit=r.maxit,
                                                  flags=self.flags)
                except L.PCGError as e:      # refused request fails alone
                    r.status = e.code
                    r.admitted = r.done = clock() - t0
                    return REFUSED
                if code == L.EBUSY:
                    return BUSY
                r.admitted = clock() - t0
                resident[slot] = r
                return ADMITTED

            waiting.admit(try_admit)
            if waiting and not resident:
                raise RuntimeError("request larger than the arena")
            max_res = max(max_res, len(resident))
            if not resident:
                if nxt < len(reqs):          # idle until the next arrival
                    delay = reqs[nxt].arrival - (clock() - t0)
                    if delay > 0:
                        time.sleep(delay)
                continue
            self.batch.step(self.replays)
            t_done = clock() - t0
            for slot in list(resident):
                code, st = self.batch.poll(slot)
                if code == L.PENDING:
                    continue
                r = resident.pop(slot)
                r.done = t_done
                r.status = st["status"]
                r.iters = st["iters"]
                r.outer = st["outer_iters"]
                r.rel_res = st["rel_res_true"]
                self.batch.release(slot)
        rep = reqs[warmup:] if warmup < len(reqs) else reqs
        wall = max(r.done for r in rep) - min(r.arrival for r in rep)
        lat = np.array([r.latency for r in rep]) * 1e3
        statuses = collections.Counter(int(r.status) for r in rep)
        cell_iters = sum(r.cells * r.iters for r in rep)
        return ServeReport(
            n=len(rep), wall_s=wall, solves_per_s=len(rep) / wall,
            p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
            mean_ms=float(lat.mean()), max_resident=max_res,
            cell_iters_per_s=cell_iters / wall, statuses=dict(statuses))


def make_requests(cases_and_tols, arrivals: Sequence[float], device="cuda"
                  ) -> List[Request]:
    """Upload generated cases (fields.Case, tol) to the device as requests."""
    out = []
    for (case, tol), t in zip(cases_and_tols, arrivals):
        mask = (torch.from_numpy(case.mask).to(device)
                if case.mask is not None and case.mask.any() else None)
        out.append(Request(rho=torch.from_numpy(case.rho).to(device), mask=mask,
                           rhs=torch.from_numpy(case.rhs).to(device),
                           bc=case.bc, h=case.h, tol=tol, arrival=float(t)))
    return out
