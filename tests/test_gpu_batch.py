"""Batched and continuously admitted solves through pcg_batch_* (GPU).

Each solve's arithmetic depends only on its own grid, tile shape and data,
so its result must be bitwise the same alone (a batch of one) and in any
mix, admitted at any time.  Each result also meets the reference's
residual.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0")


class Req:
    def __init__(self, torch, dev, case, tol, flags=0):
        self.case, self.tol, self.flags = case, tol, flags
        self.rho = torch.from_numpy(case.rho).to(dev)
        self.mask = torch.from_numpy(case.mask).to(dev)
        self.rhs = torch.from_numpy(case.rhs).to(dev)
        self.p = torch.zeros_like(self.rhs)


def _members(F, idx, lo=16, hi=48):
    return [F.batch_member(i, lo=lo, hi=hi) for i in idx]


def _run_batch(torch_dev, reqs, precision, arena=1 << 30, max_slots=64,
               stagger=None, **kw):
    """Admit all (or in waves given by stagger = list of (replays, n_admit)),
    step until every solve finishes; returns stats per request."""
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Batch
    from paper_1410_1942_amd import _lib as L
    b = Batch(arena, max_slots, precision=precision, **kw)
    slots = {}
    pending = list(range(len(reqs)))
    waves = stagger or [(0, len(reqs))]
    for replays, n_admit in waves:
        for _ in range(replays):
            b.step(1)
        for _ in range(n_admit):
            if not pending:
                break
            i = pending.pop(0)
            r = reqs[i]
            code, s = b.admit(r.rho, r.mask, r.case.bc, r.case.h, r.rhs, r.p,
                              tol=r.tol, flags=r.flags)
            assert code == L.OK, code
            slots[i] = s
    assert not pending
    for _ in range(100000):
        if b.step(1) == 0:
            break
    stats = {}
    for i, s in slots.items():
        code, st = b.poll(s)
        stats[i] = st
        b.release(s)
    torch.cuda.synchronize()
    b.close()
    return stats


def _solo(torch_dev, req, precision, **kw):
    torch, dev = torch_dev
    r2 = Req(torch, dev, req.case, req.tol, req.flags)
    st = _run_batch(torch_dev, [r2], precision, max_slots=1, **kw)[0]
    return r2.p.cpu().numpy(), st


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "ir"])
def test_alone_equals_mix(orc, F, torch_dev, precision):
    torch, dev = torch_dev
    cases = _members(F, range(6))
    reqs = [Req(torch, dev, c, 1e-8) for c in cases]
    _say(f"batch of {len(reqs)} precision={precision}: "
         + " ".join(str(c.shape) for c in cases))
    stats = _run_batch(torch_dev, reqs, precision)
    for i, r in enumerate(reqs):
        st = stats[i]
        assert st["status"] == 0, (i, st)
        p = r.p.cpu().numpy()
        rr = orc.relres(r.case.rho, r.case.mask, r.case.bc, r.case.h, r.case.rhs, p)
        assert rr <= 1e-8, (i, rr)
        alone, st1 = _solo(torch_dev, r, precision)
        assert st1["iters"] == st["iters"], (i, st1, st)
        assert np.array_equal(alone, p), i


def test_staggered_admission_and_mixed_tolerances(orc, F, torch_dev):
    """Solves join while others run (continuous batching); results equal
    the solo runs bitwise; tolerances differ per request."""
    torch, dev = torch_dev
    cases = _members(F, range(10, 18), lo=20, hi=56)
    tols = [1e-6 if i % 2 else 1e-8 for i in range(len(cases))]
    reqs = [Req(torch, dev, c, t) for c, t in zip(cases, tols)]
    _say("staggered: " + " ".join(str(c.shape) for c in cases))
    stats = _run_batch(torch_dev, reqs, 1, stagger=[(0, 3), (2, 2), (3, 3)])
    for i, r in enumerate(reqs):
        assert stats[i]["status"] == 0
        p = r.p.cpu().numpy()
        rr = orc.relres(r.case.rho, r.case.mask, r.case.bc, r.case.h, r.case.rhs, p)
        assert rr <= r.tol
        alone, _ = _solo(torch_dev, r, 1)
        assert np.array_equal(alone, p), i


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "ir"])
def test_mixed_coefficient_modes(orc, F, torch_dev, precision):
    """Solves coded by density class and solves reading per-cell densities
    in one batch: the set-up and residual actions of every slot run in the
    first coefficient mode's launch, pass A and B in each slot's own.  Each
    result is bitwise its solo run's (a batch of one launches the set-up
    actions on their own)."""
    torch, dev = torch_dev
    from paper_1410_1942_amd import _lib as L
    cases = _members(F, range(20, 26), lo=18, hi=44)
    reqs = [Req(torch, dev, c, 1e-8, L.NO_DENSITY_CLASSES if i % 2 else 0)
            for i, c in enumerate(cases)]
    _say(f"mixed modes precision={precision}: " + " ".join(str(c.shape) for c in cases))
    stats = _run_batch(torch_dev, reqs, precision, stagger=[(0, 2), (3, 2), (2, 2)])
    for i, r in enumerate(reqs):
        assert stats[i]["status"] == 0, (i, stats[i])
        p = r.p.cpu().numpy()
        rr = orc.relres(r.case.rho, r.case.mask, r.case.bc, r.case.h, r.case.rhs, p)
        assert rr <= 1e-8, (i, rr)
        alone, st1 = _solo(torch_dev, r, precision)
        assert st1["iters"] == stats[i]["iters"], (i, st1, stats[i])
        assert np.array_equal(alone, p), i


def test_wedge_requests_in_mix(orc, F, torch_dev):
    """Served-stream style requests (some with a hull) in one batch."""
    torch, dev = torch_dev
    reqs = []
    for i in range(5):
        case, tol = F.served_request(i, lo=24, hi=48)
        reqs.append(Req(torch, dev, case, tol))
    assert any(r.case.mask.any() for r in reqs)
    stats = _run_batch(torch_dev, reqs, 1)
    for i, r in enumerate(reqs):
        assert stats[i]["status"] == 0
        rr = orc.relres(r.case.rho, r.case.mask, r.case.bc, r.case.h, r.case.rhs,
                        r.p.cpu().numpy())
        assert rr <= r.tol


def test_admission_budget_and_release(F, torch_dev):
    torch, dev = torch_dev
    from paper_1410_1942_amd.solver import Batch
    from paper_1410_1942_amd import _lib as L
    case = F.make_two_phase(40, 40, 40, surface_seed=1, velocity_seed=2)
    r = Req(torch, dev, case, 1e-8)
    b = Batch(1 << 24, 4, precision=1)
    fp = b.footprint(case.shape, case.h)
    assert fp > 28 * case.ncells
    n_fit = (b.arena.numel() - 4096) // fp
    slots = []
    for k in range(6):
        code, s = b.admit(r.rho, r.mask, case.bc, case.h, r.rhs,
                          torch.empty_like(r.rhs), tol=1e-8)
        if code == L.EBUSY:
            break
        slots.append(s)
    assert 1 <= len(slots) <= min(4, n_fit + 1)
    assert code == L.EBUSY
    b.release(slots.pop())
    code, s = b.admit(r.rho, r.mask, case.bc, case.h, r.rhs,
                      torch.empty_like(r.rhs), tol=1e-8)
    assert code == L.OK
    b.close()


def test_bad_request_fails_alone(orc, F, torch_dev):
    """A request with a NaN source fails with EDOMAIN without disturbing the
    others in the same launches; one with a bad density is refused at
    admission."""
    torch, dev = torch_dev
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import Batch
    cases = _members(F, range(20, 24))
    reqs = [Req(torch, dev, c, 1e-8) for c in cases]
    bad = reqs[1].rhs.clone()
    bad.view(-1)[7] = float("nan")
    reqs[1].rhs = bad
    stats = _run_batch(torch_dev, reqs, 0)
    assert stats[1]["status"] == L.EDOMAIN
    for i in (0, 2, 3):
        assert stats[i]["status"] == 0
        alone, _ = _solo(torch_dev, reqs[i], 0)
        assert np.array_equal(alone, reqs[i].p.cpu().numpy())
    b = Batch(1 << 26, 4, precision=0)
    rho = reqs[0].rho.clone()
    rho.view(-1)[3] = -1.0
    with pytest.raises(L.PCGError) as e:
        b.admit(rho, reqs[0].mask, cases[0].bc, cases[0].h, reqs[0].rhs,
                reqs[0].p, tol=1e-8)
    assert e.value.code == L.EDOMAIN
    b.close()
