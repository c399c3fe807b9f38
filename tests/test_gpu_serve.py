"""Served stream: requests arriving while others run are admitted as memory
and slots free up; every result equals its solo solve bitwise and meets the
reference's residual (GPU)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def test_served_stream_alone_vs_mix(orc, F, torch_mod):
    torch = torch_mod
    from paper_1410_1942_amd import serve
    from paper_1410_1942_amd.solver import Batch
    from paper_1410_1942_amd import _lib as L
    cases = [F.served_request(i, lo=16, hi=40) for i in range(12)]
    arrivals = F.arrival_times(len(cases), rate=400.0)
    reqs = serve.make_requests(cases, arrivals)
    # an arena that holds only a few requests at once forces queueing
    srv = serve.Server(arena_bytes=8 << 20, max_slots=8)
    rep = srv.run(reqs)
    srv.close()
    print(rep, flush=True)
    assert rep.statuses == {0: len(reqs)}
    assert 0 < rep.p50_ms <= rep.p99_ms
    assert rep.max_resident >= 2            # solves overlapped on the device
    for r, (case, tol) in zip(sorted(reqs, key=lambda q: q.arrival), cases):
        p = r.p.cpu().numpy()
        rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, p)
        assert rr <= tol
        # alone: a batch of one with the same options
        b = Batch(64 << 20, 1, precision=L.PREC_FP32_IR, check_every=5)
        p1 = torch.empty_like(r.rhs)
        code, s = b.admit(r.rho, r.mask, r.bc, r.h, r.rhs, p1, tol=r.tol)
        while b.step(1):
            pass
        code, st = b.poll(s)
        assert code == 0 and st["iters"] == r.iters
        assert np.array_equal(p1.cpu().numpy(), p)
        b.close()


def test_capacity_mode_and_refused_request(F, torch_mod):
    torch = torch_mod
    from paper_1410_1942_amd import serve
    cases = [F.served_request(i, lo=16, hi=32) for i in range(40, 46)]
    reqs = serve.make_requests(cases, [0.0] * len(cases))
    reqs[2].rho = reqs[2].rho.clone()
    reqs[2].rho.view(-1)[0] = -5.0          # invalid density: refused alone
    if reqs[2].mask is not None:
        reqs[2].mask = reqs[2].mask.clone()
        reqs[2].mask.view(-1)[0] = 0
    srv = serve.Server(arena_bytes=64 << 20, max_slots=16, flags=0)
    rep = srv.run(reqs, realtime=False)
    srv.close()
    assert rep.statuses.get(-2) == 1 and rep.statuses.get(0) == len(reqs) - 1
