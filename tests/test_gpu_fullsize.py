"""The full-size workloads, in the launch configuration the benchmark times,
through the C ABI (GPU).

* The 512^3 two-phase wedge tank, FP64 and FP32 stencil with FP64
  refinement: the oracle's relative residual recomputed over every cell, hull
  cells exactly 0, and the error against the oracle's own 1e-12 solution,
  read at a stored strided sample (the oracle takes about an hour on this
  size, so its sample is written once by tests/golden/make_fullsize_golden.py).
* The 64-solve uneven batch and 40 requests of the served recipe: every
  member against the oracle solved to 1e-12, element by element.
"""
import sys

import numpy as np
import pytest

from tests import _ref

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_wedge_512_fp64_and_ir(orc, F):
    """Both forms reach 1e-8 by the oracle's residual; their error against
    the oracle's solution is stated at 1e-8 and held to 1e-6 at 1e-9."""
    import torch
    from paper_1410_1942_amd.solver import Solver
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    _say("case wedge512: generating")
    case = F.config_wedge(512, keep_velocity=False)
    meta, ref = _ref.golden(512)
    assert _ref.input_digest(case) == meta["input_sha256"]
    rho = torch.from_numpy(case.rho).to(dev)
    mask = torch.from_numpy(case.mask).to(dev)
    rhs = torch.from_numpy(case.rhs).to(dev)
    errs = {}
    for tol in (1e-8, 1e-9):
        for prec, name in ((0, "fp64"), (1, "fp32+ir")):
            _say(f"case wedge512 {name} tol={tol:g}: solving")
            s = Solver(rho, mask, case.bc, case.h, precision=prec)   # default tiles and grid
            try:
                p, st = s.solve(rhs, tol=tol)
            finally:
                s.close()
            torch.cuda.synchronize()
            assert st["status"] == 0, (name, st)
            ph = p.cpu().numpy()
            del p
            err = _ref.err_vs_golden(ph, meta, ref)
            _say(f"  iters {st['iters']}, err vs oracle {err:.3e}")
            errs[(name, tol)] = err
            if tol == 1e-8:
                rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, ph)
                _say(f"  rel res {rr:.4e} (reported {st['rel_res_true']:.4e})")
                assert rr <= tol, (name, rr)
                assert abs(rr - st["rel_res_true"]) <= 1e-6 * rr, (name, rr, st)
                assert not ph[case.mask.astype(bool)].any()
    for name in ("fp64", "fp32+ir"):
        assert errs[(name, 1e-8)] <= 1e-5, errs
        assert errs[(name, 1e-9)] <= 1e-6, errs


def _member_errors(orc, cases, ps):
    """max |p - p_oracle| / max |p_oracle| per member, the oracle solved to
    1e-12 (several solves at once on the host's cores)."""
    refs = _ref.solve_many(orc, cases)
    return [float(np.abs(p - r).max() / np.abs(r).max()) for p, r in zip(ps, refs)]


def _batch_run(reqs, max_slots):
    """Admit every request into one batch of max_slots and step to the end;
    returns the statuses."""
    import torch
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd.solver import Batch
    probe = Batch(1 << 20, 1, precision=L.PREC_FP32_IR)
    need = sum(probe.footprint(tuple(r.rho.shape), r.h) for r in reqs) + (16 << 20)
    probe.close()
    b = Batch(need, max_slots, precision=L.PREC_FP32_IR)
    try:
        slots = []
        for r in reqs:
            r.p = torch.empty_like(r.rhs)
            code, s = b.admit(r.rho, r.mask, r.bc, r.h, r.rhs, r.p, tol=r.tol)
            assert code == L.OK, code
            slots.append(s)
        while b.step(1):
            pass
        sts = [b.poll(s)[1] for s in slots]
        torch.cuda.synchronize()
    finally:
        b.close()
    return sts


def test_batch_of_64_full_size(orc, F):
    """The benchmark's batch: 64 solves with edges log-uniform in [16, 128],
    FP32+IR to 1e-8, in one resident batch.  Each meets the reference's
    residual; the smallest, the median and the largest equal their solo
    runs (a batch of one) bit for bit."""
    import torch
    from paper_1410_1942_amd import serve
    assert torch.cuda.is_available()
    cases = [(F.batch_member(i, keep_velocity=False), 1e-8) for i in range(64)]
    reqs = serve.make_requests(cases, [0.0] * 64)
    _say("case batch of 64: " + " ".join("x".join(map(str, c.shape)) for c, _ in cases[:8]) + " ...")
    sts = _batch_run(reqs, 64)
    ps = [r.p.cpu().numpy() for r in reqs]
    for i, ((case, tol), p, st) in enumerate(zip(cases, ps, sts)):
        assert st["status"] == 0, (i, st)
        rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, p)
        assert rr <= tol, (i, rr)
    _say("  oracle solves of the 64 members")
    errs = _member_errors(orc, [c for c, _ in cases], ps)
    worst = int(np.argmax(errs))
    _say(f"  max err vs oracle {errs[worst]:.3e} (member {worst}, "
         f"{'x'.join(map(str, cases[worst][0].shape))})")
    assert max(errs) <= 1e-6, errs
    order = sorted(range(64), key=lambda i: reqs[i].cells)
    for i in (order[0], order[32], order[-1]):
        _say(f"  solo run of member {i} ({reqs[i].cells} cells)")
        solo = serve.make_requests([cases[i]], [0.0])
        st1 = _batch_run(solo, 1)[0]
        assert st1["iters"] == sts[i]["iters"], (i, st1, sts[i])
        assert torch.equal(solo[0].p, reqs[i].p), i


def test_served_requests_full_size(orc, F):
    """The served recipe at its real sizes (edges log-uniform in [24, 192],
    a wedge hull on half of the requests, tolerance 1e-6 or 1e-8): 40
    requests through the server, all waiting at the start.  Each meets its
    own tolerance by the reference's residual, hull cells 0."""
    import torch
    from paper_1410_1942_amd import serve
    assert torch.cuda.is_available()
    cases = [F.served_request(i, keep_velocity=False) for i in range(40)]
    assert any(c.mask.any() for c, _ in cases) and not all(c.mask.any() for c, _ in cases)
    reqs = serve.make_requests(cases, [0.0] * 40)
    _say("case served 40: largest " + str(max(c.shape for c, _ in cases)))
    srv = serve.Server(24 << 30, max_slots=64)
    try:
        srv.run(reqs, realtime=False)
    finally:
        srv.close()
    torch.cuda.synchronize()
    ps = [r.p.cpu().numpy() for r in reqs]
    for i, ((case, tol), r, p) in enumerate(zip(cases, reqs, ps)):
        assert r.status == 0, (i, r.status)
        rr = orc.relres(case.rho, case.mask, case.bc, case.h, case.rhs, p)
        assert rr <= tol, (i, rr, tol)
        if case.mask is not None:
            assert not p[case.mask.astype(bool)].any()
    _say("  oracle solves of the 40 requests")
    errs = _member_errors(orc, [c for c, _ in cases], ps)
    for tol_i in (1e-8, 1e-6):
        e = [err for err, (_, t) in zip(errs, cases) if t == tol_i]
        _say(f"  tol {tol_i:g}: {len(e)} requests, max err vs oracle {max(e):.3e}")
    for err, (case, tol) in zip(errs, cases):
        # at 1e-8 the 1e-6 error bar; a 1e-6 request is held to the same
        # multiple of its tolerance
        assert err <= 100.0 * tol, (case.name, err, tol)
