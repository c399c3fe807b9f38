"""The C ABI library loads and exports what include/pcg.h declares; host-side
argument validation answers without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1410_1942_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pcg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pcg_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return L.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTED)


def test_strerror(lib):
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7, -8):
        assert lib.pcg_strerror(code)
    assert b"unknown" in lib.pcg_strerror(99)


def _g(nx, ny, nz, h=0.1):
    return L.Grid(nx, ny, nz, h)


def test_workspace_bytes_validation(lib):
    out = ctypes.c_size_t()
    o = L.Opts()
    assert lib.pcg_workspace_bytes(ctypes.byref(_g(32, 32, 32)), ctypes.byref(o),
                                   ctypes.byref(out)) == L.OK
    n = 32 ** 3
    # rho, z, three directions and (narrow plane tiles, one sweep per
    # iteration: the default at this size) the second z, in FP64
    assert out.value >= 48 * n
    assert out.value < 56 * n
    o.precision = L.PREC_FP32_IR
    out_ir = ctypes.c_size_t()
    assert lib.pcg_workspace_bytes(ctypes.byref(_g(32, 32, 32)), ctypes.byref(o),
                                   ctypes.byref(out_ir)) == L.OK
    assert 36 * n <= out_ir.value < 44 * n
    # consecutive-cell tiles drop the second z
    o.precision = L.PREC_FP64
    o.flags = L.FLAT_TILES
    assert lib.pcg_workspace_bytes(ctypes.byref(_g(32, 32, 32)), ctypes.byref(o),
                                   ctypes.byref(out)) == L.OK
    assert 40 * n <= out.value < 48 * n
    o.flags = 0
    for bad in (_g(0, 4, 4), _g(4, -1, 4), _g(4, 4, 4, 0.0), _g(4, 4, 4, float("nan"))):
        assert lib.pcg_workspace_bytes(ctypes.byref(bad), None, ctypes.byref(out)) == L.EINVAL
    big = _g(2048, 1024, 1024)
    assert lib.pcg_workspace_bytes(ctypes.byref(big), None, ctypes.byref(out)) == L.EUNSUPPORTED
    o2 = L.Opts()
    o2.precision = 7
    assert lib.pcg_workspace_bytes(ctypes.byref(_g(4, 4, 4)), ctypes.byref(o2),
                                   ctypes.byref(out)) == L.EINVAL
    o2 = L.Opts()
    o2.inner_tol = 1.5
    assert lib.pcg_workspace_bytes(ctypes.byref(_g(4, 4, 4)), ctypes.byref(o2),
                                   ctypes.byref(out)) == L.EINVAL


def test_setup_validation_without_device_work(lib):
    ctx = ctypes.c_void_p()
    g = _g(8, 8, 8)
    bc = L.BC()
    bc.kind[5] = L.BC_DIRICHLET
    fake = ctypes.c_void_p(0x1000)
    # null output, null rho, null workspace
    assert lib.pcg_setup(None, ctypes.byref(g), fake, None, ctypes.byref(bc), None,
                         fake, 1 << 20, None) == L.EINVAL
    assert lib.pcg_setup(ctypes.byref(ctx), ctypes.byref(g), None, None,
                         ctypes.byref(bc), None, fake, 1 << 20, None) == L.EINVAL
    assert lib.pcg_setup(ctypes.byref(ctx), ctypes.byref(g), fake, None,
                         ctypes.byref(bc), None, None, 1 << 20, None) == L.EINVAL
    # periodic z walls are not supported; a periodic wall without its
    # partner and unknown kinds are invalid
    bp = L.BC()
    bp.kind[4] = bp.kind[5] = L.BC_PERIODIC
    assert lib.pcg_setup(ctypes.byref(ctx), ctypes.byref(g), fake, None,
                         ctypes.byref(bp), None, fake, 1 << 20, None) == L.EUNSUPPORTED
    bq = L.BC()
    bq.kind[2] = L.BC_PERIODIC
    bq.kind[5] = L.BC_DIRICHLET
    assert lib.pcg_setup(ctypes.byref(ctx), ctypes.byref(g), fake, None,
                         ctypes.byref(bq), None, fake, 1 << 20, None) == L.EINVAL
    bx = L.BC()
    bx.kind[2] = 9
    assert lib.pcg_setup(ctypes.byref(ctx), ctypes.byref(g), fake, None,
                         ctypes.byref(bx), None, fake, 1 << 20, None) == L.EINVAL
    # workspace too small
    assert lib.pcg_setup(ctypes.byref(ctx), ctypes.byref(g), fake, None,
                         ctypes.byref(bc), None, fake, 1024, None) == L.ENOMEM
    assert not ctx.value


def test_null_handles(lib):
    st = L.Stats()
    assert lib.pcg_solve(None, None, None, 1e-8, 10, ctypes.byref(st)) == L.EINVAL
    assert lib.pcg_destroy(None) == L.OK
    assert lib.pcg_batch_step(None, 1, None) == L.EINVAL
    assert lib.pcg_batch_poll(None, 0, None) == L.EINVAL
    assert lib.pcg_batch_release(None, 0) == L.EINVAL
    assert lib.pcg_batch_destroy(None) == L.OK
    b = ctypes.c_void_p()
    assert lib.pcg_batch_create(ctypes.byref(b), ctypes.c_void_p(0x1000), 1 << 20, 0,
                                None, None) == L.EINVAL
    assert lib.pcg_last_timing(None, None, None, None) == L.EINVAL
    n = ctypes.c_int32()
    assert lib.pcg_density_classes(None, ctypes.byref(n)) == L.EINVAL
    ms = ctypes.c_double()
    assert lib.pcg_copy_probe(None, None, 0, 1, None, ctypes.byref(ms)) == L.EINVAL
    assert lib.pcg_triad_probe(None, None, None, 0, 1.0, 1, None, ctypes.byref(ms)) == L.EINVAL
    fake = ctypes.c_void_p(0x1000)
    assert lib.pcg_triad_probe(fake, fake, ctypes.c_void_p(0x2000), 16, 1.0, 1, None,
                               ctypes.byref(ms)) == L.EINVAL        # a aliases b


def _connectivity(lib, mask, bc):
    nz, ny, nx = mask.shape
    g = L.Grid(nx, ny, nz, 1.0 / nz)
    b = L.BC()
    for f in range(6):
        b.kind[f] = bc[f]
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return lib.pcg_check_connectivity(m.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(g), ctypes.byref(b))


def test_connectivity_check_matches_reference(lib, orc):
    """The library's run-based flood fill agrees with the reference's
    cell-by-cell search (regions, and regions without a Dirichlet wall) on
    random hulls, with and without periodic walls, and on hand-made
    pockets."""
    rng = np.random.default_rng(5)
    tank = (0, 0, 0, 0, 0, 1)
    kinds = [tank, (1, 0, 0, 0, 0, 0), (0, 0, 0, 1, 0, 0), (0,) * 6,
             (0, 0, 0, 0, 1, 0), (2, 2, 0, 0, 0, 1), (2, 2, 0, 0, 0, 0),
             (0, 0, 2, 2, 0, 0), (2, 2, 2, 2, 0, 0), (2, 2, 2, 2, 1, 0)]
    seen = {L.OK: 0, L.SINGULAR: 0, L.ESINGULAR: 0}
    for trial in range(300):
        shape = tuple(int(v) for v in rng.integers(1, 9, size=3))
        dens = rng.uniform(0.2, 0.7)
        mask = (rng.random(shape) < dens).astype(np.uint8)
        bc = kinds[trial % len(kinds)]
        regions, loose = orc.components(mask, bc)
        want = L.OK if loose == 0 else (L.SINGULAR if regions == 1 else L.ESINGULAR)
        got = _connectivity(lib, mask, bc)
        assert got == want, (trial, shape, bc, regions, loose)
        seen[want] += 1
    assert min(seen.values()) > 10, seen
    # rows longer than one 32-cell word of the packed mask: runs that cross
    # word boundaries, end on the row's last cell or exactly at a word end
    seen = {L.OK: 0, L.SINGULAR: 0, L.ESINGULAR: 0}
    for trial in range(120):
        nx = (31, 32, 33, 63, 64, 65, 97)[trial % 7]
        shape = (int(rng.integers(1, 5)), int(rng.integers(1, 5)), nx)
        dens = 0.04 if trial % 3 == 0 else rng.uniform(0.3, 0.75)   # sparse: one region
        mask = (rng.random(shape) < dens).astype(np.uint8)
        if trial % 5 == 0:
            mask[..., -1] = 0              # fluid up to the row's end
        bc = kinds[trial % len(kinds)]
        regions, loose = orc.components(mask, bc)
        want = L.OK if loose == 0 else (L.SINGULAR if regions == 1 else L.ESINGULAR)
        got = _connectivity(lib, mask, bc)
        assert got == want, (trial, shape, bc, regions, loose)
        seen[want] += 1
    assert min(seen.values()) > 3, seen
    # periodic x joins the two ends of a row: a hull wall across the middle
    # of a periodic tank leaves one region
    m = np.zeros((4, 3, 8), np.uint8)
    m[:, :, 3] = 1
    assert _connectivity(lib, m, (0,) * 6) == L.ESINGULAR
    assert _connectivity(lib, m, (2, 2, 0, 0, 0, 0)) == L.SINGULAR
    assert orc.components(m, (2, 2, 0, 0, 0, 0)) == (1, 1)
    # a sealed one-cell pocket at the bottom of an open tank
    m = np.zeros((6, 6, 6), np.uint8)
    m[0:2, 1:4, 1:4] = 1
    m[0, 2, 2] = 0
    assert _connectivity(lib, m, tank) == L.ESINGULAR
    m[0, 2, 2] = 1
    assert _connectivity(lib, m, tank) == L.OK
    # no hull: fine with any Dirichlet wall, singular with none
    assert lib.pcg_check_connectivity(None, ctypes.byref(_g(4, 4, 4)),
                                      ctypes.byref(_bc_of(tank))) == L.OK
    assert lib.pcg_check_connectivity(None, ctypes.byref(_g(4, 4, 4)),
                                      ctypes.byref(_bc_of((0,) * 6))) == L.SINGULAR


def _bc_of(kinds):
    b = L.BC()
    for f in range(6):
        b.kind[f] = kinds[f]
    return b


def test_tile_rules_roundtrip(lib):
    """The tile table is host state: set, read back, validation, and the
    workspace size follows the installed tile height."""
    from paper_1410_1942_amd import autotune
    saved = autotune.get_rules(0)
    try:
        autotune.set_rules(0, [[1000, 4, 256], [10**6, 8, 0], [10**9, 64, 512]])
        got = autotune.get_rules(0)
        assert [r[1:] for r in got] == [[4, 256], [8, 0], [64, 512]]
        assert got[-1][0] >= 2**62                 # last rule covers every size
        n = ctypes.c_int32()
        bad = (ctypes.c_int64 * 2)(10, 5)          # not increasing
        tz = (ctypes.c_int32 * 2)(4, 8)
        assert lib.pcg_set_tile_rules(0, 0, 2, bad, tz, None) == L.EINVAL
        assert lib.pcg_set_tile_rules(3, 0, 2, bad, tz, None) == L.EINVAL
        zero = (ctypes.c_int32 * 2)(0, 8)
        ok_mc = (ctypes.c_int64 * 2)(5, 10)
        assert lib.pcg_set_tile_rules(0, 0, 2, ok_mc, zero, None) == L.EINVAL
        assert lib.pcg_set_tile_rules(0, 4, 2, ok_mc, tz, None) == L.EINVAL
        assert lib.pcg_get_tile_rules(0, 4, 0, None, None, None, ctypes.byref(n)) == L.EINVAL
        # the batch and plane-tile tables are separate from the single-solve one
        batch_saved = autotune.get_rules(0, for_batches=True)
        autotune.set_rules(0, [[10**9, 16, 0]], for_batches=True)
        assert autotune.get_rules(0, for_batches=True)[0][1] == 16
        assert [r[1:] for r in autotune.get_rules(0)] == [[4, 256], [8, 0], [64, 512]]
        autotune.set_rules(0, batch_saved, for_batches=True)
        autotune.set_rules(0, [[10**9, 2, 0]], table=autotune.PLANE)
        assert autotune.get_rules(0, table=autotune.PLANE) == [[2**63 - 1, 2, 0]]
        assert [r[1:] for r in autotune.get_rules(0)] == [[4, 256], [8, 0], [64, 512]]
        narrow_saved = autotune.get_rules(0, table=autotune.NARROW)
        autotune.set_rules(0, [[10**9, 3, 0]], table=autotune.NARROW)
        assert autotune.get_rules(0, table=autotune.NARROW) == [[2**63 - 1, 3, 0]]
        assert autotune.get_rules(0, table=autotune.PLANE) == [[2**63 - 1, 2, 0]]
        autotune.set_rules(0, narrow_saved, table=autotune.NARROW)
        # workspace: partial sums scale with the number of tiles (tz = 64 -> fewer),
        # on consecutive-cell tiles from the single-solve table
        o = L.Opts()
        of = L.Opts()
        of.flags = L.FLAT_TILES
        w64 = ctypes.c_size_t()
        lib.pcg_workspace_bytes(ctypes.byref(_g(80, 128, 128)), ctypes.byref(of),
                                ctypes.byref(w64))
        # rows of 128 take plane tiles and the plane table (tz = 2 here)
        wp2 = ctypes.c_size_t()
        lib.pcg_workspace_bytes(ctypes.byref(_g(128, 128, 128)), ctypes.byref(o),
                                ctypes.byref(wp2))
        autotune.set_rules(0, [[10**9, 1, 0]])
        w1 = ctypes.c_size_t()
        lib.pcg_workspace_bytes(ctypes.byref(_g(80, 128, 128)), ctypes.byref(of),
                                ctypes.byref(w1))
        assert w1.value > w64.value
        wp = ctypes.c_size_t()
        lib.pcg_workspace_bytes(ctypes.byref(_g(128, 128, 128)), ctypes.byref(o),
                                ctypes.byref(wp))
        assert wp.value == wp2.value
        autotune.set_rules(0, [[10**9, 64, 0]], table=autotune.PLANE)
        lib.pcg_workspace_bytes(ctypes.byref(_g(128, 128, 128)), ctypes.byref(o),
                                ctypes.byref(wp))
        assert wp.value < wp2.value
    finally:
        autotune.set_rules(0, saved)
        autotune.install(arch="gfx950")


def test_stage_entry_points_reject_null_context(lib):
    """The Runge-Kutta stage entry points validate arguments on the host."""
    fake = ctypes.c_void_p(0x1000)
    st = L.Stats()
    assert lib.pcg_solve_ex(None, fake, fake, 1e-8, 10, 0, ctypes.byref(st)) == L.EINVAL
    assert lib.pcg_update_density(None, fake, None, 0) == L.EINVAL
    assert lib.pcg_rhs(None, 1e-3, fake, fake, fake, None, None, None, fake) == L.EINVAL
    assert lib.pcg_project_ex(None, fake, 1e-3, fake, fake, fake, None, None, None, 1.0,
                              fake, fake, fake) == L.EINVAL


def test_plane_and_tile_span_limits(lib):
    """Pass A addresses a tile's planes with 32-bit byte offsets: planes
    whose three-plane span of 8-byte values exceeds 2^32 bytes are refused,
    and the tile height is capped so tz + 2 planes fit."""
    out = ctypes.c_size_t()
    huge_plane = _g(16384, 16384, 2)            # 2^28 cells per plane
    assert lib.pcg_workspace_bytes(ctypes.byref(huge_plane), None,
                                   ctypes.byref(out)) == L.EUNSUPPORTED
    g = _g(4096, 4096, 64)                      # 2^27 bytes per plane: tz <= 30
    sizes = {}
    for tz in (16, 30, 31, 64):
        o = L.Opts()
        o.tz = tz
        assert lib.pcg_workspace_bytes(ctypes.byref(g), ctypes.byref(o),
                                       ctypes.byref(out)) == L.OK
        sizes[tz] = out.value
    assert sizes[31] == sizes[30] == sizes[64]  # clamped to 30
    assert sizes[16] != sizes[30]


def test_fraction_flag_host_rules(lib):
    """PCG_FRACTIONS reserves workspace for the four fraction arrays, is
    refused by batches, and pcg_set_fractions checks its context."""
    o = L.Opts()
    base, more = ctypes.c_size_t(), ctypes.c_size_t()
    g = _g(20, 16, 12)
    # fractions run consecutive-cell tiles: compare with that form
    o.flags = L.FLAT_TILES
    assert lib.pcg_workspace_bytes(ctypes.byref(g), ctypes.byref(o), ctypes.byref(base)) == L.OK
    o.flags = L.FRACTIONS
    assert lib.pcg_workspace_bytes(ctypes.byref(g), ctypes.byref(o), ctypes.byref(more)) == L.OK
    faces = 21 * 16 * 12 + 20 * 17 * 12 + 20 * 16 * 13 + 20 * 16 * 12
    assert 8 * faces <= more.value - base.value <= 8 * faces + 4 * 256
    b = ctypes.c_void_p()
    assert lib.pcg_batch_create(ctypes.byref(b), ctypes.c_void_p(0x1000), 1 << 20, 2,
                                ctypes.byref(o), None) == L.EINVAL
    assert lib.pcg_set_fractions(None, None, None, None, None) == L.EINVAL


def test_built_in_tile_rules_match_the_shipped_table():
    """The library's built-in rules (used when no table is installed) are
    the autotuner's table shipped with the package."""
    import json
    import subprocess
    import sys
    code = ("import json; from paper_1410_1942_amd import autotune, _lib as L; "
            "print(json.dumps({k: [list(r) for r in autotune.get_rules(p, table=b)] "
            "for k, p, b in (('fp64', L.PREC_FP64, 0), ('fp32_ir', L.PREC_FP32_IR, 0), "
            "('fp64_batch', L.PREC_FP64, 1), ('fp32_ir_batch', L.PREC_FP32_IR, 1), "
            "('fp64_plane', L.PREC_FP64, 2), ('fp32_ir_plane', L.PREC_FP32_IR, 2), "
            "('fp64_narrow', L.PREC_FP64, 3), ('fp32_ir_narrow', L.PREC_FP32_IR, 3))}))")
    env = dict(os.environ, PCGMI_TILE_TABLE="none")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, check=True,
                         capture_output=True, text=True).stdout
    built_in = json.loads(out.strip().splitlines()[-1])
    table = json.load(open(os.path.join(ROOT, "paper_1410_1942_amd", "tile_table.json")))["gfx950"]
    unbounded = lambda rules: [[None if r[0] >= 2**62 else r[0], r[1], r[2]] for r in rules]
    for k, rules in built_in.items():
        assert unbounded(rules) == unbounded(table[k]), k


def test_one_sweep_workspace(lib):
    """The one-sweep iteration (the default on plane tiles) adds one vector,
    the second z (FP64, or FP32 for the refinement), to the workspace;
    PCG_TWO_SWEEPS drops it, and nothing changes where it does not apply
    (consecutive-cell tiles)."""
    def ws(g, flags, prec=0):
        o = L.Opts()
        o.flags = flags
        o.precision = prec
        out = ctypes.c_size_t()
        assert lib.pcg_workspace_bytes(ctypes.byref(g), ctypes.byref(o), ctypes.byref(out)) == L.OK
        return out.value

    g = _g(128, 16, 8)
    n = 128 * 16 * 8
    # (the partial sums of the two tile forms differ by a few aligned blocks)
    assert 8 * n - 4 * 256 <= ws(g, L.PLANE_TILES) - ws(g, L.PLANE_TILES | L.TWO_SWEEPS) <= 8 * n
    assert ws(g, 0) == ws(g, L.PLANE_TILES)           # FP64 takes plane tiles at any size
    # with the walls unknown a periodic y axis may still send a grid to
    # consecutive-cell tiles: the workspace covers both forms
    for shape in [(128, 13, 6), (128, 1, 6), (256, 7, 5), (128, 16, 8), (384, 9, 3)]:
        gs = _g(*shape)
        for extra in (0, L.TWO_SWEEPS):
            assert ws(gs, extra) >= ws(gs, L.FLAT_TILES), (shape, extra)
            assert ws(gs, L.PLANE_TILES | extra) >= ws(gs, L.FLAT_TILES), (shape, extra)
    # rows of an odd length: narrow plane tiles (one cell a thread, one
    # sweep, so the second z) at any size; consecutive-cell tiles, without
    # it, with two sweeps
    g97 = _g(97, 64, 64)
    n97 = 97 * 64 * 64
    # (the two forms' tile counts, and so their partial sums, differ)
    assert 8 * n97 - 65536 <= ws(g97, 0) - ws(g97, L.TWO_SWEEPS) <= 8 * n97 + 65536
    assert ws(g97, L.NARROW_TILES) == ws(g97, 0)
    assert ws(g97, L.TWO_SWEEPS) == ws(g97, L.FLAT_TILES)
    # rows of 96 cells fill three quarters of a 128-cell tile: plane tiles
    # (and the second z) when asked for
    g96 = _g(96, 16, 8)
    n96 = 96 * 16 * 8
    assert 8 * n96 - 4 * 256 <= ws(g96, L.PLANE_TILES) - ws(g96, L.PLANE_TILES | L.TWO_SWEEPS) <= 8 * n96
    assert ws(g96, L.PLANE_TILES) >= ws(g96, L.FLAT_TILES)
    assert ws(g, L.PLANE_TILES | L.FLAT_TILES) == ws(g, L.PLANE_TILES | L.FLAT_TILES | L.TWO_SWEEPS)
    # the FP32 inner solve on plane tiles: a second FP32 z
    g256 = _g(256, 16, 8)
    d32 = ws(g256, L.PLANE_TILES, 1) - ws(g256, L.PLANE_TILES | L.TWO_SWEEPS, 1)
    # (at this size the sizing also covers narrow tiles, whose partial sums
    # are more)
    assert 4 * 256 * 16 * 8 - 4 * 256 <= d32 <= 4 * 256 * 16 * 8 + 65536
    assert ws(g256, 0, 1) == ws(g256, L.PLANE_TILES, 1)   # FP32: plane tiles at any size
    # a 512^3 FP64 grid takes plane tiles, hence the second z, by default
    big = _g(512, 512, 512)
    assert ws(big, 0) - ws(big, L.TWO_SWEEPS) == 8 * 512 ** 3
