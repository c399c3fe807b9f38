"""The pins catch plausible mistakes in the reference.

Each case copies the reference source, plants one mistake by text
replacement, builds the copy with gcc into a temporary directory and runs the
pins that should catch it.  The real reference source is never modified.
"""
import functools
import json
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")


class Bound:
    """The oracle module's API bound to another build of the library."""

    def __init__(self, lib):
        for name in ("apply", "pcg", "relres", "project", "divergence",
                     "connected", "components", "source"):
            setattr(self, name, functools.partial(getattr(oracle, name), lib=lib))
        for name in ("OK", "MAXIT", "EINVAL", "EDOMAIN", "ESINGULAR",
                     "EBREAKDOWN", "EUNSUPPORTED"):
            setattr(self, name, getattr(oracle, name))


def _gold(name):
    return [c for c in pins._gold_cases() if c["name"] == name][0]


def _F():
    from paper_1410_1942_amd import fields
    return fields


PIN_RUNS = {
    "hand_column": lambda o: pins.test_hand_solved(o, _gold("water_air_column")),
    "hand_hull": lambda o: pins.test_hand_solved(o, _gold("water_cell_beside_hull")),
    "hand_row": lambda o: pins.test_hand_solved(o, _gold("three_cell_row_open_ends")),
    "eig_dirichlet": lambda o: pins.test_eigvec_all_dirichlet(o, (12, 10, 8), 2.5, (1, 2, 3)),
    "eig_tank": lambda o: pins.test_eigvec_tank(o, (10, 6, 12)),
    "manufactured": lambda o: pins.test_manufactured_second_order(o),
    "dense": lambda o: pins.test_dense_cholesky(o, _F(), (8, 8, 8), (1, 0, 0, 1, 0, 1), True),
    "banded": lambda o: pins.test_column_reduction_banded(o),
    "divergence": lambda o: pins.test_projection_divergence(o, _F(), 1e-6),
    "termination": lambda o: pins.test_finite_termination(o, 8),
    "eig_periodic": lambda o: pins.test_eigvec_periodic(o, (9, 14, 7), (2, 1)),
    "eig_neumann": lambda o: pins.test_eigvec_pure_neumann(o, (7, 9, 6), (0, 3, 1), 37.0),
    "dense_periodic": lambda o: pins.test_dense_periodic(o, _F(), (9, 6, 7), (2, 2, 0, 0, 0, 0)),
    "dense_fractions": lambda o: pins.test_dense_with_fractions(o, _F()),
    "volume_scaling": lambda o: pins.test_uniform_volume_scales_the_answer(o, _F()),
    "divergence_fractions": lambda o: pins.test_projection_divergence_with_fractions(o, _F()),
    "divergence_periodic": lambda o: pins.test_projection_divergence_periodic(
        o, _F(), (2, 2, 0, 0, 0, 0)),
    "textbook_iters": lambda o: [pins.test_pcg_iterations_match_textbook(o, _F(), *case)
                                 for case in (((8, 8, 8), (1, 0, 0, 1, 0, 1), True, 11),
                                              ((16, 4, 2), (1, 1, 0, 0, 1, 1), True, 7))],
    "relres_cut_cells": lambda o: pins.test_relres_cut_cells_by_hand(o),
    "relres_singular": lambda o: pins.test_relres_singular_by_hand(o),
    "relres_hull": lambda o: pins.test_relres_ignores_hull_entries(o, _F(), pins.TANK),
    "relres_vs_pcg": lambda o: pins.test_relres_matches_what_pcg_stops_on(
        o, _F(), (2, 2, 0, 0, 0, 0), True),
}

MUTANTS = [
    # average 1/rho instead of rho on a face
    ("harmonic_face", "return 1.0 / ((P->rho[a] + P->rho[b]) / 2.0);",
     "return (1.0 / P->rho[a] + 1.0 / P->rho[b]) / 2.0;"),
    # Dirichlet ghost mirrored with the wrong sign (acts as Neumann)
    ("ghost_sign", "double pn = nb[f] >= 0 ? p[nb[f]] : -p[c]; /* ghost */",
     "double pn = nb[f] >= 0 ? p[nb[f]] : p[c]; /* ghost */"),
    # hull faces left open
    ("hull_open", "if (P->solid[a] || P->solid[b]) return 0.0;",
     "if (P->solid[a] && P->solid[b]) return 0.0;"),
    # y- and y+ walls exchanged
    ("y_walls_swapped", "int jj = j + (f == 2 ? -1 : f == 3 ? 1 : 0);",
     "int jj = j + (f == 2 ? 1 : f == 3 ? -1 : 0);"),
    # conjugate direction dropped: steepest descent
    ("no_conjugation", "pp[c] = z[c] + beta * pp[c];", "pp[c] = z[c];"),
    # grid spacing not squared in the scaled right-hand side
    ("h_not_squared", "double h2 = h * h;", "double h2 = h;"),
    # projection moves velocity up the pressure gradient
    ("projection_sign", "*uf -= s * face_beta(&P, a, b) * (p[b] - p[a]);",
     "*uf += s * face_beta(&P, a, b) * (p[b] - p[a]);"),
    # z face coefficient taken from the wrong neighbour
    ("z_index", "int kk = k + (f == 4 ? -1 : f == 5 ? 1 : 0);",
     "int kk = k + (f == 4 ? 1 : f == 5 ? 1 : 0);"),
    # periodic wrap lands one cell short
    ("periodic_wrap", "if (f < 2) ii = (ii + P->nx) % P->nx;",
     "if (f < 2) ii = (ii + P->nx - 1) % P->nx;"),
    # singular problem: source mean not removed
    ("source_mean_kept", "if (!solid[c]) b[c] -= mean;", "if (!solid[c]) b[c] -= 0.0 * mean;"),
    # singular problem: solution not shifted to zero mean
    ("solution_mean_kept", "if (!solid[c]) x[c] -= mean;", "if (!solid[c]) x[c] -= 0.0 * mean;"),
    # x area fractions ignored
    ("x_area_ignored", "return P->ax[((size_t)k * ny + j) * (nx + 1) + fi];", "return 1.0;"),
    # volume fraction left out of the right-hand side
    ("volume_off_source", "b[c] = solid[c] ? 0.0 : -h2 * volume(&P, c) * rhs[c];",
     "b[c] = solid[c] ? 0.0 : -h2 * rhs[c];"),
    # periodic y wrap lands one row short
    ("periodic_wrap_y", "else jj = (jj + P->ny) % P->ny;", "else jj = (jj + P->ny - 1) % P->ny;"),
    # Jacobi diagonal without the doubled Dirichlet ghost term (same answers,
    # other iteration counts)
    ("jacobi_diag_ghost", "s += nb[f] >= 0 ? beta[f] : 2.0 * beta[f];", "s += beta[f];"),
    # shared periodic x face corrected up the pressure gradient
    ("periodic_face_sign", "if (nx > 1) *uf -= s * face_beta(&P, a, b) * (p[b] - p[a]);",
     "if (nx > 1) *uf += s * face_beta(&P, a, b) * (p[b] - p[a]);"),
    # area divergence not divided by the volume fraction
    ("divergence_no_volume", "out[w0] = ax ? (du + dv + dw) / (vc * h) : (du + dv + dw) / h;",
     "out[w0] = (du + dv + dw) / h;"),
    # residual checker: volume weight dropped
    ("relres_no_volume", "double v = vol ? vol[c] : 1.0;\n        double w = v * rhs[c] - mean;",
     "double v = 1.0;\n        double w = v * rhs[c] - mean;"),
    # residual checker: hull cells counted
    ("relres_hull_counted", "if (solid[c]) continue;\n        double v = vol",
     "double v = vol"),
    # residual checker: singular source keeps its mean
    ("relres_mean_kept", "mean = sw / nf;", "mean = 0.0 * sw / nf;"),
    # residual checker: ratio of squared norms
    ("relres_squared", "return bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);",
     "return bb > 0.0 ? rr / bb : rr;"),
]


@pytest.fixture(scope="module")
def tmpdir_mut():
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def _caught(o, name):
    try:
        PIN_RUNS[name](o)
    except (AssertionError, ValueError):
        return True
    return False


def test_unmutated_passes_all(tmpdir_mut):
    out = os.path.join(tmpdir_mut, "lib_ref.so")
    oracle.build(SRC, out)
    o = Bound(oracle.load(out))
    for name in PIN_RUNS:
        assert not _caught(o, name), name


@pytest.mark.parametrize("mutant", MUTANTS, ids=lambda m: m[0])
def test_mutant_is_caught(tmpdir_mut, mutant):
    name, old, new = mutant
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    src = src.replace(old, new)
    cpath = os.path.join(tmpdir_mut, f"{name}.c")
    with open(cpath, "w") as f:
        f.write(src)
    out = os.path.join(tmpdir_mut, f"lib_{name}.so")
    oracle.build(cpath, out)
    o = Bound(oracle.load(out))
    caught = next((p for p in PIN_RUNS if _caught(o, p)), None)
    assert caught is not None, f"mutant {name} passed every pin"
