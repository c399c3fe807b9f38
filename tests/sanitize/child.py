"""Run in a child process with the sanitizer runtime preloaded: the oracle's
pins and the library's host checks, against the sanitized builds named on
the command line (oracle .so, library .so).  Any sanitizer report aborts the
process with a non-zero status."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)


def main(oracle_so, lib_so):
    # the binding's default library is the sanitized build (the tile-rule
    # helpers load the default one)
    os.environ["PCGMI_LIB"] = lib_so
    import oracle
    from paper_1410_1942_amd import _lib as L
    from paper_1410_1942_amd import fields as F
    from tests import test_abi_cpu as abi
    from tests import test_oracle_mutations as mut
    from tests import test_oracle_pins as pins

    o = mut.Bound(oracle.load(oracle_so))
    for case in pins._gold_cases():
        pins.test_hand_solved(o, case)
        pins.test_relres_of_hand_solutions(o, case)
    pins.test_relres_cut_cells_by_hand(o)
    pins.test_relres_singular_by_hand(o)
    pins.test_dense_cholesky(o, F, (6, 5, 7), (1, 0, 0, 1, 0, 1), True)
    pins.test_dense_periodic(o, F, (9, 6, 7), (2, 2, 0, 0, 0, 0))
    pins.test_dense_with_fractions(o, F)
    pins.test_projection_divergence(o, F, 1e-6)
    pins.test_projection_divergence_periodic(o, F, (2, 2, 0, 0, 0, 0))
    pins.test_relres_ignores_hull_entries(o, F, pins.TANK)
    print("oracle: ok", flush=True)

    lib = L.load()
    assert L.LIB_PATH == lib_so
    abi.test_strerror(lib)
    abi.test_workspace_bytes_validation(lib)
    abi.test_setup_validation_without_device_work(lib)
    abi.test_null_handles(lib)
    abi.test_connectivity_check_matches_reference(lib, o)
    abi.test_tile_rules_roundtrip(lib)
    abi.test_stage_entry_points_reject_null_context(lib)
    abi.test_plane_and_tile_span_limits(lib)
    abi.test_fraction_flag_host_rules(lib)
    print("library host code: ok", flush=True)


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2])
