"""MI355X-native pressure projection of the cartesian-grid ship-wave method.

The variable-coefficient Poisson equation of the projection step is solved
by Jacobi-preconditioned conjugate gradients in hand-written HIP kernels for
gfx950, behind the C ABI of include/pcg.h.  ``fields`` draws seeded
synthetic inputs; ``solver`` is the torch-facing wrapper of the library.
"""
from . import fields  # noqa: F401

__all__ = ["fields", "solver", "build"]
