"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This package builds matrices and right-hand sides only.  It holds none of the
solver's arithmetic (no CG step, no BFS, no neighbour search), so both the
HIP path and the CPU oracle can take their inputs from it without sharing any
part of the method.
"""

from .generators import (  # noqa: F401
    CSR,
    poisson2d,
    poisson3d,
    varcoef3d,
    banded,
    er_laplacian,
    star,
    path,
    extended_star,
    random_spd_dense,
    rhs,
    smooth_rhs,
    family_matrix,
    FAMILIES,
)
from . import paper_family  # noqa: F401,E402
