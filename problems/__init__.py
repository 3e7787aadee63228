"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package builds the linear systems ``A u = f`` that the solver is run on
(sparse matrices in CSR form and right-hand sides).  It holds none of the
multigrid method's arithmetic: no strength test, aggregation, smoothing,
transfer operator or Krylov step lives here, so both the oracle and the
device path can take their inputs from it without sharing any of the method.
"""

from .grids import (  # noqa: F401
    CSR,
    poisson3d,
    poisson3d_nnz,
    gaussian_field,
    diffusion3d,
    rhs_ones,
    rhs_uniform,
    tridiag1d,
)
from .irregular import (  # noqa: F401
    anisotropic3d,
    banded_spd,
    decoupled_boundary,
    poisson3d_27,
    random_laplacian,
)
from .blocks import (  # noqa: F401
    BSR,
    coupled_diffusion3d,
    decoupled_diffusion3d,
    random_block_rhs,
)
from .stokes import oseen_p1, oseen_rhs, stokes3d, stokes_rhs  # noqa: F401
