"""Oracle: a plain, slow, FP64 CPU implementation of smoothed-aggregation AMG
used as a Krylov preconditioner.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path imports,
links or calls this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the device path: the
two take their inputs from the separate ``problems`` package and nothing else.
"""

from .sa_amg import (  # noqa: F401
    Params,
    Level,
    Hierarchy,
    strength_graph,
    aggregate,
    tentative_prolongator,
    filtered_matrix,
    prolongator_damping,
    smoothed_prolongator,
    spai0_diagonal,
    jacobi_diagonal,
    chebyshev_upper_bound,
    chebyshev_sweep,
    setup,
    vcycle,
    vcycle_fp32,
    hierarchy_fp32,
    pcg,
    bicgstab,
    arnoldi_cgs2,
    gmres,
    solve,
)
from . import schur  # noqa: F401,E402
