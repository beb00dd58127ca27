"""Seeded synthetic inputs for the DA-CSR SpMV path.

This package produces sparse matrices in plain int32 CSR form plus dense
vectors, from fixed seeds.  It stands in for the SuiteSparse matrices the
paper measures on (Sec. 3), which are not available here.

It contains no part of the method itself (no bandwidth fit, no diagonal
addressing, no reordering, no products): both the CPU oracle and the HIP
path consume what it returns, and neither side's arithmetic lives here.
"""

from .matrices import (  # noqa: F401
    CSR,
    laplace_2d_5pt,
    poisson_3d_7pt,
    stencil_3d_27pt,
    stencil_3d_27pt_box,
    random_banded,
    scramble_symmetric,
    random_csr,
    uniform_vector,
    batch_family,
)
from .configs import (  # noqa: F401
    CONFIG_SEEDS,
    config_matrix,
    config_vector,
    config_description,
)
