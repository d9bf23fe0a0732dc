"""Seeded synthetic inputs for the condition-number estimator.

This package builds test and benchmark matrices and start vectors. It holds
none of the estimator's arithmetic: it only assembles CSR matrices from
seeded coefficient fields and draws seeded start vectors. Both the plain CPU
oracle and the GPU path consume what it produces.
"""

from .matrices import (  # noqa: F401
    Csr,
    csr_from_dense,
    diag_csr,
    scaled_banded,
    stokes2d,
    hm_fields,
    hydromech2d,
    hm_batch_specs,
)
from .starts import start_vector, start_block  # noqa: F401
