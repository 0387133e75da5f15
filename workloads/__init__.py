"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package holds input generation only: planted spectra, matrices
A = U diag(sigma) V^H with known singular triplets, integer-valued matrices for
exact sketch checks and the request stream of the served workload.  It holds
none of the RLOBPCG arithmetic; neither the oracle nor the HIP path is imported
here.
"""

from .planted import (  # noqa: F401
    CONFIGS,
    config_spec,
    spectrum_gap,
    spectrum_logspace_tail,
    spectrum_clustered,
    spectrum_nullspace,
    planted_numpy,
    planted_torch,
    integer_matrix,
    served_requests,
    request_spectrum,
    config_spectrum,
)
