"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package only *generates* inputs: SU(3) gauge fields, Gaussian even-site
sources and the rational-function coefficients that the multi-shift solver is
asked to apply.  It contains none of the staggered operator or solver
arithmetic; both the CPU oracle (``oracle/``) and the HIP library consume what
it produces, and neither imports the other.
"""

from .fields import (  # noqa: F401
    CONFIGS,
    MD_WORKLOAD,
    even_volume,
    gauge_field,
    momenta,
    random_su3,
    source,
    unit_gauge,
    volume,
)
