"""Seeded synthetic inputs for the IFEAST eigen-solves.

This package builds the matrices, initial blocks and request streams that
both the CPU oracle and the GPU path consume.  It holds none of the method's
arithmetic: no quadrature, no Krylov solve, no Rayleigh-Ritz.  Every array is
a plain numpy array so that either side can take it without importing the
other.

Matrices are returned as :class:`CSR` (0-based, column indices sorted within
each row, no duplicates), with a lexicographic grid numbering
``x + N*y + N*N*z``.
"""

from .stencils import (
    CSR,
    laplacian_2d,
    laplacian_3d,
    random_potential,
    spd27,
    mass27,
    convdiff_2d,
)
from .inputs import (
    initial_block,
    poisson_arrivals,
    Problem,
    config1,
    config2,
    config2_small,
    config3_small,
    config3,
    config3_constant_spectrum,
    config4_small,
    config4,
    config4_circle,
    convdiff_spectrum,
    serving_requests,
)

__all__ = [
    "CSR",
    "laplacian_2d",
    "laplacian_3d",
    "random_potential",
    "spd27",
    "mass27",
    "convdiff_2d",
    "initial_block",
    "poisson_arrivals",
    "Problem",
    "config1",
    "config2",
    "config2_small",
    "config3_small",
    "config3",
    "config3_constant_spectrum",
    "config4_small",
    "config4",
    "config4_circle",
    "convdiff_spectrum",
    "serving_requests",
]
