"""CPU FP64 oracle for IFEAST (Gavin & Polizzi, arXiv 1706.00692).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
numpy/scipy implementation of what the GPU path computes.  Only the tests,
the smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does.  It shares no code with the GPU library (no
kernels, headers, helpers or generated tables) and never imports it; its
inputs come from the seeded generators in ``workloads``.

Modules
-------
quadrature  nodes, weights and the rational filter (Eq. contour_int_quad, Eq. rhoh)
krylov      block GMRES on one shifted system (Sec. 2.2, Sec. 3.2)
feast       Algorithm 2 (IFEAST), Algorithm 1 (FEAST with direct solves),
            Rayleigh-Ritz and residuals, dense reference eigensolves
reference   low spectra of large 3-D stencils by preconditioned LOBPCG

Every function is pinned by a ``-m "not gpu"`` test against something other
than itself (closed forms, textbook identities, library solvers, brute
force); none is "parity unpinned".
"""

from .quadrature import contour_nodes, gauss_legendre_half, trapezoid_half, trapezoid_circle, rho_hat
from .krylov import block_gmres, shifted_operator
from .reference import lowest_eigenvalues_lap3d
from .feast import (
    IFeastResult,
    ifeast,
    feast_direct,
    rayleigh_ritz,
    residuals,
    inside_contour,
    dense_reference,
    quad_accumulate,
    minres_columns,
)

__all__ = [
    "contour_nodes",
    "gauss_legendre_half",
    "trapezoid_half",
    "trapezoid_circle",
    "rho_hat",
    "block_gmres",
    "shifted_operator",
    "IFeastResult",
    "ifeast",
    "feast_direct",
    "rayleigh_ritz",
    "residuals",
    "inside_contour",
    "dense_reference",
    "quad_accumulate",
    "minres_columns",
    "lowest_eigenvalues_lap3d",
]
