"""Seeded initial blocks, request streams and the named eigen-solve problems.

Seeds: problem ``i`` draws its matrix coefficients from ``1000+i`` and its
initial block from ``2000+i``; the serving stream draws from ``3000``.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .stencils import CSR, laplacian_2d, laplacian_3d, random_potential, spd27, mass27, convdiff_2d


def initial_block(n: int, m0: int, seed: int) -> np.ndarray:
    """Random normal n x m0 initial subspace, row-major (C order), FP64."""
    return np.random.default_rng(seed).standard_normal((n, m0))


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream with the given rate."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=count)
    return np.cumsum(gaps)


@dataclass
class Problem:
    """One eigen-solve: A x = lambda B x with lambda inside a contour.

    contour: ``{"kind": "half", "emin", "emax", "rule": "gl"|"trap", "nc"}``
    (real symmetric problems; nc systems on the upper half of the circle
    through emin and emax) or ``{"kind": "circle", "c", "r", "rule": "trap",
    "nc"}`` (general problems; nc systems around the whole circle).
    """

    name: str
    A: CSR
    B: CSR | None
    contour: dict
    m0: int
    max_inner: int
    alpha: float
    tol: float
    max_outer: int
    x0_seed: int
    kind: str = "symmetric"  # or "general"
    max_cycles: int = 20  # block-GMRES(max_inner) restart cycles per shifted solve
    inner_rule: str = "column"  # "column": per-column relative alpha; "global": alpha * ||R_F||
    tau: float = 0.5  # filter-gain threshold for counting a Ritz pair inside the contour
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.n

    def x0(self) -> np.ndarray:
        return initial_block(self.n, self.m0, self.x0_seed)


def config1() -> Problem:
    """2-D 5-point Laplacian, 20 x 20 (n = 400, nnz = 1920), B = I.

    Interval (0.5, 0.8) holds 11 eigenvalues; m0 = 16, 8 Gauss-Legendre nodes
    on the upper half circle, 4 block-GMRES iterations, residual <= 1e-10.
    """
    A = laplacian_2d(20)
    return Problem(
        name="lap2d_20",
        A=A,
        B=None,
        contour={"kind": "half", "emin": 0.5, "emax": 0.8, "rule": "gl", "nc": 8},
        m0=16,
        max_inner=4,
        alpha=1e-2,
        tol=1e-10,
        max_outer=40,
        x0_seed=2001,
    )


def _lap3d_potential(N: int, seed: int) -> CSR:
    n = N ** 3
    return laplacian_3d(N, random_potential(n, seed, 0.0, 2.0))


# Interval for the 3-D Laplacian + U[0, 2] potential (seed 1002), per grid
# side: 54 interior eigenvalues (indices 62..115 of the spectrum, so 62 lie
# below), ends in the middle of gaps about 2.5 times the mean spacing.  The
# indices come from the reference low spectrum in tests/golden.
_C2_INTERVALS = {64: (0.98977, 1.02232)}


def config2(N: int = 64, emin: float | None = None, emax: float | None = None) -> Problem:
    """3-D 7-point Laplacian + uniform [0, 2] potential on an N^3 grid, B = I.

    m0 = 80, 8 Gauss-Legendre half-circle nodes, 8 block-GMRES iterations.
    """
    A = _lap3d_potential(N, 1002)
    if emin is None:
        emin, emax = _C2_INTERVALS[N]
    return Problem(
        name=f"lap3d_pot_{N}",
        A=A,
        B=None,
        contour={"kind": "half", "emin": emin, "emax": emax, "rule": "gl", "nc": 8},
        m0=80,
        max_inner=8,
        alpha=1e-2,
        tol=1e-9,
        max_outer=60,
        x0_seed=2002,
    )


def config2_small(N: int = 16, m0: int = 24, emin: float | None = None, emax: float | None = None) -> Problem:
    """Reduced-grid version of the 3-D Laplacian + potential problem."""
    A = _lap3d_potential(N, 1002)
    return Problem(
        name=f"lap3d_pot_{N}",
        A=A,
        B=None,
        contour={"kind": "half", "emin": emin, "emax": emax, "rule": "gl", "nc": 8},
        m0=m0,
        max_inner=8,
        alpha=1e-2,
        tol=1e-9,
        max_outer=60,
        x0_seed=2002,
    )


def config3_small(N: int = 8, m0: int = 16, emin: float = 0.0, emax: float = 1.0) -> Problem:
    """Reduced-grid generalized problem: 27-point random SPD A, Q1-mass B x density."""
    return Problem(
        name=f"spd27_mass_{N}",
        A=spd27(N, 1003),
        B=mass27(N, 1003 + 100),
        contour={"kind": "half", "emin": emin, "emax": emax, "rule": "gl", "nc": 12},
        m0=m0,
        max_inner=8,
        alpha=1e-2,
        tol=1e-9,
        max_outer=60,
        x0_seed=2003,
    )


def config3(N: int = 100, m0: int = 128, emin: float | None = None, emax: float | None = None,
            constant: bool = False) -> Problem:
    """Generalized symmetric problem A x = lambda B x on an N^3 grid (n = 10^6 at N = 100): 27-point
    SPD A with log-uniform edge coefficients, Q1 mass B scaled by a U[0.5, 1.5] density
    (``constant``: all coefficients and densities 1, a closed-form spectrum); 12 Gauss-Legendre
    half-circle nodes, block GMRES with 8 iterations per cycle."""
    return Problem(
        name=f"spd27_mass_{N}" + ("_const" if constant else ""),
        A=spd27(N, 1003, constant=constant),
        B=mass27(N, 1003 + 100, density=not constant),
        contour={"kind": "half", "emin": emin, "emax": emax, "rule": "gl", "nc": 12},
        m0=m0,
        max_inner=8,
        alpha=1e-2,
        tol=1e-9,
        max_outer=60,
        x0_seed=2003,
    )


def config3_constant_spectrum(N: int) -> np.ndarray:
    """Eigenvalues (ascending) of the constant-coefficient pair (A, B) of config3: with
    t_i = cos(j_i pi / (N + 1)), lambda = (27 - prod(1 + 2 t_i)) / prod((4 + 2 t_i) / 6)."""
    t = np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    a1, b1 = 1.0 + 2.0 * t, (4.0 + 2.0 * t) / 6.0
    num = 27.0 - a1[:, None, None] * a1[None, :, None] * a1[None, None, :]
    den = b1[:, None, None] * b1[None, :, None] * b1[None, None, :]
    return np.sort((num / den).ravel())


def config4_small(N: int = 32, m0: int = 16, c: float = 0.2, r: float = 0.1) -> Problem:
    """Reduced-grid non-Hermitian problem: 2-D upwind convection-diffusion."""
    return Problem(
        name=f"convdiff_{N}",
        A=convdiff_2d(N, 20.0, 10.0),
        B=None,
        contour={"kind": "circle", "c": c, "r": r, "rule": "trap", "nc": 16},
        m0=m0,
        max_inner=10,
        alpha=1e-2,
        tol=1e-9,
        max_outer=60,
        x0_seed=2004,
        kind="general",
    )


def convdiff_spectrum(N: int, beta_x: float = 20.0, beta_y: float = 10.0) -> np.ndarray:
    """Eigenvalues (ascending, real) of convdiff_2d(N, beta_x, beta_y): the upwind operator is
    D S D^-1 with S a symmetric tridiagonal Toeplitz sum per direction, so each direction
    contributes 2 + h b - 2 sqrt(1 + h b) cos(j pi / (N + 1))."""
    h = 1.0 / (N + 1)
    j = np.arange(1, N + 1)

    def mu(b):
        return 2.0 + h * b - 2.0 * np.sqrt(1.0 + h * b) * np.cos(j * np.pi / (N + 1))

    return np.sort((mu(beta_x)[:, None] + mu(beta_y)[None, :]).ravel())


def config4_circle(N: int, target: float | None = None, count: int = 40, slack: int = 4):
    """Circle on the real axis around about ``count`` eigenvalues: the lowest ones (target None;
    the left end 10% of the window below the lowest eigenvalue) or those above ``target`` (the
    left end in the widest gap within ``slack`` places).  The right end sits in the widest gap
    within ``slack`` places of the nominal end, so no eigenvalue is near the contour.  Returns
    (centre, radius, eigenvalues inside)."""
    ev = convdiff_spectrum(N)
    gaps = np.diff(ev)
    if target is None:
        lo_i = 0
    else:
        i0 = int(np.searchsorted(ev, target))
        lo_i = max(1, i0 - slack) + int(np.argmax(gaps[max(1, i0 - slack) - 1:i0 + slack]))
    hi_n = lo_i + count
    hi_i = hi_n - slack + int(np.argmax(gaps[hi_n - slack - 1:hi_n + slack]))
    hi = 0.5 * (ev[hi_i - 1] + ev[hi_i])
    lo = ev[0] - 0.1 * (hi - ev[0]) if lo_i == 0 else 0.5 * (ev[lo_i - 1] + ev[lo_i])
    return 0.5 * (lo + hi), 0.5 * (hi - lo), ev[lo_i:hi_i]


def config4(N: int = 512, target: float | None = None, count: int = 40) -> Problem:
    """2-D upwind convection-diffusion, beta = (20, 10), h^2-scaled, on an N x N grid (n = N^2,
    262,144 at N = 512), B = I: a full circle on the real axis around about 40 eigenvalues (the
    lowest ones by default), 16 trapezoidal nodes, m0 = 64, block GMRES with 10 iterations per
    cycle and at most 30 cycles (300 iterations) per shifted solve."""
    c, r, inside = config4_circle(N, target, count)
    return Problem(
        name=f"convdiff_{N}",
        A=convdiff_2d(N, 20.0, 10.0),
        B=None,
        contour={"kind": "circle", "c": c, "r": r, "rule": "trap", "nc": 16},
        m0=64,
        max_inner=10,
        alpha=1e-2,
        tol=1e-9,
        max_outer=30,
        x0_seed=2004,
        kind="general",
        max_cycles=30,
        meta={"inside": inside},
    )


def serving_requests(count: int, seed: int = 3000, rate: float = 20.0,
                     sides=(32, 48, 64, 96, 128), m0s=(16, 32, 64, 128)):
    """Parameters of a seeded Poisson stream of eigen-solve requests.

    Returns a list of dicts with the arrival time, grid side, m0 and the
    seeds of the request's potential and initial block.
    """
    rng = np.random.default_rng(seed)
    t = poisson_arrivals(rate, count, seed + 1)
    out = []
    for i in range(count):
        out.append({
            "arrival": float(t[i]),
            "side": int(rng.choice(sides)),
            "m0": int(rng.choice(m0s)),
            "pot_seed": int(seed + 10 + i),
            "x0_seed": int(seed + 5000 + i),
        })
    return out
