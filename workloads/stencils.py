"""Finite-difference / finite-element stencil matrices on structured grids.

All generators return a :class:`CSR` in FP64 with 0-based, sorted column
indices.  The grid numbering is lexicographic: ``x + N*y`` in 2-D and
``x + N*y + N*N*z`` in 3-D, Dirichlet boundaries (off-grid neighbours are
dropped from the pattern).
"""

from __future__ import annotations

from dataclasses import dataclass
import itertools

import numpy as np


@dataclass
class CSR:
    """Compressed sparse row matrix, 0-based, columns sorted within each row."""

    n: int
    rowptr: np.ndarray  # int64, length n+1
    colind: np.ndarray  # int32, length nnz
    val: np.ndarray  # float64, length nnz
    symmetric: bool = False

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        out[rows, self.colind] = self.val
        return out


def _assemble(dims, offsets, coef_fn, symmetric):
    """Assemble a stencil matrix.

    ``offsets`` is a list of integer tuples (dx, dy[, dz]); ``coef_fn(k, idx)``
    returns the coefficient of offset ``k`` for the (valid) rows ``idx``
    (arrays of grid coordinates, one per dimension).
    """
    dims = tuple(int(d) for d in dims)
    ndim = len(dims)
    n = int(np.prod(dims))
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    lin = [sum(o[a] * strides[a] for a in range(ndim)) for o in offsets]
    order = np.argsort(lin, kind="stable")
    offsets = [offsets[i] for i in order]
    lin = [lin[i] for i in order]
    perm = [int(i) for i in order]

    coords = np.indices(dims[::-1]).reshape(ndim, -1)[::-1]  # coords[a] = coordinate along axis a
    cols = np.empty((len(offsets), n), dtype=np.int64)
    vals = np.zeros((len(offsets), n))
    valid = np.empty((len(offsets), n), dtype=bool)
    rows = np.arange(n, dtype=np.int64)
    for k, (off, lo) in enumerate(zip(offsets, lin)):
        ok = np.ones(n, dtype=bool)
        for a in range(ndim):
            c = coords[a] + off[a]
            ok &= (c >= 0) & (c < dims[a])
        valid[k] = ok
        cols[k] = rows + lo
        vals[k] = coef_fn(perm[k], coords)
    valid = valid.T
    colind = cols.T[valid].astype(np.int32)
    val = vals.T[valid]
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(n=n, rowptr=rowptr, colind=colind, val=np.ascontiguousarray(val), symmetric=symmetric)


def laplacian_2d(N: int) -> CSR:
    """5-point Dirichlet Laplacian on an N x N grid: 4 on the diagonal, -1 off it."""
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]

    def coef(k, coords):
        return np.full(coords.shape[1], 4.0 if k == 0 else -1.0)

    return _assemble((N, N), offs, coef, symmetric=True)


def random_potential(n: int, seed: int, low: float = 0.0, high: float = 2.0) -> np.ndarray:
    """i.i.d. uniform diagonal potential drawn from ``default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(low, high, size=n)


def laplacian_3d(N: int, potential: np.ndarray | None = None) -> CSR:
    """7-point Dirichlet Laplacian on an N^3 grid plus an optional diagonal potential."""
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    pot = None if potential is None else np.asarray(potential, dtype=np.float64)

    def coef(k, coords):
        if k == 0:
            d = np.full(coords.shape[1], 6.0)
            if pot is not None:
                d = d + pot
            return d
        return np.full(coords.shape[1], -1.0)

    return _assemble((N, N, N), offs, coef, symmetric=True)


_OFFS27 = [o for o in itertools.product((-1, 0, 1), repeat=3) if o != (0, 0, 0)]


def _forward(o):
    """True for the 13 offsets whose linear index offset is positive."""
    dx, dy, dz = o
    return (dz, dy, dx) > (0, 0, 0)


def spd27(N: int, seed: int, constant: bool = False) -> CSR:
    """27-point SPD operator with random edge coefficients.

    Every undirected edge {p, p+d} of the 26-neighbour graph (including edges
    that leave the grid) carries a coefficient drawn log-uniformly from
    [0.1, 10] (all 1 when ``constant``: then A = 27 I - the all-ones stencil).
    Off-diagonal entries are the negated in-grid edge coefficients; the
    diagonal is the sum over all 26 edge slots of the cell, so the matrix is
    irreducibly diagonally dominant and hence SPD.
    """
    fwd = [o for o in _OFFS27 if _forward(o)]  # 13 directions
    rng = np.random.default_rng(seed)
    # c[z+1, y+1, x+1, d] is the coefficient of edge {p, p+fwd[d]} for p in [-1, N]^3
    if constant:
        c = np.ones((N + 2, N + 2, N + 2, len(fwd)))
    else:
        c = 10.0 ** rng.uniform(-1.0, 1.0, size=(N + 2, N + 2, N + 2, len(fwd)))

    def edge(coords, o, sign):
        """Coefficient of edge {p, p+o} (sign > 0) or {p-o, p} (sign < 0), o forward."""
        x, y, z = coords
        d = fwd.index(o)
        if sign > 0:
            px, py, pz = x, y, z
        else:
            px, py, pz = x - o[0], y - o[1], z - o[2]
        return c[pz + 1, py + 1, px + 1, d]

    offs = [(0, 0, 0)] + _OFFS27

    def coef(k, coords):
        if k == 0:
            diag = np.zeros(coords.shape[1])
            for o in fwd:
                diag += edge(coords, o, +1) + edge(coords, o, -1)
            return diag
        o = offs[k]
        if _forward(o):
            return -edge(coords, o, +1)
        return -edge(coords, (-o[0], -o[1], -o[2]), -1)

    return _assemble((N, N, N), offs, coef, symmetric=True)


def mass27(N: int, seed: int, density: bool = True) -> CSR:
    """Trilinear (Q1) finite-element mass stencil scaled by a random density.

    M = ([1, 4, 1] / 6) tensored three times (centre 8/27, faces 2/27, edges
    1/54, corners 1/216), truncated at the Dirichlet boundary; the density
    rho ~ U[0.5, 1.5] per cell enters as B = D^(1/2) M D^(1/2), D = diag(rho).
    """
    if density:
        rho = np.random.default_rng(seed).uniform(0.5, 1.5, size=N * N * N)
    else:
        rho = np.ones(N * N * N)
    sq = np.sqrt(rho)
    w1 = {-1: 1.0 / 6.0, 0: 4.0 / 6.0, 1: 1.0 / 6.0}
    offs = [(0, 0, 0)] + _OFFS27

    def coef(k, coords):
        o = offs[k]
        x, y, z = coords
        p = x + N * y + N * N * z
        q = np.clip(p + o[0] + N * o[1] + N * N * o[2], 0, N ** 3 - 1)
        return w1[o[0]] * w1[o[1]] * w1[o[2]] * sq[p] * sq[q]

    return _assemble((N, N, N), offs, coef, symmetric=True)


def convdiff_2d(N: int, beta_x: float, beta_y: float) -> CSR:
    """h^2-scaled 2-D convection-diffusion operator, first-order upwind (beta > 0).

    h = 1/(N+1); centre 4 + h*bx + h*by, west -(1 + h*bx), south -(1 + h*by),
    east -1, north -1.  Real and nonsymmetric.
    """
    h = 1.0 / (N + 1)
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    w = [4.0 + h * beta_x + h * beta_y, -(1.0 + h * beta_x), -1.0, -(1.0 + h * beta_y), -1.0]

    def coef(k, coords):
        return np.full(coords.shape[1], w[k])

    return _assemble((N, N), offs, coef, symmetric=False)
