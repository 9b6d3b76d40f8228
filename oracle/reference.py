"""Reference low spectra of the 3-D Laplacian + diagonal potential at sizes
where a dense eigensolver is out of reach.

Test infrastructure (see the package docstring).

The reference is scipy's LOBPCG (a library eigensolver, independent of any
contour integration) preconditioned by the exact inverse of the shifted pure
7-point Laplacian: L = S diag(mu) S with S the orthonormal type-I discrete
sine transform in each direction and mu the sums of 2 - 2 cos(j pi/(N+1)),
so (L + sigma I)^{-1} x = S diag(1/(mu + sigma)) S x.  The potential enters
only through the operator, never through the preconditioner.
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sf
import scipy.sparse.linalg as spla


def _dst_preconditioner(N: int, sigma: float):
    mu = 2.0 - 2.0 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    lam0 = mu[:, None, None] + mu[None, :, None] + mu[None, None, :]

    def apply(X):
        X = np.asarray(X)
        m = X.shape[1] if X.ndim == 2 else 1
        Y = sf.dstn(X.reshape(N, N, N, m), type=1, norm="ortho", axes=(0, 1, 2))
        Y /= (lam0 + sigma)[..., None]
        return sf.dstn(Y, type=1, norm="ortho", axes=(0, 1, 2)).reshape(N ** 3, m)

    return spla.LinearOperator((N ** 3, N ** 3), matvec=apply, matmat=apply, dtype=float)


def lowest_eigenvalues_lap3d(A, N: int, k: int, sigma: float = 1.0, seed: int = 0, tol: float = 1e-9,
                             maxiter: int = 250):
    """The k lowest eigenvalues of A (a 3-D Laplacian + potential on an N^3 grid)
    and their residual norms, by preconditioned LOBPCG."""
    if hasattr(A, "to_scipy"):
        A = A.to_scipy()
    X0 = np.random.default_rng(seed).standard_normal((N ** 3, k))
    vals, vecs = spla.lobpcg(A, X0, M=_dst_preconditioner(N, sigma), largest=False, tol=tol, maxiter=maxiter)
    order = np.argsort(vals)
    vals, vecs = vals[order], vecs[:, order]
    res = np.linalg.norm(A @ vecs - vecs * vals[None, :], axis=0)
    return vals, res
