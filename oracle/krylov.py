"""Block GMRES on one shifted system (z B - A) Y = RHS.

Test infrastructure (see the package docstring).

IFEAST solves its shifted systems with a Krylov method stopped early
(Algorithm 2, step 1).  The paper's analysis uses GMRES (Sec. 2.2) and
writes its iterate as the minimiser of the residual over the Krylov space
(Sec. 3.2: Y = V (V^H M^H M V)^{-1} V^H M^H X).  This is the block version
with block size m (every column minimised over the same block Krylov
space), built by block Arnoldi (Sec. 3.1):

    V_1 S = qr(RHS)
    for j = 1..k:
        W = M V_j
        H_{i,j} = V_i^H W, W -= V_i H_{i,j}   (all i <= j, classical, two passes)
        V_{j+1} H_{j+1,j} = qr(W)
        Y_j = argmin || E_1 S - Hbar_j Y ||  (column by column, lstsq)
        stop when every column residual <= tol
    D = [V_1 .. V_j] Y_j

so M [V_1..V_j] = [V_1..V_{j+1}] Hbar_j and the small least-squares residual
equals the true residual ||RHS - M D|| column by column.

``block_gmres_restarted`` repeats such cycles of at most k block iterations
(block GMRES(k)), each from the current true residual, until the stopping
rule holds: the number of block iterations per cycle bounds the basis to
k+1 blocks, while Algorithm 2's tolerance decides when the solve ends.
"""

from __future__ import annotations

import numpy as np


def shifted_operator(A, B, z):
    """Return v -> (z B - A) v for sparse A, B (B None means the identity)."""
    if B is None:
        return lambda V: z * V - A @ V
    return lambda V: z * (B @ V) - A @ V


def block_gmres(apply_M, rhs: np.ndarray, k: int, tol=0.0):
    """One block GMRES cycle: block size rhs.shape[1], at most k block iterations.

    ``tol`` is a scalar or one value per column.  Returns (D, info): D is the
    n x m iterate (zero initial guess); info holds ``iters`` (block
    iterations done), ``res`` (final per-column residual norms of the small
    problem), ``res_hist`` (row 0 = ||rhs|| per column, then one row per
    iteration), ``H`` (block Hessenberg Hbar), ``V`` (basis list), ``S`` and
    ``Y``.
    """
    rhs = np.asarray(rhs, dtype=complex)
    n, m = rhs.shape
    tol = np.broadcast_to(np.asarray(tol, dtype=float), (m,))
    V1, S = np.linalg.qr(rhs)
    V = [V1]
    H = np.zeros(((k + 1) * m, k * m), dtype=complex)
    E1S = np.zeros(((k + 1) * m, m), dtype=complex)
    E1S[:m] = S
    hist = [np.linalg.norm(rhs, axis=0)]
    Y = np.zeros((0, m), dtype=complex)
    res = hist[0]
    iters = 0
    for j in range(k):
        W = apply_M(V[j])
        basis = np.hstack(V)
        for _ in range(2):  # classical Gram-Schmidt, applied twice
            h = basis.conj().T @ W
            W = W - basis @ h
            H[: (j + 1) * m, j * m:(j + 1) * m] += h
        Vn, Rn = np.linalg.qr(W)
        H[(j + 1) * m:(j + 2) * m, j * m:(j + 1) * m] = Rn
        V.append(Vn)
        Hj = H[: (j + 2) * m, : (j + 1) * m]
        g = E1S[: (j + 2) * m]
        Y = np.linalg.lstsq(Hj, g, rcond=None)[0]
        res = np.linalg.norm(g - Hj @ Y, axis=0)
        hist.append(res)
        iters = j + 1
        if np.all(res <= tol):
            break
    D = np.hstack(V[:iters]) @ Y if iters else np.zeros_like(rhs)
    info = {"iters": iters, "res": res, "res_hist": np.array(hist), "H": H[: (iters + 1) * m, : iters * m],
            "V": V, "S": S, "Y": Y}
    return D, info


def block_gmres_restarted(apply_M, rhs: np.ndarray, k: int, tol, max_cycles: int):
    """Block GMRES(k) restarted until every column residual is <= tol.

    ``tol`` is a scalar or one value per column.  Returns (D, info) with
    ``iters`` = total block iterations, ``cycles`` and ``res`` = true
    residual column norms ||rhs - M D||.
    """
    rhs = np.asarray(rhs, dtype=complex)
    m = rhs.shape[1]
    tol = np.broadcast_to(np.asarray(tol, dtype=float), (m,))
    D = np.zeros_like(rhs)
    res = np.linalg.norm(rhs, axis=0)
    iters = cycles = 0
    while cycles < max_cycles and not np.all(res <= tol):
        d, info = block_gmres(apply_M, rhs - apply_M(D) if cycles else rhs, k, tol)
        D = D + d
        iters += info["iters"]
        cycles += 1
        res = np.linalg.norm(rhs - apply_M(D), axis=0)
    return D, {"iters": iters, "cycles": cycles, "res": res}
