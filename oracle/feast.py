"""IFEAST (Algorithm 2) and FEAST (Algorithm 1) in plain FP64 numpy/scipy.

Test infrastructure (see the package docstring).

Readings taken where the paper is silent (each listed with its reason in the
design notes of the repository):

* Initial ||R_F||: computed exactly by a Rayleigh-Ritz on X0 (the footnote of
  Algorithm 2 allows it); the literal mode uses ||R_F|| = 1 instead.
* Inner initial guess ("ritz" mode): Y0_k = X (z_k - Lambda)^{-1}.  Then the
  residual of (z_k B - A) Y = B X at Y0 is R (z_k - Lambda)^{-1} with
  R = A X - B X Lambda, so each shifted system is solved for the correction
  D_k = Y_k - Y0_k from that right-hand side, and the quadrature sum becomes
  Q = X rho_hat(Lambda) + sum_k w_k D_k.  "literal" mode starts from Y0 = 0
  with right-hand side B X, as Algorithm 2 is printed.
* Inner stopping rule: Algorithm 2's unscaled ||B X - (z_k B - A) Y_k|| <=
  alpha ||R_F||, column by column, all columns of a shift at once, at most
  ``max_inner`` block iterations.
* Rayleigh-Ritz (Algorithm 2, step 3): A_Q = Q^T A Q and B_Q = Q^T B Q; the
  reduced generalized problem is solved by B-orthonormalising Q with SVQB
  (scale by diag(B_Q)^{-1/2}, eigendecompose, floor tiny eigenvalues at
  eps * m0 * max) and a standard symmetric eigensolve.  Non-Hermitian
  problems (right-only Galerkin): orthonormalise Q, eig(Q^H A Q).
* Residual (Algorithm 2, step 4): ||A x_j - lambda_j B x_j||_2 with x_j
  B-normalised (unit 2-norm for general problems); ||R_F|| is the max over
  the pairs inside the contour (over all pairs if none is inside).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .quadrature import contour_nodes, rho_hat
from .krylov import block_gmres, block_gmres_restarted, shifted_operator


def _sparse(M):
    if M is None:
        return None
    if hasattr(M, "to_scipy"):
        return M.to_scipy()
    return sp.csr_matrix(M)


def inside_contour(lam, contour: dict) -> np.ndarray:
    """Membership of eigenvalues: open interval (emin, emax) or open disc |lambda - c| < r."""
    lam = np.asarray(lam)
    if contour["kind"] in ("half", "explicit"):
        lo, hi = contour["emin"], contour["emax"]
        return (lam.real > lo) & (lam.real < hi)
    return np.abs(lam - contour["c"]) < contour["r"]


def rayleigh_ritz(A, B, Q, kind: str = "symmetric"):
    """Rayleigh-Ritz on span(Q) (Algorithm 2, step 3).

    Returns (lam, X, AX, BX, C) with X = Q C, sorted ascending (by real then
    imaginary part).
    """
    A = _sparse(A)
    B = _sparse(B)
    m0 = Q.shape[1]
    if kind == "symmetric":
        Q = np.asarray(Q, dtype=np.float64)
        AQ = A @ Q
        BQ = Q if B is None else B @ Q
        AQr = Q.T @ AQ
        BQr = Q.T @ BQ
        AQr = 0.5 * (AQr + AQr.T)
        BQr = 0.5 * (BQr + BQr.T)
        # SVQB: B-orthonormalise the basis, then a standard eigenproblem.
        d = 1.0 / np.sqrt(np.diag(BQr))
        Gs = d[:, None] * BQr * d[None, :]
        theta, U = np.linalg.eigh(Gs)
        theta = np.maximum(theta, np.finfo(float).eps * m0 * theta.max())
        T = (d[:, None] * U) / np.sqrt(theta)[None, :]
        Ar = T.T @ AQr @ T
        lam, W = np.linalg.eigh(0.5 * (Ar + Ar.T))
        C = T @ W
        return lam, Q @ C, AQ @ C, BQ @ C, C
    # general (non-Hermitian): right-only Galerkin on an orthonormal basis
    Q = np.asarray(Q, dtype=complex)
    Qo, Rq = np.linalg.qr(Q)
    AQ = A @ Qo
    lam, XQ = np.linalg.eig(Qo.conj().T @ AQ)
    order = np.lexsort((lam.imag, lam.real))
    lam, XQ = lam[order], XQ[:, order]
    XQ = XQ / np.linalg.norm(XQ, axis=0)[None, :]
    X = Qo @ XQ
    BX = X if B is None else B @ X
    C = np.linalg.solve(Rq, XQ)
    return lam, X, AQ @ XQ, BX, C


def residuals(AX, BX, lam):
    """Eigen-residual block R = A X - B X Lambda and its column 2-norms."""
    R = AX - BX * lam[None, :]
    return R, np.linalg.norm(R, axis=0)


def quad_accumulate(X, lam, D, z, w, half: bool):
    """Q = X rho_hat(Lambda) + sum_k w_k D_k  (2 Re of the sum on a half contour).

    This is Algorithm 2, step 2 (Q = sum_k w_k Y_k) with Y_k = X (z_k - Lambda)^{-1} + D_k.
    """
    Q = X * rho_hat(lam, z, w, half)[None, :]
    for wk, Dk in zip(w, D):
        Q = Q + (2.0 * (wk * Dk).real if half else wk * Dk)
    return Q


def filter_gain(C, GX):
    """eta_l = 1 / ||X c_l||_B for new Ritz vectors X' = Q C, Q = filter(X).

    GX = X^H B X of the block that was filtered (the identity when X is
    B-orthonormal).  For a Ritz vector that approximates an eigenvector with
    eigenvalue lambda, eta ~ |rho_hat(lambda)|; a Ritz vector assembled from
    damped components and solve error has eta far below |rho_hat|.
    """
    q = np.einsum("il,ij,jl->l", C.conj(), GX, C).real
    return 1.0 / np.sqrt(np.maximum(q, 1e-300))


@dataclass
class IFeastResult:
    lam: np.ndarray  # all m0 Ritz values, ascending
    X: np.ndarray  # n x m0 Ritz vectors
    resid: np.ndarray  # per-pair residual norms
    inside: np.ndarray  # bool mask of counted pairs inside the contour
    m: int
    outer_iters: int
    converged: bool
    rf_hist: list = field(default_factory=list)
    inner_hist: list = field(default_factory=list)  # block iterations per shift, per outer iteration
    total_matvec: int = 0
    seq_matvec: int = 0
    spurious: np.ndarray = None  # bool mask: inside the contour but failing the filter-gain test
    status: str = "not_converged"  # "ok", "not_converged", "m0_too_small" or "no_eig"

    @property
    def lam_in(self):
        return self.lam[self.inside]

    @property
    def X_in(self):
        return self.X[:, self.inside]


def classify(lam, r, eta, contour, z, w, half, tau):
    """Pairs counted inside the contour, spurious ones, and ||R_F|| (Algorithm 2, step 4).

    A Ritz pair inside the contour counts when its filter gain is consistent,
    eta_l >= tau |rho_hat(lambda_l)|.  ||R_F|| is the max residual over the
    counted pairs (over all inside pairs if none counts, over all pairs if
    none is inside).
    """
    geo = inside_contour(lam, contour)
    ok = eta >= tau * np.abs(rho_hat(lam, z, w, half))
    ins = geo & ok
    if ins.any():
        rf = r[ins].max()
    elif geo.any():
        rf = r[geo].max()
    else:
        rf = r.max()
    return ins, geo & ~ok, float(rf)


def minres_columns(M, rhs, steps: int, tol):
    """MINRES iterates of M y = rhs, column by column (Sec. 2: the paper's inner solver).

    MINRES's iterate after k steps is the vector of the Krylov space K_k(M, b) that minimises
    ||b - M y||, which is what one GMRES cycle with block size 1 computes; each column stops on
    its own when its residual is <= tol (scalar or per column), after at most ``steps`` steps.
    Returns (D, steps per column).
    """
    rhs = np.asarray(rhs, dtype=complex)
    tol = np.broadcast_to(np.asarray(tol, dtype=float), (rhs.shape[1],))
    cols, its = [], []
    for c in range(rhs.shape[1]):
        d, info = block_gmres(M, rhs[:, [c]], steps, tol[c])
        cols.append(d)
        its.append(info["iters"])
    return np.hstack(cols), its


def ifeast(A, B, contour: dict, m0: int, max_inner: int, alpha: float, tol: float, X0: np.ndarray,
           max_outer: int = 50, mode: str = "ritz", kind: str = "symmetric", max_cycles: int = 1,
           inner_rule: str = "global", tau: float = 0.5, callback=None, inner: str = "gmres") -> IFeastResult:
    """IFEAST with block-GMRES(k) inner solves (Algorithm 2), k = max_inner.

    ``inner="minres"``: each column of each shifted system is solved by MINRES (minres_columns)
    for at most max_inner * max_cycles steps instead.

    ``mode``: "ritz" (Y0 = X (z - Lambda)^{-1}) or "literal" (Y0 = 0).
    ``inner_rule``: "global" stops a shift when every column residual is
    <= alpha ||R_F|| (Algorithm 2 as printed); "column" stops column j when
    its residual drops by alpha relative to its start (alpha_j = alpha for
    every eigenvector, Eq. alpha).  ``max_cycles`` restart cycles at most.
    Stops when a counted pair is inside the contour and ||R_F|| <= tol, or
    after ``max_outer`` outer iterations.  Two early exits test the premise
    of Algorithm 2 (fewer than m0 eigenvalues inside the contour, and at
    least one) on the Ritz values after a filter application: all m0 of them
    inside the contour means m0 is too small ("m0_too_small"), none inside
    means the contour holds no eigenvalue ("no_eig").
    """
    A = _sparse(A)
    B = _sparse(B)
    z, w, half = contour_nodes(contour)
    cplx = kind != "symmetric"
    X = np.array(X0, dtype=complex if cplx else np.float64)
    res = IFeastResult(lam=None, X=None, resid=None, inside=None, m=0, outer_iters=0, converged=False)

    def gram(Xb):
        BXb = Xb if B is None else B @ Xb
        return Xb.conj().T @ BXb

    if mode == "ritz":
        lam, X, AX, BX, C = rayleigh_ritz(A, B, X, kind)
        R, r = residuals(AX, BX, lam)
        ins, spur, rf = classify(lam, r, np.full(m0, np.inf), contour, z, w, half, tau)
    else:
        lam, R, r = None, None, None
        BX = X if B is None else B @ X
        rf = 1.0
    for it in range(max_outer):
        D, iters = [], []
        for zk in z:
            M = shifted_operator(A, B, zk)
            rhs = R / (zk - lam)[None, :] if mode == "ritz" else BX
            tol_in = alpha * rf if inner_rule == "global" else alpha * np.linalg.norm(rhs, axis=0)
            if inner == "minres":
                Dk, its = minres_columns(M, rhs, max_inner * max_cycles, tol_in)
                D.append(Dk)
                iters.append(max(its))
                continue
            Dk, info = block_gmres_restarted(M, rhs, max_inner, tol_in, max_cycles)
            D.append(Dk)
            iters.append(info["iters"])
        if mode == "ritz":
            Q = quad_accumulate(X, lam, D, z, w, half)
        else:
            Q = sum((2.0 * (wk * Dk).real if half else wk * Dk) for wk, Dk in zip(w, D))
        GX = gram(X) if (cplx or mode != "ritz" or B is not None) else np.eye(m0)
        lam, X, AX, BX, C = rayleigh_ritz(A, B, Q, kind)
        R, r = residuals(AX, BX, lam)
        eta = filter_gain(C, GX)
        ins, spur, rf = classify(lam, r, eta, contour, z, w, half, tau)
        res.inner_hist.append(iters)
        res.rf_hist.append(rf)
        res.total_matvec += int(sum(iters)) * m0
        res.seq_matvec += int(max(iters))
        res.outer_iters = it + 1
        if callback is not None:
            callback(it, lam, r, ins, rf)
        geo = inside_contour(lam, contour)
        if ins.any() and rf <= tol:
            res.converged = True
            res.status = "m0_too_small" if ins.sum() >= m0 else "ok"
            break
        if geo.all():
            res.status = "m0_too_small"
            break
        if not geo.any():
            res.status = "no_eig"
            break
    res.lam, res.X, res.resid, res.inside, res.m = lam, X, r, ins, int(ins.sum())
    res.spurious = spur
    return res


def feast_direct(A, B, contour: dict, X0: np.ndarray, tol: float, max_outer: int = 30,
                 kind: str = "symmetric") -> IFeastResult:
    """Classical FEAST with direct (sparse LU) solves (Algorithm 1)."""
    A = _sparse(A).tocsc()
    Bs = None if B is None else _sparse(B).tocsc()
    n = A.shape[0]
    z, w, half = contour_nodes(contour)
    Id = sp.identity(n, format="csc")
    lus = [spla.splu((zk * (Id if Bs is None else Bs) - A).astype(complex).tocsc()) for zk in z]
    X = np.array(X0, dtype=complex if kind != "symmetric" else np.float64)
    res = IFeastResult(lam=None, X=None, resid=None, inside=None, m=0, outer_iters=0, converged=False)
    for it in range(max_outer):
        BX = X if Bs is None else Bs @ X
        Q = 0
        for wk, lu in zip(w, lus):
            Yk = lu.solve(np.asarray(BX, dtype=complex))
            Q = Q + (2.0 * (wk * Yk).real if half else wk * Yk)
        lam, X, AX, BXn, _ = rayleigh_ritz(A, Bs, Q, kind)
        _, r = residuals(AX, BXn, lam)
        ins = inside_contour(lam, contour)
        rf = r[ins].max() if ins.any() else r.max()
        res.rf_hist.append(float(rf))
        res.outer_iters = it + 1
        if ins.any() and rf <= tol:
            res.converged = True
            break
    res.lam, res.X, res.resid, res.inside, res.m = lam, X, r, ins, int(ins.sum())
    return res


def dense_reference(A, B, contour: dict, kind: str = "symmetric"):
    """All eigenpairs inside the contour from a dense eigensolver (small n only)."""
    Ad = _sparse(A).toarray()
    Bd = None if B is None else _sparse(B).toarray()
    if kind == "symmetric":
        lam, V = sla.eigh(Ad, Bd)
    else:
        lam, V = (np.linalg.eig(Ad) if Bd is None else sla.eig(Ad, Bd))
        order = np.lexsort((lam.imag, lam.real))
        lam, V = lam[order], V[:, order]
    ins = inside_contour(lam, contour)
    return lam[ins], V[:, ins], lam
