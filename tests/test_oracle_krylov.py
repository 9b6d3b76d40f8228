"""Pins for the oracle's block GMRES (Sec. 2.2, Sec. 3.1, Sec. 3.2)."""

import numpy as np
import scipy.sparse as sp

from oracle.krylov import block_gmres, block_gmres_restarted, shifted_operator

import workloads as W


def _small_problem(n=60, m=3, seed=0):
    """Random symmetric A (simple eigenvalues, so a block Krylov space can fill C^n) and RHS."""
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    A = sp.csr_matrix(M + M.T)
    R = rng.standard_normal((n, m)) + 1j * rng.standard_normal((n, m))
    return A, R


def test_full_krylov_space_gives_exact_solve():
    A, R = _small_problem(n=36, m=4)
    z = 1.7 + 0.3j
    M = shifted_operator(A, None, z)
    k = 36 // 4 + 1
    D, info = block_gmres(M, R, k, 0.0)
    exact = np.linalg.solve(z * np.eye(36) - A.toarray(), R)
    assert np.allclose(D, exact, atol=1e-9)


def test_normal_equation_closed_form():
    # Sec. 3.2: Y = V (V^H M^H M V)^{-1} V^H M^H X, V any orthonormal basis of the block Krylov space.
    A, R = _small_problem(n=64, m=3, seed=1)
    z = 3.1 + 0.2j
    Md = z * np.eye(64) - A.toarray()
    k = 3
    D, info = block_gmres(shifted_operator(A, None, z), R, k, 0.0)
    # independent basis: QR of the explicit power basis [R, M R, M^2 R]
    K = np.hstack([np.linalg.matrix_power(Md, p) @ R for p in range(k)])
    V, _ = np.linalg.qr(K)
    MV = Md @ V
    Y = V @ np.linalg.solve(MV.conj().T @ MV, MV.conj().T @ R)
    assert np.allclose(D, Y, atol=1e-10)
    # minimal residual: any other element of the space does no better, column by column
    res = np.linalg.norm(R - Md @ D, axis=0)
    rng = np.random.default_rng(2)
    for _ in range(5):
        other = D + V @ (1e-3 * rng.standard_normal((V.shape[1], 3)))
        assert np.all(np.linalg.norm(R - Md @ other, axis=0) >= res - 1e-12)
    assert np.allclose(info["res"], res, atol=1e-10)


def test_arnoldi_relation_and_orthonormality():
    A, R = _small_problem(n=100, m=4, seed=3)
    z = 0.4 + 0.05j
    Md = z * np.eye(100) - A.toarray()
    D, info = block_gmres(shifted_operator(A, None, z), R, 5, 0.0)
    V = np.hstack(info["V"])
    j = info["iters"]
    assert np.allclose(V.conj().T @ V, np.eye(V.shape[1]), atol=1e-12)
    # M V_{1:j} = V_{1:j+1} Hbar_j
    assert np.allclose(Md @ V[:, : 4 * j], V @ info["H"], atol=1e-11)
    # shift invariance of the Krylov space (Sec. 3): H = z I - V^H A V on the square part
    Vj = V[:, : 4 * j]
    assert np.allclose(info["H"][: 4 * j], z * np.eye(4 * j) - Vj.conj().T @ A.toarray() @ Vj, atol=1e-11)
    # residual norms never increase
    hist = info["res_hist"]
    assert np.all(np.diff(hist, axis=0) <= 1e-12)


def test_stopping_rule_and_restarts():
    A, R = _small_problem(n=100, m=2, seed=4)
    z = 2.0 + 12.0j  # well away from the spectrum: fast convergence
    M = shifted_operator(A, None, z)
    D1, info1 = block_gmres(M, R, 50, 1e-6)
    assert info1["iters"] < 50 and np.all(info1["res"] <= 1e-6)
    D2, info2 = block_gmres_restarted(M, R, 3, 1e-8, 200)
    assert np.all(info2["res"] <= 1e-8) and info2["cycles"] > 1
    exact = np.linalg.solve(z * np.eye(100) - A.toarray(), R)
    assert np.allclose(D2, exact, atol=1e-6)
    # per-column tolerances: a zero column needs no work
    Rz = R.copy()
    Rz[:, 1] = 0
    D3, info3 = block_gmres_restarted(M, Rz, 3, np.array([1e-8, 1e-8]), 200)
    assert np.allclose(D3[:, 1], 0)


def test_generalized_operator():
    rng = np.random.default_rng(5)
    A = sp.csr_matrix(W.spd27(3, 9).to_dense())
    B = sp.csr_matrix(W.mass27(3, 9).to_dense())
    z = 5.0 + 0.5j
    R = rng.standard_normal((27, 2))
    D, info = block_gmres(shifted_operator(A, B, z), R, 14, 0.0)
    exact = np.linalg.solve(z * B.toarray() - A.toarray(), R)
    assert np.allclose(D, exact, atol=1e-8)


def test_minres_columns_are_minimal_residual_iterates():
    """MINRES's k-step iterate minimises ||b - M y|| over K_k(M, b): for a complex-shifted symmetric
    matrix it equals the projection solution computed from an explicit Krylov matrix (normal
    equations of the minimisation), column by column, and the residual does not grow with k."""
    import oracle as O

    rng = np.random.default_rng(7)
    n = 60
    A = rng.standard_normal((n, n))
    A = A + A.T
    z = 0.3 + 0.7j
    M = lambda V: z * V - A @ V
    B = rng.standard_normal((n, 3))
    prev = np.full(3, np.inf)
    for k in (1, 3, 6):
        D, its = O.minres_columns(M, B, k, 0.0)
        assert its == [k, k, k]
        for c in range(3):
            b = B[:, c].astype(complex)
            K = np.column_stack([np.linalg.matrix_power(z * np.eye(n) - A, i) @ b for i in range(k)])
            MK = (z * np.eye(n) - A) @ K
            coef = np.linalg.lstsq(MK, b, rcond=None)[0]
            assert np.allclose(D[:, c], K @ coef, rtol=1e-8, atol=1e-10 * np.abs(b).max())
        r = np.linalg.norm(B - M(D), axis=0)
        assert np.all(r <= prev * (1 + 1e-12))
        prev = r
    # a full-dimension space solves exactly
    D, _ = O.minres_columns(M, B, n, 0.0)
    assert np.allclose(D, np.linalg.solve(z * np.eye(n) - A, B), rtol=1e-8, atol=1e-10)
