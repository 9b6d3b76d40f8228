"""Seeded generators: structure, symmetry, definiteness and closed-form spectra."""

import numpy as np
import pytest

import workloads as W


def _check_csr(M):
    assert M.rowptr.dtype == np.int64 and M.colind.dtype == np.int32
    assert M.rowptr[0] == 0 and M.rowptr[-1] == len(M.colind) == len(M.val)
    for i in range(M.n):
        c = M.colind[M.rowptr[i]:M.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0), "columns sorted, no duplicates"
        assert c.min() >= 0 and c.max() < M.n


def test_laplacian_2d_structure_and_spectrum():
    A = W.laplacian_2d(20)
    assert A.n == 400 and A.nnz == 1920
    _check_csr(A)
    D = A.to_dense()
    assert np.array_equal(D, D.T)
    # closed form: (2 - 2cos(j pi/21)) + (2 - 2cos(k pi/21))
    j = np.arange(1, 21)
    mu = 2 - 2 * np.cos(j * np.pi / 21)
    exact = np.sort((mu[:, None] + mu[None, :]).ravel())
    assert np.allclose(np.linalg.eigvalsh(D), exact, atol=1e-12)
    # the interval (0.5, 0.8) holds 11 eigenvalues, (0.5, 1.2) holds 26
    assert ((exact > 0.5) & (exact < 0.8)).sum() == 11
    assert ((exact > 0.5) & (exact < 1.2)).sum() == 26


def test_laplacian_3d_with_potential():
    N = 6
    pot = W.random_potential(N ** 3, 1002)
    assert pot.min() >= 0 and pot.max() <= 2
    A = W.laplacian_3d(N, pot)
    _check_csr(A)
    assert A.nnz == 7 * N ** 3 - 6 * N ** 2
    D = A.to_dense()
    assert np.array_equal(D, D.T)
    assert np.allclose(np.diag(D), 6 + pot)
    A0 = W.laplacian_3d(N).to_dense()
    mu = 2 - 2 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    exact = np.sort((mu[:, None, None] + mu[None, :, None] + mu[None, None, :]).ravel())
    assert np.allclose(np.linalg.eigvalsh(A0), exact, atol=1e-12)
    assert W.laplacian_3d(64).nnz == 1810432


def test_spd27_is_spd_and_dominant():
    A = W.spd27(5, 1003)
    _check_csr(A)
    D = A.to_dense()
    assert np.array_equal(D, D.T)
    off = np.abs(D).sum(axis=1) - np.abs(np.diag(D))
    assert np.all(np.diag(D) >= off - 1e-12)
    assert np.linalg.eigvalsh(D).min() > 0
    vals = -D[D < 0]
    assert vals.min() >= 0.1 - 1e-12 and vals.max() <= 10 + 1e-12
    # interior cells have all 26 neighbours
    assert np.diff(A.rowptr).max() == 27


def test_mass27_closed_form_and_density():
    N = 6
    M = W.mass27(N, 7, density=False).to_dense()
    th = np.arange(1, N + 1) * np.pi / (N + 1)
    g = (4 + 2 * np.cos(th)) / 6
    exact = np.sort((g[:, None, None] * g[None, :, None] * g[None, None, :]).ravel())
    assert np.allclose(np.linalg.eigvalsh(M), exact, atol=1e-13)
    assert np.isclose(M[0, 0], 8 / 27)
    B = W.mass27(N, 7).to_dense()
    assert np.allclose(B, B.T) and np.linalg.eigvalsh(B).min() > 0


def test_convdiff_closed_form():
    N, bx, by = 12, 20.0, 10.0
    A = W.convdiff_2d(N, bx, by)
    _check_csr(A)
    h = 1.0 / (N + 1)
    j = np.arange(1, N + 1)

    def mu(b):
        return 2 + h * b - 2 * np.sqrt(1 + h * b) * np.cos(j * np.pi / (N + 1))

    exact = np.sort((mu(bx)[:, None] + mu(by)[None, :]).ravel())
    ev = np.linalg.eigvals(A.to_dense())
    assert np.abs(ev.imag).max() < 1e-8
    assert np.allclose(np.sort(ev.real), exact, atol=1e-9)


def test_seeded_inputs_are_reproducible():
    a = W.initial_block(100, 8, 5)
    b = W.initial_block(100, 8, 5)
    assert a.shape == (100, 8) and a.flags["C_CONTIGUOUS"] and np.array_equal(a, b)
    t = W.poisson_arrivals(20.0, 2000, 3)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 20.0) < 2.0
    reqs = W.serving_requests(10)
    assert reqs == W.serving_requests(10)
    assert all(r["side"] in (32, 48, 64, 96, 128) and r["m0"] in (16, 32, 64, 128) for r in reqs)
