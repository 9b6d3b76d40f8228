"""Pins for the oracle's Rayleigh-Ritz, quadrature sum and full IFEAST/FEAST solves.

Whole solves are checked against closed-form spectra and dense eigensolvers;
the filter against a dense spectral evaluation of rho_hat(A) X (Eq. rhoh).
"""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from oracle.feast import filter_gain, classify
from oracle.quadrature import contour_nodes, rho_hat
import workloads as W


def _lap_exact(N):
    mu = 2 - 2 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    return np.sort((mu[:, None] + mu[None, :]).ravel())


def test_rayleigh_ritz_exact_subspace():
    A = W.laplacian_2d(10).to_scipy()
    lam, V = np.linalg.eigh(A.toarray())
    rng = np.random.default_rng(0)
    idx = [3, 7, 8, 20, 21]
    Q = V[:, idx] @ rng.standard_normal((5, 5))  # same span, mixed basis
    l, X, AX, BX, C = O.rayleigh_ritz(A, None, Q)
    assert np.allclose(l, lam[idx], atol=1e-12)
    R, r = O.residuals(AX, BX, l)
    assert r.max() < 1e-12
    assert np.allclose(X.T @ X, np.eye(5), atol=1e-12)
    assert np.allclose(Q @ C, X, atol=1e-12)


def test_rayleigh_ritz_generalized_matches_scipy():
    A = W.spd27(4, 1).to_scipy()
    B = W.mass27(4, 2).to_scipy()
    rng = np.random.default_rng(1)
    Q = rng.standard_normal((64, 6))
    l, X, AX, BX, C = O.rayleigh_ritz(A, B, Q)
    ref = sla.eigh(Q.T @ A @ Q, Q.T @ B @ Q, eigvals_only=True)
    assert np.allclose(l, ref, rtol=1e-11)
    assert np.allclose(X.T @ (B @ X), np.eye(6), atol=1e-11)


def test_quad_accumulate_equals_dense_filter():
    # exact shifted solves: X rho_hat(Lambda) + sum 2 Re w_k D_k = rho_hat(A) X
    A = W.laplacian_2d(12).to_scipy()
    Ad = A.toarray()
    evals, evecs = np.linalg.eigh(Ad)
    contour = {"kind": "half", "emin": 0.5, "emax": 0.8, "rule": "gl", "nc": 8}
    z, w, half = contour_nodes(contour)
    rng = np.random.default_rng(2)
    X0 = rng.standard_normal((144, 6))
    lam, X, AX, BX, _ = O.rayleigh_ritz(A, None, X0)
    R, _ = O.residuals(AX, BX, lam)
    D = [np.linalg.solve(zk * np.eye(144) - Ad, R / (zk - lam)[None, :]) for zk in z]
    Q = O.quad_accumulate(X, lam, D, z, w, half)
    dense = evecs @ (rho_hat(evals, z, w, True)[:, None] * (evecs.T @ X))
    assert np.allclose(Q, dense, atol=1e-11)


def test_filter_gain_exact_filter():
    A = W.laplacian_2d(10).to_scipy()
    lam_all, V = np.linalg.eigh(A.toarray())
    contour = {"kind": "half", "emin": 0.5, "emax": 1.5, "rule": "gl", "nc": 8}
    z, w, half = contour_nodes(contour)
    X = V[:, 10:16]
    gam = rho_hat(lam_all[10:16], z, w, True)
    Q = X * gam[None, :]
    l, Xn, AX, BX, C = O.rayleigh_ritz(A, None, Q)
    eta = filter_gain(C, np.eye(6))
    assert np.allclose(np.sort(eta), np.sort(np.abs(gam)), rtol=1e-10)
    ins, spur, rf = classify(l, np.zeros(6), eta, contour, z, w, half, 0.1)
    assert not spur.any()


def test_ifeast_config1_closed_form():
    p = W.config1()
    res = O.ifeast(p.A, None, p.contour, p.m0, p.max_inner, p.alpha, p.tol, p.x0(), p.max_outer,
                   max_cycles=p.max_cycles, inner_rule=p.inner_rule, tau=p.tau)
    exact = _lap_exact(20)
    want = exact[(exact > 0.5) & (exact < 0.8)]
    assert res.converged and res.m == len(want) == 11
    assert np.allclose(np.sort(res.lam_in), want, rtol=1e-10, atol=0)
    assert res.resid[res.inside].max() <= p.tol
    # B-orthonormal Ritz vectors; the cluster subspaces match the dense eigenvectors
    Xin = res.X_in
    assert np.allclose(Xin.T @ Xin, np.eye(11), atol=1e-10)
    lam_d, V_d = np.linalg.eigh(p.A.to_dense())
    Vin = V_d[:, (lam_d > 0.5) & (lam_d < 0.8)]
    sines = np.linalg.svd(Vin - Xin @ (Xin.T @ Vin), compute_uv=False)
    assert sines.max() < 1e-8
    # linear outer convergence: the history falls by orders of magnitude
    assert res.rf_hist[-1] < 1e-6 * res.rf_hist[0]


def test_ifeast_literal_mode_converges():
    p = W.config1()
    res = O.ifeast(p.A, None, p.contour, p.m0, p.max_inner, p.alpha, p.tol, p.x0(), p.max_outer,
                   mode="literal", max_cycles=p.max_cycles, inner_rule="column", tau=p.tau)
    exact = _lap_exact(20)
    want = exact[(exact > 0.5) & (exact < 0.8)]
    assert res.converged and np.allclose(np.sort(res.lam_in), want, rtol=1e-10, atol=0)


def test_feast_direct_rate_matches_filter_ratio():
    # Algorithm 1 with exact solves converges at about |gamma_{m0+1}| / |gamma_m| per iteration.
    p = W.config1()
    res = O.feast_direct(p.A, None, p.contour, p.x0(), 1e-12)
    exact = _lap_exact(20)
    z, w, half = contour_nodes(p.contour)
    g = np.sort(np.abs(rho_hat(exact, z, w, True)))[::-1]
    rate = g[p.m0] / g[10]
    assert res.converged and res.outer_iters <= 5
    h = res.rf_hist
    observed = h[-1] / h[-2]
    assert observed < 30 * rate
    want = exact[(exact > 0.5) & (exact < 0.8)]
    assert np.allclose(np.sort(res.lam_in), want, rtol=1e-11, atol=0)


def test_ifeast_generalized_small_vs_dense():
    p = W.config3_small(N=6, m0=12, emin=0.0, emax=1.0)
    lam_in, V_in, lam_all = O.dense_reference(p.A, p.B, {"kind": "half", "emin": 0.0, "emax": 1.0})
    # choose an interval with gaps at both ends from the dense spectrum
    emin = 0.5 * (lam_all[1] + lam_all[2])
    emax = 0.5 * (lam_all[8] + lam_all[9])
    contour = dict(p.contour, emin=emin, emax=emax)
    res = O.ifeast(p.A, p.B, contour, p.m0, p.max_inner, p.alpha, p.tol, p.x0(), p.max_outer,
                   max_cycles=p.max_cycles, inner_rule=p.inner_rule, tau=p.tau)
    want = lam_all[2:9]
    assert res.converged and res.m == 7
    assert np.allclose(np.sort(res.lam_in), want, rtol=1e-10, atol=0)
    B = p.B.to_scipy()
    Xin = res.X_in
    assert np.allclose(Xin.T @ (B @ Xin), np.eye(7), atol=1e-9)


def test_ifeast_nonhermitian_small_closed_form():
    N = 16
    h = 1.0 / (N + 1)
    j = np.arange(1, N + 1)

    def mu(b):
        return 2 + h * b - 2 * np.sqrt(1 + h * b) * np.cos(j * np.pi / (N + 1))

    exact = np.sort((mu(20.0)[:, None] + mu(10.0)[None, :]).ravel())
    c, r = 0.5 * (exact[3] + exact[9]), 0.5 * (exact[9] - exact[3])
    # put the circle through mid-gaps
    lo = 0.5 * (exact[2] + exact[3])
    hi = 0.5 * (exact[9] + exact[10])
    c, r = 0.5 * (lo + hi), 0.5 * (hi - lo)
    p = W.config4_small(N=N, m0=16, c=c, r=r)
    # a full-dimension Krylov space (k * m0 >= n) makes the inner solves exact, so this
    # pins the non-Hermitian Rayleigh-Ritz and full-circle quadrature against the closed form
    res = O.ifeast(p.A, None, p.contour, p.m0, N * N // p.m0 + 1, 0.0, p.tol, p.x0(), 10,
                   kind="general", max_cycles=1, inner_rule=p.inner_rule, tau=p.tau)
    want = exact[3:10]
    assert res.converged and res.m == 7
    assert np.allclose(np.sort(res.lam_in.real), want, rtol=1e-9, atol=0)
    assert np.abs(res.lam_in.imag).max() < 1e-8
    d = O.feast_direct(p.A, None, p.contour, p.x0(), 1e-10, 10, kind="general")
    assert d.converged and np.allclose(np.sort(d.lam_in.real), want, rtol=1e-9, atol=0)


def test_lobpcg_reference_matches_dense():
    N = 10
    A = W.laplacian_3d(N, W.random_potential(N ** 3, 1002))
    vals, res = O.lowest_eigenvalues_lap3d(A, N, 24)
    dense = np.linalg.eigvalsh(A.to_dense())[:20]
    assert np.allclose(vals[:20], dense, rtol=1e-10, atol=0)
    assert res[:20].max() < 1e-7


def test_classify_flags_junk_pair_from_damped_components():
    """A Ritz pair built from two damped eigenvectors on either side of the interval has its
    Rayleigh quotient inside the interval but a filter gain equal to the damping, far below
    |rho_hat| there: classify must flag it and keep it out of m and ||R_F||."""
    lam_all = np.array([0.1, 0.2, 0.9, 1.1, 1.8, 1.9, 3.0, 4.0])
    n = len(lam_all)
    A = np.diag(lam_all)
    contour = {"kind": "half", "emin": 0.5, "emax": 1.5, "rule": "gl", "nc": 8}
    z, w, half = contour_nodes(contour)
    E = np.eye(n)
    # two genuine directions (0.9, 1.1), one mix of 0.2 and 1.8 (symmetric about the centre 1.0)
    X = np.column_stack([E[:, 2], E[:, 3], (E[:, 1] + E[:, 4]) / np.sqrt(2.0)])
    gam = rho_hat(lam_all, z, w, True)
    Q = (gam[:, None] * E) @ X  # the exact filter rho_hat(A) X
    l, Xn, AX, BX, C = O.rayleigh_ritz(A, None, Q)
    R, r = O.residuals(AX, BX, l)
    eta = filter_gain(C, X.T @ X)
    junk = np.argmin(np.abs(l - 1.0))
    assert 0.5 < l[junk] < 1.5 and abs(l[junk] - 1.0) < 1e-9  # the mix's quotient sits at the centre
    # its gain is the damping |rho_hat(0.2)| = |rho_hat(1.8)|, against |rho_hat(1.0)| ~ 1
    assert abs(eta[junk] - abs(gam[1])) < 1e-12 and eta[junk] < 0.1 * abs(rho_hat(np.array([1.0]), z, w, True)[0])
    ins, spur, rf = classify(l, r, eta, contour, z, w, half, 0.5)
    assert spur[junk] and not ins[junk]
    assert ins.sum() == 2 and not spur[np.arange(3) != junk].any()
    assert r[junk] > 0.5 and rf < 1e-12  # the junk residual (~0.8) does not enter ||R_F||


def test_ifeast_status_m0_too_small_and_no_eig():
    """Algorithm 2's premise (fewer than m0 eigenvalues inside, at least one): the literal
    configuration-1 interval holds 26 > m0 = 16 eigenvalues, an interval inside a spectral gap
    holds none; both end after the first filter application."""
    exact = _lap_exact(20)
    p = W.config1()
    wide = dict(p.contour, emin=0.5, emax=1.2)
    assert ((exact > 0.5) & (exact < 1.2)).sum() == 26
    res = O.ifeast(p.A, None, wide, p.m0, p.max_inner, p.alpha, p.tol, p.x0(), p.max_outer,
                   max_cycles=p.max_cycles, inner_rule=p.inner_rule, tau=p.tau)
    assert res.status == "m0_too_small" and res.outer_iters == 1 and not res.converged
    gap = int(np.argmax(np.diff(exact[:60])))
    lo, hi = exact[gap], exact[gap + 1]
    empty = dict(p.contour, emin=lo + 0.1 * (hi - lo), emax=hi - 0.1 * (hi - lo))
    assert not ((exact > empty["emin"]) & (exact < empty["emax"])).any()
    res = O.ifeast(p.A, None, empty, p.m0, p.max_inner, p.alpha, p.tol, p.x0(), p.max_outer,
                   max_cycles=p.max_cycles, inner_rule=p.inner_rule, tau=p.tau)
    assert res.status == "no_eig" and res.m == 0 and res.outer_iters == 1
    res = O.ifeast(p.A, None, p.contour, p.m0, p.max_inner, p.alpha, p.tol, p.x0(), p.max_outer,
                   max_cycles=p.max_cycles, inner_rule=p.inner_rule, tau=p.tau)
    assert res.status == "ok" and res.m == 11


def test_ifeast_minres_inner_closed_form():
    """IFEAST with MINRES inner solves (the paper's experiments) reaches configuration 1's
    closed-form eigenvalues."""
    p = W.config1()
    res = O.ifeast(p.A, None, p.contour, p.m0, p.max_inner, p.alpha, p.tol, p.x0(), p.max_outer,
                   max_cycles=p.max_cycles, inner_rule=p.inner_rule, tau=p.tau, inner="minres")
    exact = _lap_exact(20)
    want = exact[(exact > 0.5) & (exact < 0.8)]
    assert res.converged and res.m == 11 and res.status == "ok"
    assert np.allclose(np.sort(res.lam_in), want, rtol=1e-10, atol=0)
