"""Pins for the oracle's quadrature and rational filter (Eq. contour_int_quad, Eq. rhoh).

Each check compares against something the mathematics fixes, not against a
retyped formula: closed forms of the trapezoidal filter, exact values of
symmetric rules at special points, brute-force contour integration.
"""

import numpy as np

from oracle.quadrature import gauss_legendre_half, trapezoid_circle, trapezoid_half, rho_hat, contour_nodes


def _brute_contour_integral(f, c, r, npts=200000):
    """(1/2 pi i) closed-contour integral of f by a fine midpoint sum (independent of the rules)."""
    th = (np.arange(npts) + 0.5) * 2 * np.pi / npts
    z = c + r * np.exp(1j * th)
    dz = 1j * r * np.exp(1j * th) * (2 * np.pi / npts)
    return np.sum(f(z) * dz) / (2j * np.pi)


def test_brute_force_projector_values():
    # the exact filter is the indicator of the disc (Eq. contourprojector)
    for lam, want in [(0.65, 1.0), (0.5001, 1.0), (0.9, 0.0), (0.3, 0.0)]:
        val = _brute_contour_integral(lambda z: 1.0 / (z - lam), 0.65, 0.15)
        assert abs(val - want) < 1e-6


def test_gauss_legendre_half_special_values():
    emin, emax = 0.5, 0.8
    for nc in (4, 8, 12, 16):
        z, w = gauss_legendre_half(emin, emax, nc)
        assert np.all(z.imag > 0)
        assert np.allclose(np.abs(z - 0.65), 0.15)
        # rho_hat(c) = 2 Re sum g_k / 4 = 1
        assert abs(rho_hat(0.65, z, w, True) - 1.0) < 1e-14
        # endpoints: Re[1 / (1 - e^{-i theta})] = 1/2 for every node
        assert abs(rho_hat(emin, z, w, True) - 0.5) < 1e-13
        assert abs(rho_hat(emax, z, w, True) - 0.5) < 1e-13
    # approaches the indicator as nc grows (Eq. rhoh)
    z, w = gauss_legendre_half(emin, emax, 32)
    assert abs(rho_hat(0.6, z, w, True) - 1.0) < 1e-6
    assert abs(rho_hat(1.0, z, w, True)) < 1e-6


def test_gauss_legendre_half_matches_brute_force_integral():
    # with real lambda, 2 Re of the upper half equals the full contour integral
    z, w = gauss_legendre_half(0.5, 0.8, 8)
    for lam in (0.55, 0.7, 0.45, 0.95, 2.0):
        brute = _brute_contour_integral(lambda zz: 1.0 / (zz - lam), 0.65, 0.15).real
        approx = rho_hat(lam, z, w, True)
        # GL8 is a good rule away from the circle: agreement to a few digits
        if abs(lam - 0.65) > 0.2:
            assert abs(approx - brute) < 1e-3


def test_trapezoid_closed_form():
    c, r, nc = 0.3, 0.2, 16
    z, w = trapezoid_circle(c, r, nc)
    assert abs(np.sum(w)) < 1e-15
    lam = np.array([0.3, 0.31, 0.45, 0.1000001, 0.7, -1.0, 0.3 + 0.05j, 0.6 - 0.1j])
    t = (lam - c) / r
    exact = 1.0 / (1.0 + t ** nc)
    assert np.allclose(rho_hat(lam, z, w, False), exact, atol=1e-13)


def test_trapezoid_half_is_conjugate_half_of_full_rule():
    emin, emax, nc = 0.5, 0.8, 4
    zh, wh = trapezoid_half(emin, emax, nc)
    zf, wf = trapezoid_circle(0.65, 0.15, 2 * nc)
    lam = np.linspace(0.3, 1.0, 17)
    assert np.allclose(rho_hat(lam, zh, wh, True), rho_hat(lam, zf, wf, False).real, atol=1e-14)
    t = (lam - 0.65) / 0.15
    assert np.allclose(rho_hat(lam, zh, wh, True), 1 / (1 + t ** (2 * nc)), atol=1e-13)


def test_contour_nodes_dispatch():
    z, w, half = contour_nodes({"kind": "half", "emin": 0.0, "emax": 1.0, "rule": "gl", "nc": 8})
    assert half and len(z) == 8
    z, w, half = contour_nodes({"kind": "circle", "c": 0.2, "r": 0.1, "rule": "trap", "nc": 16})
    assert not half and len(z) == 16
