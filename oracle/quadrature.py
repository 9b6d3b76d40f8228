"""Quadrature nodes/weights for the FEAST contour integral and its rational filter.

Test infrastructure (see the package docstring).

The spectral projector is the contour integral (1/2 pi i) \\oint (zI - A)^{-1} X dz
(Eq. contourprojector / contour_int); a quadrature rule replaces it by
sum_k w_k (z_k I - A)^{-1} X (Eq. contour_int_quad).  The paper leaves the
rule open (Gauss, trapezoidal or Zolotarev, Algorithm 1 footnote) and places
the nodes on a circle through the interval ends (Sec. 4.1, Fig. 1 caption).

Parametrising the circle z = c + r e^{i theta} turns the integral into
(1/2 pi) \\int_0^{2 pi} f(z) r e^{i theta} d theta.

* Gauss-Legendre on the upper half circle: theta = (pi/2)(1 - x) maps
  x in [-1, 1] onto theta in [0, pi]; with GL nodes x_k and weights g_k the
  upper half is sum_k g_k (r e^{i theta_k} / 4) f(z_k).  For a real symmetric
  pencil and real X the lower half is the complex conjugate of the upper
  half (Sec. 4.1, half-contour symmetry), so the full sum is 2 Re of it.
* Trapezoidal rule on the full circle: theta_k = 2 pi (k - 1/2)/nc,
  w_k = r e^{i theta_k} / nc.  Its upper half (nc/2 nodes, same weights,
  2 Re) is the half-contour trapezoidal rule of Sec. 4.1.
"""

from __future__ import annotations

import numpy as np


def gauss_legendre_half(emin: float, emax: float, nc: int):
    """nc Gauss-Legendre nodes/weights on the upper half circle through emin, emax.

    Returns complex arrays (z, w); the filter uses 2 Re sum_k w_k / (z_k - lambda).
    """
    x, g = np.polynomial.legendre.leggauss(nc)
    c = 0.5 * (emin + emax)
    r = 0.5 * (emax - emin)
    theta = 0.5 * np.pi * (1.0 - x)
    e = np.exp(1j * theta)
    return c + r * e, g * r * e / 4.0


def trapezoid_circle(c: complex, r: float, nc: int):
    """nc trapezoidal nodes/weights around the whole circle |z - c| = r."""
    k = np.arange(1, nc + 1)
    theta = 2.0 * np.pi * (k - 0.5) / nc
    e = np.exp(1j * theta)
    return c + r * e, r * e / nc


def trapezoid_half(emin: float, emax: float, nc: int):
    """Upper-half nodes of the 2*nc-point trapezoidal rule on the circle through emin, emax."""
    c = 0.5 * (emin + emax)
    r = 0.5 * (emax - emin)
    z, w = trapezoid_circle(c, r, 2 * nc)
    return z[:nc], w[:nc]


def contour_nodes(contour: dict):
    """(z, w, half) for a contour description (see ``workloads.Problem``)."""
    if contour["kind"] == "half":
        if contour.get("rule", "gl") == "gl":
            z, w = gauss_legendre_half(contour["emin"], contour["emax"], contour["nc"])
        else:
            z, w = trapezoid_half(contour["emin"], contour["emax"], contour["nc"])
        return z, w, True
    if contour["kind"] == "circle":
        z, w = trapezoid_circle(contour["c"], contour["r"], contour["nc"])
        return z, w, False
    if contour["kind"] == "explicit":
        return np.asarray(contour["z"]), np.asarray(contour["w"]), bool(contour.get("half", False))
    raise ValueError(f"unknown contour kind {contour['kind']!r}")


def rho_hat(lam, z, w, half: bool):
    """Rational filter rho_hat(lambda) = sum_k w_k / (z_k - lambda)  (Eq. rhoh).

    With ``half`` the sum runs over the upper-half nodes and the real part is
    doubled (real symmetric pencils).
    """
    lam = np.asarray(lam)
    s = np.zeros(lam.shape, dtype=complex)
    for zk, wk in zip(z, w):
        s = s + wk / (zk - lam)
    return 2.0 * s.real if half else s
