"""The stored low spectrum of the 64^3 Laplacian + U[0, 2] potential (tests/golden).

The file was written by tests/golden/make_lap3d_spectrum.py, which calls only
the oracle.  It is pinned here to what mathematics fixes independently of the
oracle: Weyl's inequality brackets eigenvalue i of L + D between eigenvalue i
of L plus min(D) and plus max(D), and the 7-point Dirichlet Laplacian L has
the closed-form spectrum sum over axes of 2 - 2 cos(j pi / (N + 1)).
"""

import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lap3d_pot_64_lowest.txt")
N = 64


def _load():
    rows = np.loadtxt(GOLDEN, comments="#")
    return rows[:, 0].astype(int), rows[:, 1], rows[:, 2]


def _laplacian_low(k, with_modes=False):
    t = 2.0 - 2.0 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    # the k lowest sums t_a + t_b + t_c: the lowest sums use small indices only
    m = 20
    s = (t[:m, None, None] + t[None, :m, None] + t[None, None, :m]).ravel()
    order = np.argsort(s, kind="stable")[:k]
    if not with_modes:
        return s[order]
    return s[order], np.stack(np.unravel_index(order, (m, m, m)), axis=1)


def test_golden_is_ordered_and_converged():
    idx, lam, res = _load()
    assert np.array_equal(idx, np.arange(len(idx))) and len(idx) == 180
    assert np.all(np.diff(lam) >= 0)
    assert res.max() <= 1e-8


def test_golden_within_weyl_bounds():
    _, lam, _ = _load()
    pot = W.random_potential(N ** 3, 1002, 0.0, 2.0)
    low = _laplacian_low(len(lam))
    assert np.all(lam >= low + pot.min() - 1e-12)
    assert np.all(lam <= low + pot.max() + 1e-12)


def test_golden_ky_fan_sums():
    """Ky Fan: the sum of the k lowest eigenvalues of L + D is at most the Rayleigh quotients of any
    k orthonormal vectors; the k lowest Laplacian modes (products of sines) give the closed bound."""
    _, lam, _ = _load()
    pot = W.random_potential(N ** 3, 1002, 0.0, 2.0).reshape(N, N, N)  # index x + N y + N^2 z -> [z, y, x]
    low, modes = _laplacian_low(len(lam), with_modes=True)
    x = np.arange(1, N + 1)
    sines = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(np.arange(1, 21), x) * np.pi / (N + 1))  # mode a -> row a-1
    q = np.empty(len(lam))
    for i, (a, b, c) in enumerate(modes):
        # mode (a, b, c): a along x, b along y, c along z
        w = np.einsum("z,y,x->zyx", sines[c] ** 2, sines[b] ** 2, sines[a] ** 2)
        q[i] = np.sum(w * pot)
    for k in (1, 10, 62, 116, 180):
        assert lam[:k].sum() <= low[:k].sum() + q[:k].sum() + 1e-9, k


def test_c2_interval_holds_indices_62_to_115():
    _, lam, _ = _load()
    prob = W.config2(N)
    lo, hi = prob.contour["emin"], prob.contour["emax"]
    inside = np.nonzero((lam > lo) & (lam < hi))[0]
    assert inside[0] == 62 and inside[-1] == 115 and len(inside) == 54
    gap = np.mean(np.diff(lam[62:116]))
    # both ends sit well inside gaps of the spectrum
    assert min(lo - lam[61], lam[62] - lo, hi - lam[115], lam[116] - hi) > 0.5 * gap
