"""Full-size parity: the 64^3 Laplacian + potential solve (m0 80, 8 Gauss-Legendre nodes on the
upper half circle, k = 8) against the stored oracle spectrum of tests/golden.

The mixed path (inner solves by block GMRES on one real FP32 Krylov basis shared by the 8 shifts,
FP64 outer iteration) must find exactly the 54 eigenvalues inside the interval, each within 1e-10
relative of the oracle's, with residual <= 1e-9.  The solve takes well under a second on one
MI355X; the first import and the workspace allocation dominate the test's time.
"""

import os

import numpy as np
import pytest

import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lap3d_pot_64_lowest.txt")


@pytest.mark.timeout(900)
def test_c2_full_size_mixed_matches_oracle_spectrum():
    import torch
    import paper_1706_00692_amd as pk

    assert torch.cuda.is_available()
    gold = np.loadtxt(GOLDEN, comments="#")[:, 1]
    prob = W.config2(64)
    lo, hi = prob.contour["emin"], prob.contour["emax"]
    want = gold[(gold > lo) & (gold < hi)]
    print(f"[c2 full] n={prob.A.n} m0={prob.m0} expecting {len(want)} eigenvalues", flush=True)
    ctx = pk.Context(0)
    try:
        r = ctx.solve_problem(prob, precision=pk.PREC_MIXED)
    finally:
        ctx.close()
    print(f"[c2 full] status={r.status} m={r.m} outer={r.outer_iters} rf={r.max_resid:.2e}", flush=True)
    assert r.converged and r.m == len(want) == 54
    got = np.sort(r.lam_in)
    rel = np.abs(got - want) / np.abs(want)
    assert rel.max() <= 1e-10, rel.max()
    assert r.resid[: r.m].max() <= prob.tol
