"""GPU parity: every step of the HIP path through the C ABI against the CPU oracle.

Tolerances: FP64 steps agree with the oracle to rounding amplified by the
conditioning of the small problems (rtol 1e-9 on the filtered block at
config-1 size); complex-FP32 inner solves to ~1e-5 relative (single
precision with a few hundred accumulated operations); converged eigenpairs
of both paths to the tolerance the method states (relative eigenvalue error
<= 1e-10, residual <= tol).
"""

import numpy as np
import pytest

import oracle as O
from oracle.quadrature import contour_nodes
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    import paper_1706_00692_amd as pk

    c = pk.Context(0)
    yield c
    c.close()


def _cplx(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _rand_block(n, w, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, w)) + 1j * rng.standard_normal((n, w))


# ------------------------------------------------------------------ SpMM
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["lap2d", "gen27_ragged"])
def test_spmm_shifted_parity(ctx, torch_cuda, prec, case):
    import paper_1706_00692_amd as pk

    torch = torch_cuda
    if case == "lap2d":
        A, B, m0, ns = W.laplacian_2d(20), None, 16, 8
    else:
        A, B, m0, ns = W.spd27(7, 11), W.mass27(7, 12), 16, 3  # n = 343: ragged row tiles
    z = np.array([0.3 + 0.2j, 1.1 + 0.05j, -0.4 + 1.5j, 0.7 + 0.01j, 2 + 3j, 0.65 + 0.15j, 0.1 + 0.9j, 5 + 0.5j])[:ns]
    V = _rand_block(A.n, ns * m0, 7)
    dt = torch.complex128 if prec == "fp64" else torch.complex64
    Vd = _cplx(torch, V, dt)
    Wd = torch.zeros_like(Vd)
    Am = ctx.matrix(A)
    Bm = None if B is None else ctx.matrix(B)
    ctx.spmm_shifted(Am, Bm, pk.PREC_FP64 if prec == "fp64" else pk.PREC_MIXED, z, m0, Vd, Wd)
    torch.cuda.synchronize()
    got = Wd.cpu().numpy()
    As = A.to_scipy()
    Bs = None if B is None else B.to_scipy()
    for s in range(ns):
        sl = slice(s * m0, (s + 1) * m0)
        want = O.shifted_operator(As, Bs, z[s])(V[:, sl])
        scale = np.abs(want).max()
        tol = 1e-14 if prec == "fp64" else 2e-6
        assert np.abs(got[:, sl] - want).max() <= tol * scale * 10, (s, np.abs(got[:, sl] - want).max() / scale)


@pytest.mark.parametrize("sched", range(15))
def test_spmm_every_schedule(torch_cuda, sched, monkeypatch):
    """Each autotuner candidate (forced through IFEAST_SPMM_SCHED on a fresh matrix) against the oracle,
    on widths that leave partial passes: 3 x 18 complex columns (FP32: 27 vectors, FP64: 54) and B present.
    Schedules 8 and up (whole rows per lane group) only take rows of 8 to 64 vectors, and the
    pipelined ones (12 and up) only B = I.  The last case has one shift at zero (W = -A V, the shared
    basis's product), where the row's own term is not read."""
    import paper_1706_00692_amd as pk

    torch = torch_cuda
    monkeypatch.setenv("IFEAST_SPMM_SCHED", str(sched))
    c = pk.Context(0)
    try:
        for prec, dt, tol in [(pk.PREC_MIXED, torch.complex64, 2e-5), (pk.PREC_FP64, torch.complex128, 1e-13)]:
            for A, B, m0, ns, zero in [(W.spd27(7, 31), W.mass27(7, 32), 18, 3, False),
                                       (W.laplacian_2d(19), None, 80, 5, False),
                                       (W.laplacian_3d(9, W.random_potential(729, 4)), None, 40, 1, False),
                                       (W.laplacian_3d(9, W.random_potential(729, 5)), None, 40, 1, True)]:
                nvec = ns * m0 // (2 if prec == pk.PREC_MIXED else 1)
                if sched >= 8 and not 8 <= nvec <= 64:
                    continue
                if sched >= 12 and B is not None:
                    continue
                z = np.array([0.3 + 0.2j, 1.1 + 0.05j, -0.4 + 1.5j, 0.7 + 0.01j, 2 + 3j])[:ns]
                if zero:
                    z = np.zeros(ns, dtype=complex)
                V = _rand_block(A.n, ns * m0, 17)
                Vd = _cplx(torch, V, dt)
                Wd = torch.zeros_like(Vd)
                Am = c.matrix(A)
                Bm = None if B is None else c.matrix(B)
                c.spmm_shifted(Am, Bm, prec, z, m0, Vd, Wd)
                torch.cuda.synchronize()
                got = Wd.cpu().numpy()
                for s in range(ns):
                    sl = slice(s * m0, (s + 1) * m0)
                    want = O.shifted_operator(A.to_scipy(), None if B is None else B.to_scipy(), z[s])(V[:, sl])
                    err = np.abs(got[:, sl] - want).max() / np.abs(want).max()
                    assert err <= tol, (sched, prec, A.n, s, err)
    finally:
        c.close()


def test_kernel_timing_accounting(torch_cuda):
    """Timed SpMM launches: count and algorithmic bytes per launch (CSR once, V read once, W written once)."""
    import paper_1706_00692_amd as pk

    torch = torch_cuda
    c = pk.Context(0)
    try:
        A, m0, ns = W.laplacian_2d(30), 32, 4
        Am = c.matrix(A)
        Vd = _cplx(torch, _rand_block(A.n, ns * m0, 3), torch.complex64)
        Wd = torch.empty_like(Vd)
        z = [0.5 + 0.1j] * ns
        c.spmm_shifted(Am, None, pk.PREC_MIXED, z, m0, Vd, Wd)  # autotune, untimed
        c.set_timing(True)
        for _ in range(3):
            c.spmm_shifted(Am, None, pk.PREC_MIXED, z, m0, Vd, Wd)
        st = c.kernel_stats()
        c.set_timing(False)
        assert st["spmm"]["launches"] == 3 and st["spmm"]["seconds"] > 0
        want = (A.n + 1) * 4 + A.nnz * 8 + 2 * A.n * ns * m0 * 8
        assert st["spmm"]["bytes"] == pytest.approx(3 * want, rel=1e-12)
        assert st["gram"]["launches"] == 0
    finally:
        c.close()


def test_spmm_full_size_sampled(ctx, torch_cuda):
    """64^3 Laplacian + potential, 8 shifts x 80 columns, complex FP32: sampled rows against the oracle."""
    import paper_1706_00692_amd as pk

    torch = torch_cuda
    N, m0, ns = 64, 80, 8
    A = W.laplacian_3d(N, W.random_potential(N ** 3, 1002))
    z = 1.0 + np.exp(1j * np.linspace(0.1, 3.0, ns))
    g = torch.Generator(device="cuda").manual_seed(5)
    Vd = torch.randn((A.n, ns * m0), dtype=torch.complex64, device="cuda", generator=g)
    Wd = torch.empty_like(Vd)
    Am = ctx.matrix(A)
    ctx.spmm_shifted(Am, None, pk.PREC_MIXED, z, m0, Vd, Wd)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([np.random.default_rng(3).integers(0, A.n, 200), [0, A.n - 1, 4095, 4096]]))
    need = np.unique(np.concatenate([A.colind[A.rowptr[r]:A.rowptr[r + 1]] for r in rows] + [rows]))
    Vn = Vd[torch.from_numpy(need).cuda()].cpu().numpy().astype(np.complex128)
    pos = {int(c): i for i, c in enumerate(need)}
    Wn = Wd[torch.from_numpy(rows).cuda()].cpu().numpy()
    for t, r in enumerate(rows):
        acc = np.zeros(ns * m0, dtype=complex)
        for e in range(A.rowptr[r], A.rowptr[r + 1]):
            acc += np.float32(A.val[e]) * Vn[pos[int(A.colind[e])]]
        zr = np.repeat(z.astype(np.complex64).astype(np.complex128), m0)
        want = zr * Vn[pos[int(r)]] - acc
        assert np.abs(Wn[t] - want).max() <= 1e-5 * max(1.0, np.abs(want).max())


# ------------------------------------------------------------- filter step
def _first_iterate(prob):
    lam, X, AX, BX, _ = O.rayleigh_ritz(prob.A.to_scipy(), None if prob.B is None else prob.B.to_scipy(), prob.x0())
    R, r = O.residuals(AX, BX, lam)
    return lam, X, R, r


def _oracle_filter(prob, lam, X, R, k, cycles, restarted=True):
    """restarted=False: one block GMRES cycle of k * cycles iterations per shift (what the shared
    basis computes; in exact arithmetic the shifted block Krylov spaces coincide)."""
    A = prob.A.to_scipy()
    B = None if prob.B is None else prob.B.to_scipy()
    z, w, half = contour_nodes(prob.contour)
    D = []
    for zk in z:
        rhs = R / (zk - lam)[None, :]
        if cycles == 1 or not restarted:
            Dk, _ = O.block_gmres(O.shifted_operator(A, B, zk), rhs, k * cycles, 0.0)
        else:
            from oracle.krylov import block_gmres_restarted

            Dk, _ = block_gmres_restarted(O.shifted_operator(A, B, zk), rhs, k, 0.0, cycles)
        D.append(Dk)
    return O.quad_accumulate(X, lam, D, z, w, half)


def _gpu_filter(ctx, torch, prob, lam, X, R, prec, k, cycles, reorth_eta=0.0, basis=None):
    import paper_1706_00692_amd as pk

    Am = ctx.matrix(prob.A)
    Bm = None if prob.B is None else ctx.matrix(prob.B)
    p = pk.params_struct(prob.m0, max_outer=1, max_inner=k, max_cycles=cycles, alpha=0.0, tol=1e-9,
                         precision=prec, reorth_eta=reorth_eta,
                         basis=pk.BASIS_AUTO if basis is None else basis)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    ld = torch.from_numpy(np.ascontiguousarray(lam)).cuda()
    Rd = torch.from_numpy(np.ascontiguousarray(R)).cuda()
    Qd = torch.zeros_like(Xd)
    iters = ctx.filter(Am, Bm, prob.contour, p, Xd, ld, Rd, 1.0, Qd)
    torch.cuda.synchronize()
    return Qd.cpu().numpy(), iters


@pytest.mark.parametrize("basis", ["per_shift", "shared"])
@pytest.mark.parametrize("cycles,reorth", [(1, 0.0), (3, 0.0), (1, 2.0), (3, 2.0)])
def test_filter_parity_fp64(ctx, torch_cuda, cycles, reorth, basis):
    """reorth 0: the default selective second Gram-Schmidt pass; 2.0: always two passes.
    per_shift: restarted complex block GMRES(k) per shift; shared: one real Arnoldi of A for all
    shifts, k * cycles steps without restarts (the oracle runs that many steps per shift)."""
    import paper_1706_00692_amd as pk

    prob = W.config1()
    lam, X, R, r = _first_iterate(prob)
    shared = basis == "shared"
    want = _oracle_filter(prob, lam, X, R, prob.max_inner, cycles, restarted=not shared)
    got, iters = _gpu_filter(ctx, torch_cuda, prob, lam, X, R, pk.PREC_FP64, prob.max_inner, cycles, reorth,
                             pk.BASIS_SHARED if shared else pk.BASIS_PER_SHIFT)
    assert list(iters) == [prob.max_inner * cycles] * 8
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 1e-9, err


@pytest.mark.parametrize("m0", [48, 80, 96, 128])
def test_filter_parity_shared_wide(ctx, torch_cuda, m0):
    """Shared basis with several 16-column panels in the block Cholesky-QR factor (m0 = 48 ... 128;
    above 96 the previous R factor sits in global memory): 4 Arnoldi steps on a 10^3 Laplacian +
    potential, FP64, against per-shift block GMRES."""
    import paper_1706_00692_amd as pk

    N = 10
    lam_all = np.linalg.eigvalsh(W.laplacian_3d(N, W.random_potential(N ** 3, 1002)).to_dense())
    prob = W.config2_small(N=N, m0=m0, emin=0.5 * (lam_all[5] + lam_all[6]), emax=0.5 * (lam_all[20] + lam_all[21]))
    lam, X, R, r = _first_iterate(prob)
    want = _oracle_filter(prob, lam, X, R, 2, 2, restarted=False)
    got, iters = _gpu_filter(ctx, torch_cuda, prob, lam, X, R, pk.PREC_FP64, 2, 2, 0.0, pk.BASIS_SHARED)
    assert list(iters) == [4] * 8
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 1e-9, err


@pytest.mark.parametrize("m0", [64, 80])
def test_filter_parity_shared_mixed(ctx, torch_cuda, m0):
    """Mixed precision on the shared basis at the benchmark's block widths (m0 = 64, 80): 8 Arnoldi
    steps on a 10^3 Laplacian + potential, so steps 2..7 take the Lanczos path (sketched estimate,
    local second pass folded into the normalisation, one-pass Cholesky-QR when certified), against
    per-shift block GMRES in FP64; the FP32 part is the correction Q - X rho_hat(Lambda)."""
    import paper_1706_00692_amd as pk
    from oracle.quadrature import rho_hat

    N = 10
    lam_all = np.linalg.eigvalsh(W.laplacian_3d(N, W.random_potential(N ** 3, 1002)).to_dense())
    prob = W.config2_small(N=N, m0=m0, emin=0.5 * (lam_all[5] + lam_all[6]), emax=0.5 * (lam_all[20] + lam_all[21]))
    lam, X, R, r = _first_iterate(prob)
    want = _oracle_filter(prob, lam, X, R, 4, 2, restarted=False)
    got, iters = _gpu_filter(ctx, torch_cuda, prob, lam, X, R, pk.PREC_MIXED, 4, 2, 0.0, pk.BASIS_SHARED)
    assert list(iters) == [8] * 8
    z, w, half = contour_nodes(prob.contour)
    base = X * rho_hat(lam, z, w, half)[None, :]
    err = np.abs(got - want).max() / np.abs(want - base).max()
    assert err <= 1e-4, err


def test_solve_shared_m0_128_mixed(ctx):
    """A full mixed-precision solve with m0 = 128 on the shared basis (the widest block the
    serving mix draws), against the dense spectrum of a 12^3 Laplacian + potential."""
    import paper_1706_00692_amd as pk

    N = 12
    lam_all = np.linalg.eigvalsh(W.laplacian_3d(N, W.random_potential(N ** 3, 1002)).to_dense())
    prob = W.config2_small(N=N, m0=128, emin=0.5 * (lam_all[9] + lam_all[10]), emax=0.5 * (lam_all[69] + lam_all[70]))
    res = ctx.solve_problem(prob, precision=pk.PREC_MIXED)
    assert res.status == 0 and res.converged and res.m == 60
    assert np.allclose(np.sort(res.lam_in), lam_all[10:70], rtol=1e-10, atol=0)
    assert res.resid[: res.m].max() <= prob.tol


def test_solve_shared_mixed_repeats_bitwise(ctx):
    """Three mixed solves on the shared basis in a row agree to the last bit.  The FP32 basis
    copies each step's decision words to the host, and forms the next step's sketch update, on a
    third stream ordered by events alone (a missing order would show as a change between runs);
    the pairs match the dense spectrum of a 14^3 Laplacian + potential."""
    import paper_1706_00692_amd as pk

    N = 14
    lam_all = np.linalg.eigvalsh(W.laplacian_3d(N, W.random_potential(N ** 3, 1002)).to_dense())
    prob = W.config2_small(N=N, m0=48, emin=0.5 * (lam_all[9] + lam_all[10]), emax=0.5 * (lam_all[39] + lam_all[40]))
    runs = [ctx.solve_problem(prob, precision=pk.PREC_MIXED) for _ in range(3)]
    r0 = runs[0]
    assert r0.status == 0 and r0.converged and r0.m == 30
    assert np.allclose(np.sort(r0.lam_in), lam_all[10:40], rtol=1e-10, atol=0)
    assert r0.resid[: r0.m].max() <= prob.tol
    for r in runs[1:]:
        assert (r.m, r.outer_iters, r.seq_matvec) == (r0.m, r0.outer_iters, r0.seq_matvec)
        assert np.array_equal(r.lam, r0.lam) and np.array_equal(r.resid, r0.resid)
        assert np.array_equal(r.X, r0.X)


def test_filter_parity_mixed(ctx, torch_cuda):
    import paper_1706_00692_amd as pk

    prob = W.config1()
    lam, X, R, r = _first_iterate(prob)
    want = _oracle_filter(prob, lam, X, R, prob.max_inner, 1)
    got, _ = _gpu_filter(ctx, torch_cuda, prob, lam, X, R, pk.PREC_MIXED, prob.max_inner, 1)
    # the FP32 part is the correction Q - X rho_hat(Lambda)
    from oracle.quadrature import rho_hat

    z, w, half = contour_nodes(prob.contour)
    base = X * rho_hat(lam, z, w, half)[None, :]
    err = np.abs(got - want).max() / np.abs(want - base).max()
    assert err <= 1e-4, err


def test_filter_parity_generalized_ragged(ctx, torch_cuda):
    import paper_1706_00692_amd as pk

    prob = W.config3_small(N=7, m0=16, emin=0.0, emax=1.0)
    lam_all = np.sort(np.real(O.dense_reference(prob.A, prob.B, {"kind": "half", "emin": -1, "emax": 1e9})[2]))
    prob.contour = dict(prob.contour, emin=0.5 * (lam_all[1] + lam_all[2]), emax=0.5 * (lam_all[8] + lam_all[9]))
    lam, X, R, r = _first_iterate(prob)
    want = _oracle_filter(prob, lam, X, R, 3, 1)
    got, _ = _gpu_filter(ctx, torch_cuda, prob, lam, X, R, pk.PREC_FP64, 3, 1)
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 1e-9, err


# --------------------------------------------------------- Rayleigh-Ritz
@pytest.mark.parametrize("gen", [False, True])
def test_rayleigh_ritz_parity(ctx, torch_cuda, gen):
    torch = torch_cuda
    if gen:
        A, B = W.spd27(6, 21), W.mass27(6, 22)
    else:
        A, B = W.laplacian_3d(9, W.random_potential(729, 5)), None  # n = 729, ragged
    m0 = 32
    rng = np.random.default_rng(9)
    Q = rng.standard_normal((A.n, m0))
    lam, X, AX, BX, C = O.rayleigh_ritz(A.to_scipy(), None if B is None else B.to_scipy(), Q)
    R, r = O.residuals(AX, BX, lam)
    Am = ctx.matrix(A)
    Bm = None if B is None else ctx.matrix(B)
    Qd = torch.from_numpy(Q).cuda()
    out = {k: torch.zeros(v, dtype=torch.float64, device="cuda") for k, v in
           dict(lam=m0, X=(A.n, m0), R=(A.n, m0), resid=m0, eta=m0).items()}
    ctx.rayleigh_ritz(Am, Bm, Qd, out["lam"], out["X"], out["R"], out["resid"], out["eta"])
    torch.cuda.synchronize()
    gl, gX, gr = out["lam"].cpu().numpy(), out["X"].cpu().numpy(), out["resid"].cpu().numpy()
    assert np.allclose(gl, lam, rtol=1e-11, atol=1e-12 * np.abs(lam).max())
    # eigenvectors up to sign (the Ritz values of random Q are simple)
    sgn = np.sign(np.sum(gX * X, axis=0))
    assert np.abs(gX * sgn[None, :] - X).max() <= 1e-8 * np.abs(X).max()
    assert np.allclose(gr, r, rtol=1e-8, atol=1e-12)
    eta = 1.0 / np.linalg.norm(C, axis=0)
    assert np.allclose(out["eta"].cpu().numpy(), eta, rtol=1e-8)


# ------------------------------------------------------------ full solves
def _check_against_oracle(prob, res, ref, rel=1e-10):
    assert res.converged and ref.converged
    assert res.m == ref.m
    got, want = np.sort(res.lam_in), np.sort(ref.lam_in)
    assert np.all(np.abs(got - want) <= rel * np.abs(want)), np.abs(got - want) / np.abs(want)
    assert res.resid[: res.m].max() <= prob.tol
    # invariant subspace of the eigenvalues inside: compare as subspaces (clusters are degenerate)
    Xg, Xr = res.X_in, ref.X_in
    Bs = None if prob.B is None else prob.B.to_scipy()
    proj = Xg @ (Xg.T @ (Xr if Bs is None else Bs @ Xr))  # B-orthogonal projection onto span(Xg)
    sines = np.linalg.norm(Xr - proj, axis=0)
    assert sines.max() <= 1e-7, sines.max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_config1(ctx, prec):
    import paper_1706_00692_amd as pk

    prob = W.config1()
    res = ctx.solve_problem(prob, precision=pk.PREC_FP64 if prec == "fp64" else pk.PREC_MIXED)
    ref = O.ifeast(prob.A, None, prob.contour, prob.m0, prob.max_inner, prob.alpha, prob.tol, prob.x0(),
                   prob.max_outer, max_cycles=prob.max_cycles, inner_rule=prob.inner_rule, tau=prob.tau)
    _check_against_oracle(prob, res, ref)
    mu = 2 - 2 * np.cos(np.arange(1, 21) * np.pi / 21)
    exact = np.sort((mu[:, None] + mu[None, :]).ravel())
    exact = exact[(exact > 0.5) & (exact < 0.8)]
    assert np.allclose(np.sort(res.lam_in), exact, rtol=1e-10, atol=0)
    assert res.status == 0


def test_solve_ragged_3d_with_potential(ctx):
    import paper_1706_00692_amd as pk

    N = 9
    lam_all = np.linalg.eigvalsh(W.laplacian_3d(N, W.random_potential(N ** 3, 1002)).to_dense())
    emin, emax = 0.5 * (lam_all[3] + lam_all[4]), 0.5 * (lam_all[15] + lam_all[16])
    prob = W.config2_small(N=N, m0=32, emin=emin, emax=emax)
    res = ctx.solve_problem(prob, precision=pk.PREC_MIXED)
    ref = O.ifeast(prob.A, None, prob.contour, prob.m0, prob.max_inner, prob.alpha, prob.tol, prob.x0(),
                   prob.max_outer, max_cycles=prob.max_cycles, inner_rule=prob.inner_rule, tau=prob.tau)
    _check_against_oracle(prob, res, ref)
    assert np.allclose(np.sort(res.lam_in), lam_all[4:16], rtol=1e-10, atol=0)


def test_solve_generalized_small(ctx):
    import paper_1706_00692_amd as pk

    prob = W.config3_small(N=6, m0=16)
    lam_all = np.sort(np.real(O.dense_reference(prob.A, prob.B, {"kind": "half", "emin": -1, "emax": 1e9})[2]))
    prob.contour = dict(prob.contour, emin=0.5 * (lam_all[1] + lam_all[2]), emax=0.5 * (lam_all[8] + lam_all[9]))
    res = ctx.solve_problem(prob, precision=pk.PREC_FP64)
    assert res.converged and res.m == 7
    assert np.allclose(np.sort(res.lam_in), lam_all[2:9], rtol=1e-10, atol=0)
    B = prob.B.to_scipy()
    assert np.allclose(res.X_in.T @ (B @ res.X_in), np.eye(7), atol=1e-9)


# ------------------------------------------------------- status and errors
def test_not_converged_and_m0_too_small(ctx):
    import paper_1706_00692_amd as pk

    prob = W.config1()
    res = ctx.solve_problem(prob, precision=pk.PREC_FP64, max_outer=1)
    assert res.status == 1 and not res.converged and res.outer_iters == 1
    prob.contour = dict(prob.contour, emin=0.5, emax=1.2)  # 26 eigenvalues, m0 = 16
    for prec in (pk.PREC_FP64, pk.PREC_MIXED):
        res = ctx.solve_problem(prob, precision=prec, max_outer=10)
        # every Ritz value lands inside after the first filter application: the solve stops there
        assert res.status == 2 and res.outer_iters == 1 and not res.converged
        assert np.all((res.lam > 0.5) & (res.lam < 1.2))
    ref = O.ifeast(prob.A, None, prob.contour, prob.m0, prob.max_inner, prob.alpha, prob.tol, prob.x0(), 10,
                   max_cycles=prob.max_cycles, inner_rule=prob.inner_rule, tau=prob.tau)
    assert ref.status == "m0_too_small" and ref.outer_iters == 1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_no_eigenvalue_in_contour(ctx, prec):
    """An interval inside a spectral gap of the 20 x 20 Laplacian: status NO_EIG, as the oracle.
    The shared basis's inner solves are longer than the oracle's restarted ones, so Ritz values
    of damped directions may sit inside the gap for a few outer iterations before the rule fires."""
    import paper_1706_00692_amd as pk

    mu = 2 - 2 * np.cos(np.arange(1, 21) * np.pi / 21)
    exact = np.sort((mu[:, None] + mu[None, :]).ravel())
    gap = int(np.argmax(np.diff(exact[:60])))
    lo, hi = exact[gap], exact[gap + 1]
    prob = W.config1()
    prob.contour = dict(prob.contour, emin=lo + 0.1 * (hi - lo), emax=hi - 0.1 * (hi - lo))
    res = ctx.solve_problem(prob, precision=pk.PREC_FP64 if prec == "fp64" else pk.PREC_MIXED)
    assert res.status == 3 and res.m == 0 and res.outer_iters <= 8
    assert not np.any((res.lam > prob.contour["emin"]) & (res.lam < prob.contour["emax"]))
    ref = O.ifeast(prob.A, None, prob.contour, prob.m0, prob.max_inner, prob.alpha, prob.tol, prob.x0(),
                   prob.max_outer, max_cycles=prob.max_cycles, inner_rule=prob.inner_rule, tau=prob.tau)
    assert ref.status == "no_eig" and ref.outer_iters == 1


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_inner_global_rule_matches_oracle(ctx, prec):
    """Algorithm 2's printed inner stopping rule (every column residual <= alpha ||R_F||) end to end."""
    import paper_1706_00692_amd as pk

    prob = W.config1()
    prob.inner_rule = "global"
    res = ctx.solve_problem(prob, precision=pk.PREC_FP64 if prec == "fp64" else pk.PREC_MIXED)
    ref = O.ifeast(prob.A, None, prob.contour, prob.m0, prob.max_inner, prob.alpha, prob.tol, prob.x0(),
                   prob.max_outer, max_cycles=prob.max_cycles, inner_rule="global", tau=prob.tau)
    _check_against_oracle(prob, res, ref)
    assert res.status == 0


def test_invalid_inputs_rejected(ctx):
    import paper_1706_00692_amd as pk

    A = W.laplacian_2d(6)
    bad = W.CSR(A.n, A.rowptr.copy(), A.colind.copy(), A.val.copy())
    bad.colind[[0, 1]] = bad.colind[[1, 0]]  # unsorted row
    with pytest.raises(pk.IFeastError) as e:
        ctx.matrix(bad)
    assert e.value.status == -1
    nan = W.CSR(A.n, A.rowptr.copy(), A.colind.copy(), A.val.copy())
    nan.val[3] = np.nan
    with pytest.raises(pk.IFeastError):
        ctx.matrix(nan)
    oob = W.CSR(A.n, A.rowptr.copy(), A.colind.copy(), A.val.copy())
    oob.colind[-1] = A.n
    with pytest.raises(pk.IFeastError):
        ctx.matrix(oob)
    prob = W.config1()
    with pytest.raises(pk.IFeastError) as e:
        ctx.solve_problem(prob, m0=24)
    assert e.value.status == -1
    with pytest.raises(pk.IFeastError) as e:
        ctx.solve_problem(prob, problem=1)
    assert e.value.status == -7


# ------------------------------------------------------------- serving
def test_serving_alone_vs_mix(ctx):
    import paper_1706_00692_amd as pk

    probs = [W.config1()]
    for N, lo, hi, m0 in [(9, 4, 16, 32), (8, 2, 10, 16)]:
        lam_all = np.linalg.eigvalsh(W.laplacian_3d(N, W.random_potential(N ** 3, 1002)).to_dense())
        probs.append(W.config2_small(N=N, m0=m0, emin=0.5 * (lam_all[lo - 1] + lam_all[lo]),
                                     emax=0.5 * (lam_all[hi - 1] + lam_all[hi])))
    alone = [ctx.solve_problem(p, precision=pk.PREC_MIXED) for p in probs]
    tickets = []
    for p in probs:
        params = pk.params_struct(p.m0, p.max_outer, p.max_inner, p.max_cycles, p.alpha, p.tol, p.tau,
                                  pk.PREC_MIXED)
        tickets.append(ctx.submit(p.A, p.B, p.contour, params, p.x0()))
    for p, t, a in zip(probs, tickets, alone):
        r = ctx.wait(t, p.n, p.m0, p.max_outer, p.contour["nc"])
        assert r.converged and r.m == a.m
        assert np.all(np.abs(r.lam_in - a.lam_in) <= 1e-10 * np.abs(a.lam_in))
        assert r.resid[: r.m].max() <= p.tol
        assert r.latency > 0
    with pytest.raises(pk.IFeastError) as e:
        ctx.poll(987654321)
    assert e.value.status == -6


def _small_serving_problems():
    probs = [W.config1()]
    for N, lo, hi, m0 in [(9, 4, 16, 32), (8, 2, 10, 16)]:
        lam_all = np.linalg.eigvalsh(W.laplacian_3d(N, W.random_potential(N ** 3, 1002)).to_dense())
        probs.append(W.config2_small(N=N, m0=m0, emin=0.5 * (lam_all[lo - 1] + lam_all[lo]),
                                     emax=0.5 * (lam_all[hi - 1] + lam_all[hi])))
    return probs


def _serving_params(pk, p):
    return pk.params_struct(p.m0, p.max_outer, p.max_inner, p.max_cycles, p.alpha, p.tol, p.tau, pk.PREC_MIXED)


def test_serving_budget_rejects_and_queues(torch_cuda):
    """A request larger than the context budget is REJECTED at submit; with a budget that fits
    only the largest request, requests run one at a time (each waits for the previous one) and
    still give the results they give alone."""
    import paper_1706_00692_amd as pk

    small = _small_serving_problems()
    probs = [small[1], small[1], small[1]]  # three requests of one footprint
    fp = pk.footprint(probs[0].n, probs[0].A.nnz, 0, probs[0].contour, _serving_params(pk, probs[0]))
    c = pk.Context(0, budget=fp)
    try:
        alone = [c.solve_problem(p, precision=pk.PREC_MIXED) for p in probs]
        tight = pk.Context(0, budget=fp - 1)
        try:
            with pytest.raises(pk.IFeastError) as e:
                tight.submit(probs[0].A, None, probs[0].contour, _serving_params(pk, probs[0]), probs[0].x0())
            assert e.value.status == -5
        finally:
            tight.close()
        # two requests exceed the budget, so none runs beside another
        tickets = [c.submit(p.A, None, p.contour, _serving_params(pk, p), p.x0()) for p in probs]
        out = [c.wait(t, p.n, p.m0, p.max_outer, p.contour["nc"]) for p, t in zip(probs, tickets)]
        for p, r, a in zip(probs, out, alone):
            assert r.converged and r.m == a.m
            assert np.all(np.abs(r.lam_in - a.lam_in) <= 1e-10 * np.abs(a.lam_in))
        # FIFO and one at a time: each latency covers the solves queued before it
        lat = [r.latency for r in out]
        assert lat[0] < lat[1] < lat[2]
        assert lat[2] >= sum(r.solve_seconds for r in out) * 0.9
    finally:
        c.close()


def test_serving_destroy_fails_queued_requests(torch_cuda):
    """Destroying a context with requests still queued: they fail with ERR_DEVICE, a thread
    blocked in wait() on one of them returns, and nothing hangs."""
    import threading

    import paper_1706_00692_amd as pk

    import time

    N = 20
    lam_all = np.linalg.eigvalsh(W.laplacian_3d(N, W.random_potential(N ** 3, 1002)).to_dense())
    p = W.config2_small(N=N, m0=32, emin=0.5 * (lam_all[3] + lam_all[4]), emax=0.5 * (lam_all[15] + lam_all[16]))
    fp = pk.footprint(p.n, p.A.nnz, 0, p.contour, _serving_params(pk, p))
    c = pk.Context(0, budget=fp)  # one request at a time: the later ones queue
    tickets = [c.submit(p.A, None, p.contour, _serving_params(pk, p), p.x0()) for _ in range(8)]
    got = {}

    import ctypes

    h, lib = c.h, c.lib

    def waiter():
        # the raw call: after a destroy the context handle must not be touched again
        bufs = pk._binding._ResultBuffers(p.n, p.m0, p.max_outer, p.contour["nc"])
        lat = ctypes.c_double(0.0)
        st = lib.ifeast_wait(h, ctypes.c_uint64(tickets[-1]), ctypes.byref(bufs.s), ctypes.byref(lat))
        if st < 0:
            got["err"] = st
        else:
            got["res"] = bufs.result(st, p.contour["nc"])

    th = threading.Thread(target=waiter)
    th.start()
    time.sleep(0.2)  # the waiter is blocked in wait() by now (the context must outlive its entry)
    c.close()
    th.join(timeout=120)
    assert not th.is_alive()
    # the last request either ran before the destroy reached it or failed as queued
    assert got.get("err") == -3 or got["res"].converged


def test_solve_dev_matches_host_buffers(ctx, torch_cuda):
    """ifeast_solve_dev (initial block and eigenvectors in HBM) computes what the host-buffer
    entry point computes: same pairs, same histories, eigenvectors equal to the last bit."""
    import paper_1706_00692_amd as pk

    torch = torch_cuda
    prob = W.config1()
    Am = ctx.matrix(prob.A)
    params = pk.problem_params(prob, pk.PREC_MIXED)
    X0 = prob.x0()
    ctx.solve_resident(Am, None, prob.contour, params, X0)  # first call of the shape: SpMM autotune
    rh = ctx.solve_resident(Am, None, prob.contour, params, X0)
    X0d = torch.from_numpy(X0).cuda()
    Xd = torch.zeros_like(X0d)
    rd = ctx.solve_dev(Am, None, prob.contour, params, X0d.data_ptr(), Xd.data_ptr())
    torch.cuda.synchronize()
    assert rd.converged and rh.converged
    assert (rd.m, rd.outer_iters, rd.seq_matvec) == (rh.m, rh.outer_iters, rh.seq_matvec)
    assert np.array_equal(rd.lam, rh.lam) and np.array_equal(rd.resid, rh.resid)
    assert np.array_equal(rd.flags, rh.flags)
    assert rd.X is None
    assert np.array_equal(Xd.cpu().numpy(), rh.X)
    # the input block is left as it was
    assert np.array_equal(X0d.cpu().numpy(), X0)
    Am.close()


# ------------------------------------------------------------- non-Hermitian
def _convdiff_exact(N, bx=20.0, by=10.0):
    """Closed-form spectrum of the h^2-scaled upwind convection-diffusion operator (real)."""
    h = 1.0 / (N + 1)
    j = np.arange(1, N + 1)

    def mu(b):
        return 2 + h * b - 2 * np.sqrt(1 + h * b) * np.cos(j * np.pi / (N + 1))

    return np.sort((mu(bx)[:, None] + mu(by)[None, :]).ravel())


def _pairs_to_complex(X, lam_im):
    """Complex eigenvectors from a pair-format block (a pair's columns: Re x, Im x of a + ib)."""
    Z = X.astype(np.complex128).copy()
    for j in range(X.shape[1]):
        if lam_im[j] < 0:
            Z[:, j] = X[:, j] - 1j * X[:, j + 1]
        elif lam_im[j] > 0:
            Z[:, j] = X[:, j - 1] + 1j * X[:, j]
    return Z


@pytest.mark.parametrize("m0", [32, 64])
def test_rayleigh_ritz_general_parity(ctx, torch_cuda, m0):
    """The device non-Hermitian Rayleigh-Ritz (SVQB, Hessenberg, Francis double-shift QR,
    quasi-triangular back substitution) on a random block of a 24^2 convection-diffusion
    operator: Ritz values against numpy's eig of the projected matrix, complex residuals and
    gains against the oracle's right-Galerkin Rayleigh-Ritz."""
    from oracle.feast import filter_gain

    torch = torch_cuda
    A = W.convdiff_2d(24, 20.0, 10.0)
    As = A.to_scipy()
    n = A.n
    rng = np.random.default_rng(31 + m0)
    Q = rng.standard_normal((n, m0))
    Xp = rng.standard_normal((n, m0))
    lam_o, X_o, AX_o, BX_o, C_o = O.rayleigh_ritz(As, None, Q, kind="general")
    R_o, r_o = O.residuals(AX_o, BX_o, lam_o)
    eta_o = filter_gain(C_o, Xp.T @ Xp)
    assert np.abs(lam_o.imag).max() > 1e-3  # the random block has complex Ritz pairs
    Am = ctx.matrix(A)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = {k: torch.zeros(v, dtype=torch.float64, device="cuda") for k, v in
           dict(lam=m0, lam_im=m0, X=(n, m0), R=(n, m0), resid=m0, eta=m0).items()}
    ctx.rayleigh_ritz_general(Am, dev(Q), dev(Xp), out["lam"], out["lam_im"], out["X"], out["R"], out["resid"],
                              out["eta"])
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    lam = g["lam"] + 1j * g["lam_im"]
    scale = np.abs(lam_o).max()
    # the oracle's complex eigensolver leaves a conjugate pair's real parts a rounding apart, so
    # its order within a pair is arbitrary: match each Ritz value to the nearest of the oracle's
    match = np.array([int(np.argmin(np.abs(lam_o - l))) for l in lam])
    assert len(set(match.tolist())) == m0
    lam_o, X_o, r_o = lam_o[match], X_o[:, match], r_o[match]
    eta_o = eta_o[match]
    assert np.abs(lam - lam_o).max() <= 1e-10 * scale, np.abs(lam - lam_o).max()
    assert np.all(np.diff(g["lam"]) >= 0)  # ascending real part
    # pair format: conjugate pairs adjacent, (-b, +b)
    for j in range(m0):
        if g["lam_im"][j] < 0:
            assert g["lam_im"][j + 1] == -g["lam_im"][j] and g["lam"][j + 1] == g["lam"][j]
    Xc = _pairs_to_complex(g["X"], g["lam_im"])
    assert np.allclose(np.linalg.norm(Xc, axis=0), 1.0, atol=1e-10)
    Rc = As @ Xc - Xc * lam[None, :]
    assert np.allclose(np.linalg.norm(Rc, axis=0), g["resid"], rtol=1e-7, atol=1e-12)
    assert np.allclose(g["resid"], r_o, rtol=1e-6, atol=1e-11)
    # the pair-format residual block is [Re, Im] of the complex residual of a + ib
    Rg = _pairs_to_complex(g["R"], g["lam_im"])
    assert np.abs(Rg - Rc).max() <= 1e-9 * np.abs(Rc).max()
    # same eigenvectors as the oracle up to phase (simple Ritz values)
    ph = np.sum(Xc.conj() * X_o, axis=0)
    assert np.allclose(np.abs(ph), 1.0, atol=1e-7)
    assert np.allclose(g["eta"], eta_o, rtol=1e-7)


def _general_problem(N, lo_i, hi_i, m0):
    ex = _convdiff_exact(N)
    lo, hi = 0.5 * (ex[lo_i - 1] + ex[lo_i]), 0.5 * (ex[hi_i - 1] + ex[hi_i])
    prob = W.config4_small(N=N, m0=m0, c=0.5 * (lo + hi), r=0.5 * (hi - lo))
    return prob, ex[lo_i:hi_i]


def _kappa_tol(A, lam_got, resid):
    """R13's eigenvalue bound for a nonnormal operator: |dlambda| <= max(1e-10 |lambda|,
    2 kappa r + 10 kappa u ||A||_1), kappa from dense left and right eigenvectors."""
    import scipy.linalg as sla

    Ad = A.to_dense()
    w, vl, vr = sla.eig(Ad, left=True, right=True)
    kap = np.linalg.norm(vl, axis=0) * np.linalg.norm(vr, axis=0) / np.abs(np.sum(vl.conj() * vr, axis=0))
    a1 = np.abs(Ad).sum(axis=0).max()
    tol = []
    for l, r in zip(lam_got, resid):
        k = kap[np.argmin(np.abs(w - l))]
        tol.append(max(1e-10 * abs(l), 2 * k * r + 10 * k * 2.220446049250313e-16 * a1))
    return np.array(tol), kap


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("N,lo_i,hi_i,m0", [(16, 3, 10, 16), (32, 20, 32, 32)])
def test_solve_general_closed_form(ctx, prec, N, lo_i, hi_i, m0):
    """Non-Hermitian solve (16 trapezoidal nodes on a circle around part of the convection-
    diffusion spectrum) against the closed-form eigenvalues with R13's conditioning-scaled
    tolerance, the eigenvectors against dense eig, and (16^2) the oracle's IFEAST run."""
    import paper_1706_00692_amd as pk

    prob, want = _general_problem(N, lo_i, hi_i, m0)
    res = ctx.solve_problem(prob, precision=pk.PREC_FP64 if prec == "fp64" else pk.PREC_MIXED)
    print(f"[general {N}^2 {prec}] status={res.status} m={res.m} outer={res.outer_iters} rf={res.max_resid:.2e} "
          f"inner={res.inner_hist.max(axis=1).tolist()}", flush=True)
    assert res.status == 0 and res.converged and res.m == len(want)
    got = res.lam_in
    order = np.argsort(got.real)
    got, resid, Xin = got[order], res.resid[: res.m][order], res.X_in[:, order]
    assert resid.max() <= prob.tol
    tol, kap = _kappa_tol(prob.A, got, resid)
    assert np.all(np.abs(got - want) <= tol), (np.abs(got - want), tol)
    # eigenvectors: unit norm, residual recomputed on the host, direction of the dense eigenvector
    As = prob.A.to_scipy()
    assert np.allclose(np.linalg.norm(Xin, axis=0), 1.0, atol=1e-10)
    r_host = np.linalg.norm(As @ Xin - Xin * got[None, :], axis=0)
    assert r_host.max() <= 2 * prob.tol
    ref_in, V_in, _ = O.dense_reference(prob.A, None, prob.contour, kind="general")
    V_in = V_in[:, np.argsort(ref_in.real)]
    cosv = np.abs(np.sum(Xin.conj() * V_in, axis=0)) / np.linalg.norm(V_in, axis=0)
    assert np.all(cosv >= 1 - 1e-6), cosv
    if N == 16:
        ref = O.ifeast(prob.A, None, prob.contour, prob.m0, prob.max_inner * prob.max_cycles, prob.alpha, prob.tol,
                       prob.x0(), 10, kind="general", max_cycles=1, inner_rule=prob.inner_rule, tau=prob.tau)
        assert ref.status == "ok" and ref.m == res.m
        assert np.all(np.abs(np.sort_complex(ref.lam_in) - np.sort_complex(res.lam_in)) <= tol)


# ------------------------------------------------------------- generalized (B SPD)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_generalized_constant_closed_form(ctx, prec):
    """A x = lambda B x with the constant-coefficient 27-point A and Q1 mass B on a 24^3 grid
    (Eq. generalized_linsys): the 17 lowest eigenvalues (clusters of multiplicity up to 6)
    against lambda = (27 - prod(1 + 2 t_i)) / prod((4 + 2 t_i) / 6), residuals <= tol and
    B-orthonormal eigenvectors, through the per-shift restarted block GMRES."""
    import paper_1706_00692_amd as pk

    N = 24
    ev = W.config3_constant_spectrum(N)
    want = ev[:17]
    prob = W.config3(N, m0=32, emin=0.5 * ev[0], emax=0.5 * (ev[16] + ev[17]), constant=True)
    res = ctx.solve_problem(prob, precision=pk.PREC_FP64 if prec == "fp64" else pk.PREC_MIXED)
    print(f"[gen const {N}^3 {prec}] status={res.status} m={res.m} outer={res.outer_iters} rf={res.max_resid:.2e} "
          f"t={res.solve_seconds:.2f}s", flush=True)
    assert res.status == 0 and res.converged and res.m == 17
    assert np.allclose(np.sort(res.lam_in), want, rtol=1e-10, atol=0)
    assert res.resid[: res.m].max() <= prob.tol
    B = prob.B.to_scipy()
    assert np.allclose(res.X_in.T @ (B @ res.X_in), np.eye(17), atol=1e-9)


def test_solve_generalized_random_vs_dense(ctx):
    """The random-coefficient generalized pair on a 12^3 grid (mixed precision): the eigenvalues
    inside an interval of the low spectrum against dense eigh(A, B), eigenvectors as subspaces."""
    import scipy.linalg as sla
    import paper_1706_00692_amd as pk

    N = 12
    prob = W.config3(N, m0=16)
    lam_all, V = sla.eigh(prob.A.to_dense(), prob.B.to_dense())
    prob.contour = dict(prob.contour, emin=0.5 * (lam_all[1] + lam_all[2]), emax=0.5 * (lam_all[10] + lam_all[11]))
    res = ctx.solve_problem(prob, precision=pk.PREC_MIXED)
    assert res.status == 0 and res.converged and res.m == 9
    assert np.allclose(np.sort(res.lam_in), lam_all[2:11], rtol=1e-10, atol=0)
    assert res.resid[: res.m].max() <= prob.tol
    B = prob.B.to_scipy()
    Xg, Xr = res.X_in, V[:, 2:11]
    sines = np.linalg.norm(Xr - Xg @ (Xg.T @ (B @ Xr)), axis=0)
    assert sines.max() <= 1e-7, sines.max()


# ------------------------------------------------------------- MINRES inner solves
def test_filter_parity_minres_fp64(ctx, torch_cuda):
    """Batched shifted MINRES (one Lanczos recurrence per column serving every shift, three-term
    direction updates) against the oracle's column-by-column minimal-residual iterates: 16 steps
    on every (column, shift), FP64, configuration 1."""
    import paper_1706_00692_amd as pk

    torch = torch_cuda
    prob = W.config1()
    lam, X, R, r = _first_iterate(prob)
    A = prob.A.to_scipy()
    z, w, half = contour_nodes(prob.contour)
    D = [O.minres_columns(O.shifted_operator(A, None, zk), R / (zk - lam)[None, :], 16, 0.0)[0] for zk in z]
    want = O.quad_accumulate(X, lam, D, z, w, half)
    Am = ctx.matrix(prob.A)
    p = pk.params_struct(prob.m0, max_outer=1, max_inner=4, max_cycles=4, alpha=0.0, tol=1e-9,
                         precision=pk.PREC_FP64, basis=pk.BASIS_MINRES)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Qd = torch.zeros_like(Xd)
    iters = ctx.filter(Am, None, prob.contour, p, Xd, torch.from_numpy(lam).cuda(),
                       torch.from_numpy(np.ascontiguousarray(R)).cuda(), 1.0, Qd)
    torch.cuda.synchronize()
    assert list(iters) == [16] * 8
    err = np.abs(Qd.cpu().numpy() - want).max() / np.abs(want).max()
    assert err <= 1e-8, err


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_minres_inner(ctx, prec):
    """Whole solves with MINRES inner solves: configuration 1 against its closed form and the
    oracle (MINRES inner solves too), a ragged 9^3 Laplacian + potential against dense eigh."""
    import paper_1706_00692_amd as pk

    pr = pk.PREC_FP64 if prec == "fp64" else pk.PREC_MIXED
    prob = W.config1()
    res = ctx.solve_problem(prob, precision=pr, basis=pk.BASIS_MINRES)
    ref = O.ifeast(prob.A, None, prob.contour, prob.m0, prob.max_inner, prob.alpha, prob.tol, prob.x0(),
                   prob.max_outer, max_cycles=prob.max_cycles, inner_rule=prob.inner_rule, tau=prob.tau,
                   inner="minres")
    _check_against_oracle(prob, res, ref)
    mu = 2 - 2 * np.cos(np.arange(1, 21) * np.pi / 21)
    exact = np.sort((mu[:, None] + mu[None, :]).ravel())
    assert np.allclose(np.sort(res.lam_in), exact[(exact > 0.5) & (exact < 0.8)], rtol=1e-10, atol=0)
    N = 9
    lam_all = np.linalg.eigvalsh(W.laplacian_3d(N, W.random_potential(N ** 3, 1002)).to_dense())
    prob = W.config2_small(N=N, m0=32, emin=0.5 * (lam_all[3] + lam_all[4]), emax=0.5 * (lam_all[15] + lam_all[16]))
    res = ctx.solve_problem(prob, precision=pr, basis=pk.BASIS_MINRES)
    assert res.status == 0 and res.m == 12
    assert np.allclose(np.sort(res.lam_in), lam_all[4:16], rtol=1e-10, atol=0)
    assert res.resid[: res.m].max() <= prob.tol
