"""The allocation-free Rayleigh-Ritz entry point (ifeast_rayleigh_ritz_dev_noalloc) against the
allocating one (ifeast_rayleigh_ritz_dev) through the C ABI: several calls in a row on one
context, each next one on a smaller or different input, with B = I and with an SPD B.  Both
run the same kernels, so the outputs agree to rounding (eigenvectors up to sign)."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _outputs(torch, n, m0):
    return {k: torch.zeros(v, dtype=torch.float64, device="cuda") for k, v in
            dict(lam=m0, X=(n, m0), R=(n, m0), resid=m0, eta=m0).items()}


def test_noalloc_rayleigh_ritz_matches_allocating_entry_point(torch_cuda):
    import paper_1706_00692_amd as pk

    torch = torch_cuda
    ctx = pk.Context(0)
    try:
        cases = [
            (W.laplacian_3d(9, W.random_potential(729, 5)), None, 32),  # n = 729: ragged tiles
            (W.laplacian_3d(6, W.random_potential(216, 6)), None, 16),  # smaller
            (W.spd27(6, 21), W.mass27(6, 22), 32),
            (W.spd27(5, 23), W.mass27(5, 24), 16),  # smaller, B given
        ]
        for i, (A, B, m0) in enumerate(cases):
            print(f"[noalloc] case {i}: n={A.n} m0={m0} B={'yes' if B is not None else 'no'}", flush=True)
            Am = ctx.matrix(A)
            Bm = None if B is None else ctx.matrix(B)
            Q = np.random.default_rng(40 + i).standard_normal((A.n, m0))
            Qd = torch.from_numpy(Q).cuda()
            ref, got = _outputs(torch, A.n, m0), _outputs(torch, A.n, m0)
            ctx.rayleigh_ritz(Am, Bm, Qd, ref["lam"], ref["X"], ref["R"], ref["resid"], ref["eta"])
            ctx.rayleigh_ritz_noalloc(Am, Bm, Qd, got["lam"], got["X"], got["R"], got["resid"], got["eta"])
            torch.cuda.synchronize()
            r = {k: v.cpu().numpy() for k, v in ref.items()}
            g = {k: v.cpu().numpy() for k, v in got.items()}
            assert np.allclose(g["lam"], r["lam"], rtol=1e-12, atol=1e-13 * np.abs(r["lam"]).max())
            sgn = np.sign(np.sum(g["X"] * r["X"], axis=0))
            assert np.abs(g["X"] * sgn[None, :] - r["X"]).max() <= 1e-10 * np.abs(r["X"]).max()
            assert np.abs(g["R"] * sgn[None, :] - r["R"]).max() <= 1e-10 * max(np.abs(r["R"]).max(), 1e-300)
            assert np.allclose(g["resid"], r["resid"], rtol=1e-9, atol=1e-14)
            assert np.allclose(g["eta"], r["eta"], rtol=1e-10)
            # the input block is left as it was
            assert np.array_equal(Qd.cpu().numpy(), Q)
            Am.close()
            if Bm is not None:
                Bm.close()
    finally:
        ctx.close()


def test_noalloc_rejects_problems_beyond_its_scratch(torch_cuda):
    """B given: B Q needs n m0 doubles of scratch; 120,000 x 128 exceeds the 64 MiB array and
    the call fails with INVALID_ARG before queueing any work."""
    import paper_1706_00692_amd as pk

    torch = torch_cuda
    n, m0 = 120000, 128
    D = W.CSR(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.full(n, 2.0))
    ctx = pk.Context(0)
    try:
        Dm = ctx.matrix(D)
        Qd = torch.zeros((n, m0), dtype=torch.float64, device="cuda")
        out = _outputs(torch, n, m0)
        with pytest.raises(pk.IFeastError) as e:
            ctx.rayleigh_ritz_noalloc(Dm, Dm, Qd, out["lam"], out["X"], out["R"], out["resid"], out["eta"])
        assert e.value.status == -1 and "scratch" in str(e.value)
        Dm.close()
    finally:
        ctx.close()
