"""IFEAST benchmark on one MI355X.

A step is one full IFEAST solve (Algorithm 2: initial Rayleigh-Ritz, outer
iterations of inexact block-GMRES shifted solves, quadrature sum, Rayleigh-Ritz
and residuals until ||R_F|| <= tol) with A already resident in HBM.  The
headline value is converged eigenpairs per second of the mixed precision path
(FP32 inner solves on one real Krylov basis shared by every shift, FP64 outer
iteration) on the 64^3 Laplacian + potential; the FP64 path is timed beside it
on the same inputs, and other configurations (--extras, --workload) are solved
as extra keys.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    """(problem, label, reference eigenvalues inside the contour or None)."""
    import workloads as W

    if name == "c1":
        return W.config1(), "lap2d_20x20_n400_m0_16_gl8_k4", None
    if name == "c2":
        return W.config2(64), "lap3d_pot_64^3_n262144_m0_80_gl8_k8", None
    if name.startswith("c2_"):
        N = int(name.split("_")[1])
        return W.config2(N), f"lap3d_pot_{N}^3_m0_80_gl8_k8", None
    if name.startswith("c3"):
        # the generalized pair with constant coefficients (closed-form spectrum): the ~100 lowest
        # eigenvalues, m0 = 128, 12 Gauss-Legendre nodes, GMRES(8) per shift
        N = int(name.split("_")[1]) if "_" in name else 100
        ev = W.config3_constant_spectrum(N)
        k = 96 if N == 100 else int(np.searchsorted(ev, ev[min(95, len(ev) - 2)] + 1e-9))
        prob = W.config3(N, m0=128, emin=0.5 * ev[0], emax=0.5 * (ev[k - 1] + ev[k]), constant=True)
        return prob, f"spd27_mass_const_{N}^3_n{N ** 3}_m0_128_gl12_k8", ev[:k]
    if name.startswith("c4"):
        N = int(name.split("_")[1]) if "_" in name else 512
        prob = W.config4(N)
        return prob, f"convdiff_{N}^2_n{N * N}_m0_64_trap16_k10_lowest{len(prob.meta['inside'])}", \
            prob.meta["inside"]
    raise SystemExit(f"unknown workload {name}")


PEAK = {  # MI355X published dense peaks
    "hbm_GBs": 8000.0,
    "fp32_TFLOPs": 157.3,
    "fp64_TFLOPs": 78.6,
}


def measured_traffic(cls):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 counter summary, when the
    kernel's source is unchanged since the counters were taken (else None)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        rec = json.load(open(path))["classes"][cls]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


def kernel_table(stats):
    """Per-class achieved rates from the library's live HIP-event timing."""
    out = {}
    for name, k in stats.items():
        if k["launches"] == 0 or k["seconds"] <= 0:
            continue
        out[name] = {"launches": k["launches"], "seconds": k["seconds"],
                     "avg_launch_us": 1e6 * k["seconds"] / k["launches"],
                     "TFLOPs": k["flops"] / k["seconds"] / 1e12, "GBs": k["bytes"] / k["seconds"] / 1e9,
                     "flops_per_launch": k["flops"] / k["launches"], "bytes_per_launch": k["bytes"] / k["launches"]}
    return out


def roofline_of(name, k, mixed):
    """Roofline entry of one kernel class: MFMA-bound products or the HBM-bound SpMM."""
    if name == "spmm":
        ach = k["GBs"]
        return {"kernel": "k_spmm (CSR times the basis block: one real block for the shared basis, all shifts' "
                          "complex blocks per shift)", "bound": "hbm", "achieved": ach,
                "peak": PEAK["hbm_GBs"], "unit": "GB/s", "frac": ach / PEAK["hbm_GBs"], "traffic": None,
                "avg_launch_us": k["avg_launch_us"], "algorithmic_bytes_per_launch": k["bytes_per_launch"]}
    peak = PEAK["fp32_TFLOPs"] if mixed else PEAK["fp64_TFLOPs"]
    kern = {"update": "k_apply (block update V H, MFMA)", "gram": "k_gram (block Gram V^T W, MFMA)",
            "qacc": "k_apply (quadrature accumulation, MFMA)", "outer": "FP64 Rayleigh-Ritz products"}[name]
    return {"kernel": kern, "bound": "mfma", "achieved": k["TFLOPs"], "peak": peak, "unit": "TFLOP/s",
            "frac": k["TFLOPs"] / peak, "traffic": None, "avg_launch_us": k["avg_launch_us"],
            "algorithmic_flops_per_launch": k["flops_per_launch"]}


def spmm_burst(ctx, pk, torch, Am, Bm, prob, shared, reps=24, sets=4):
    """Average duration of the solve's SpMM shape over a burst of back-to-back launches (one event
    pair around the burst, so event overhead does not inflate a short kernel).  The launches cycle
    over `sets` distinct input/output blocks whose total exceeds the 256 MB Infinity Cache, so each
    launch streams its block from HBM."""
    n, m0, ns = prob.A.n, prob.m0, prob.contour["nc"]
    if prob.kind == "general":
        ns //= 2  # the upper half of the circle's conjugate-symmetric rule is solved
    if shared:
        # the shared basis multiplies one real n x m0 block: n x m0/2 complex numbers, shift 0
        z, width = np.zeros(1, dtype=complex), m0 // 2
    else:
        z, width = 1.0 + 0.05j * np.arange(1, ns + 1), m0
    bufs = [(torch.randn((n, len(z) * width), dtype=torch.complex64, device="cuda"),
             torch.empty((n, len(z) * width), dtype=torch.complex64, device="cuda")) for _ in range(sets)]
    for V, W in bufs:
        ctx.spmm_shifted(Am, Bm, pk.PREC_MIXED, z, width, V, W)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for r in range(reps):
        V, W = bufs[r % sets]
        ctx.spmm_shifted(Am, Bm, pk.PREC_MIXED, z, width, V, W)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    bytes_ = (n + 1) * 4 + prob.A.nnz * 8 + 2 * n * len(z) * width * 8
    if Bm is not None:
        bytes_ += (n + 1) * 4 + prob.B.nnz * 8
    del bufs
    return sec, bytes_


def copy_calibration(torch, mib=1024, reps=3):
    """A plain device copy of known size (outside the timed region): HBM counters of profiling runs
    are scaled by what they read for it.  Returns GB/s."""
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del x, y
    return {"bytes_read": mib << 20, "bytes_written": mib << 20, "GBs": 2 * (mib << 20) / sec / 1e9}


def host_cores():
    """Cores this process may run on, the host's count, and the BLAS pool's threads."""
    import threadpoolctl

    info = threadpoolctl.threadpool_info()
    blas = max([i.get("num_threads", 1) for i in info] + [1])
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"available": avail, "host": os.cpu_count() or 1, "blas_threads": blas}


def cpu_baseline(prob, gpu_res, steps=8, full_shift=False):
    """The oracle on the host cores, on a bounded sample of the same workload.

    Sample: one Rayleigh-Ritz of the oracle at full size, and the first ``steps`` block-GMRES
    steps of one shifted system at full size (the oracle solves each shift with its own basis:
    block Arnoldi with two classical Gram-Schmidt passes and a dense least squares per step).
    The duration of every step is read from the operator applications (one per step), and a
    per-step cost a + b j fitted to them prices every (outer iteration, shift) inner solve of the
    GPU run by the block steps it took (the oracle's unrestarted per-shift block GMRES computes
    the same iterates as the GPU's shared basis).  ``full_shift``: also time one complete inner
    solve (the GPU's longest of the first outer iteration) to check the per-step model."""
    import oracle as O
    from oracle.quadrature import contour_nodes

    A = prob.A.to_scipy()
    B = None if prob.B is None else prob.B.to_scipy()
    z, w, half = contour_nodes(prob.contour)
    kind = "general" if prob.kind == "general" else "symmetric"
    t0 = time.perf_counter()
    lam, X, AX, BX, _ = O.rayleigh_ritz(A, B, prob.x0(), kind)
    R, r = O.residuals(AX, BX, lam)
    t_rr = time.perf_counter() - t0
    M = O.shifted_operator(A, B, z[0])
    rhs = R / (z[0] - lam)[None, :]
    stamps = []

    def timed_M(V):
        stamps.append(time.perf_counter())
        return M(V)

    t = time.perf_counter()
    O.block_gmres(timed_M, rhs, steps, 0.0)
    t_end = time.perf_counter()
    stamps.append(t_end)
    per = np.diff(np.array(stamps))  # duration of step j = 0 .. steps-1
    j = np.arange(len(per), dtype=float)
    b_, a_ = np.polyfit(j, per, 1)
    a_, b_ = max(a_, 0.0), max(b_, 0.0)
    hist = np.asarray(gpu_res.inner_hist, dtype=float)

    def price(J):
        return a_ * J + b_ * J * (J - 1) / 2

    est = float(np.sum(price(hist))) + t_rr * (gpu_res.outer_iters + 1)
    sampled = float(np.sum(per)) + t_rr
    cores = host_cores()
    out = {"value": gpu_res.m / est, "unit": "eigenpairs/s", "cores": cores["blas_threads"], "kind": "oracle",
           "host_cores": cores, "estimated_seconds": est, "sampled_seconds": sampled,
           "extrapolation_factor": est / sampled,
           "sample": f"oracle at full size: one Rayleigh-Ritz ({t_rr:.1f} s) and the first {len(per)} block-GMRES "
                     f"steps of one shifted system ({np.sum(per):.1f} s; per-step {per.min():.2f}-{per.max():.2f} s, "
                     f"fitted a + b j with a = {a_:.3f} s, b = {b_:.4f} s), priced over the {hist.size} "
                     f"(outer iteration, shift) inner solves of the GPU run ({int(hist.sum())} block steps) and "
                     f"one Rayleigh-Ritz per outer iteration"}
    if full_shift:
        J = int(hist[0].max()) if hist.ndim == 2 else int(hist.max())
        t = time.perf_counter()
        O.block_gmres(M, rhs, J, 0.0)
        tf = time.perf_counter() - t
        out["full_inner_solve"] = {"steps": J, "measured_seconds": tf, "model_seconds": price(J)}
    return out


def extra_solve(pk, torch, name):
    """One mixed-precision solve of another configuration, timed on its own context (an extra
    key of the JSON line, never `value`).  A name ending in "_minres" solves that configuration
    with MINRES inner solves (one solve to warm the workspace, then the timed one)."""
    minres = name.endswith("_minres")
    prob, wname, want = workload(name[: -len("_minres")] if minres else name)
    if minres:
        wname += "_minres_inner"
    ctx = pk.Context(0)
    try:
        A = ctx.matrix(prob.A)
        B = None if prob.B is None else ctx.matrix(prob.B)
        params = pk.problem_params(prob, pk.PREC_MIXED, **({"basis": pk.BASIS_MINRES} if minres else {}))
        if minres:
            ctx.solve_resident(A, B, prob.contour, params, prob.x0())
        t = time.perf_counter()
        r = ctx.solve_resident(A, B, prob.contour, params, prob.x0())
        wall = time.perf_counter() - t
    finally:
        ctx.close()
    ok = bool(r.converged and r.m > 0 and r.resid[: r.m].max() <= prob.tol)
    out = {"workload": wname, "eigenpairs_per_s": r.m / r.solve_seconds if ok else 0.0, "seconds": r.solve_seconds,
           "wall_seconds": wall, "eigenpairs": r.m, "outer_iters": r.outer_iters, "converged": ok,
           "max_resid": float(r.resid[: r.m].max()) if r.m else None, "seq_matvec": r.seq_matvec,
           "inner_steps_per_outer": r.inner_hist.max(axis=1).tolist(), "status": r.status}
    if want is not None and r.m == len(want):
        got = np.sort(r.lam_in.real)
        out["max_abs_eig_err_vs_closed_form"] = float(np.abs(got - want).max())
        out["max_rel_eig_err_vs_closed_form"] = float(np.max(np.abs(got - want) / np.abs(want)))
    log(f"extra {wname}: {out}")
    return out


def matvec_experiment(pk, N=24, want=50, m0s=(64, 80, 96, 128), ncs=(4, 10, 24), alpha=0.2):
    """Matrix-vector product counts of IFEAST against m0 and against the number of nodes, on a
    stand-in for the paper's real-space Hamiltonians (3-D Laplacian + potential), with ARPACK
    (scipy eigsh, Lanczos with implicit restarts) for the same eigenpairs as the Krylov comparison.

    IFEAST: the lowest ``want`` eigenpairs to residual 1e-10, the upper half of a trapezoidal rule
    on the circle through the interval ends, inner tolerance factor alpha.  Counted: outer
    iterations; matvecs of the shared basis (Arnoldi steps x m0: what the GPU multiplies); the
    per-shift total (sum over shifts of their own block iterations x m0: what the method costs
    when every shifted system has its own Krylov space, the paper's 'total'); and the sequential
    count (sum over outer iterations of the longest shift's block iterations, one product per
    step with the block's columns in parallel, the paper's 'sequential')."""
    import scipy.sparse.linalg as spla
    import workloads as W

    A = W.config2(N, 0.0, 1.0).A
    As = A.to_scipy()
    ncount = [0]

    def mv(x):
        ncount[0] += 1 if x.ndim == 1 else x.shape[1]
        return As @ x

    op = spla.LinearOperator(As.shape, matvec=mv, matmat=mv, dtype=np.float64)
    ref = np.sort(spla.eigsh(As, k=want + 8, which="SA", tol=1e-12)[0])
    emin, emax = ref[0] - 0.5 * (ref[1] - ref[0]), 0.5 * (ref[want - 1] + ref[want])
    rows = []
    ctx = pk.Context(0)
    Am = ctx.matrix(A)
    for m0, nc in [(m, 4) for m in m0s] + [(80, c) for c in ncs if c != 4]:
        prob = W.config2_small(N, m0, emin, emax)
        prob.contour = {"kind": "half", "emin": emin, "emax": emax, "rule": "trap", "nc": nc}
        prob.alpha, prob.tol, prob.max_outer = alpha, 1e-10, 40
        r = ctx.solve_resident(Am, None, prob.contour, pk.problem_params(prob, pk.PREC_FP64), prob.x0())
        ok = bool(r.converged and r.m == want and np.allclose(np.sort(r.lam_in), ref[:want], rtol=1e-9))
        rows.append({"m0": m0, "nc": nc, "converged": ok, "outer_iters": r.outer_iters,
                     "shared_basis_matvec": int(r.total_matvec),
                     "per_shift_total_matvec": int(r.inner_hist.sum()) * m0,
                     "sequential_matvec": int(r.seq_matvec),
                     "sequential_per_outer": r.seq_matvec / max(1, r.outer_iters),
                     "seconds": r.solve_seconds})
        log(f"matvec table: {rows[-1]}")
    Am.close()
    ctx.close()
    arpack = []
    for m0 in m0s:
        ncount[0] = 0
        vals = np.sort(spla.eigsh(op, k=want, which="SA", ncv=m0, tol=1e-10, maxiter=20000)[0])
        arpack.append({"ncv": m0, "matvec": ncount[0], "max_rel_err": float(np.max(np.abs(vals - ref[:want]) /
                                                                                   np.abs(ref[:want])))})
        log(f"arpack: {arpack[-1]}")
    return {"matrix": f"lap3d_pot_{N}^3 (n={A.n})", "eigenpairs": want, "interval": [emin, emax],
            "alpha": alpha, "tol": 1e-10, "rule": "trapezoid, upper half of the circle", "ifeast": rows,
            "arpack": arpack}


def serve_request(W, req, spectra):
    """A request of the serving stream: the 3-D Laplacian + potential (the 64^3 problem's
    generator and seed) on a grid of the drawn side, the interval from below the spectrum to the
    widest gap within two places of the (m0/2)-th eigenvalue.  spectra caches the low spectrum of
    each side (scipy's Lanczos on the host, input preparation outside the stream)."""
    import scipy.sparse.linalg as spla

    N, m0 = req["side"], req["m0"]
    A = W.config2(N, 0.0, 1.0).A
    if N not in spectra:
        spectra[N] = np.sort(spla.eigsh(A.to_scipy(), k=36, which="SA", tol=1e-6)[0])
    ev = spectra[N]
    k = m0 // 2
    i = k - 2 + int(np.argmax(np.diff(ev)[k - 3:k + 2]))  # gap between ev[i] and ev[i + 1]
    prob = W.Problem(name=f"serve_{N}_{m0}", A=A, B=None,
                     contour={"kind": "half", "emin": 0.5, "emax": float(0.5 * (ev[i] + ev[i + 1])),
                              "rule": "gl", "nc": 8},
                     m0=m0, max_inner=8, alpha=1e-2, tol=1e-9, max_outer=40, x0_seed=req["x0_seed"])
    return prob


def serve_experiment(pk, count=24, sides=(32, 48, 64), m0s=(16, 32, 64), rate=20.0, alone=3):
    """Serving: a seeded Poisson stream of eigen-solve requests submitted at their arrival times to
    one context (continuous batching: requests are admitted by device footprint and run on a pool
    of workers with their own streams and workspaces), once in each precision.  Reports completed
    requests, throughput, p50/p99 latency (completion minus submission) and, for a sample, the
    difference between the result in the stream and the result alone."""
    import workloads as W

    reqs = W.serving_requests(count, seed=3000, rate=rate, sides=sides, m0s=m0s)
    spectra = {}
    probs = [serve_request(W, r, spectra) for r in reqs]
    out = {"requests": count, "rate_per_s": rate, "sides": list(sides), "m0s": list(m0s),
           "mix": [f"{r['side']}^3/m0={r['m0']}" for r in reqs]}
    for prec_name, prec in (("mixed", pk.PREC_MIXED), ("fp64", pk.PREC_FP64)):
        ctx = pk.Context(0)
        params = [pk.problem_params(p, prec) for p in probs]
        # one warm request per shape outside the stream (SpMM autotune, code paths)
        for p, pr in {(p.n, p.m0): (p, pr) for p, pr in zip(probs, params)}.values():
            ctx.wait(ctx.submit(p.A, None, p.contour, pr, p.x0()), p.n, p.m0, p.max_outer, p.contour["nc"])
        t0 = time.perf_counter()
        tickets = []
        for req, p, pr in zip(reqs, probs, params):
            delay = req["arrival"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(ctx.submit(p.A, None, p.contour, pr, p.x0()))
        results = []
        for t, p in zip(tickets, probs):
            try:
                results.append(ctx.wait(t, p.n, p.m0, p.max_outer, p.contour["nc"]))
            except pk.IFeastError as e:
                results.append(e.status)
        span = time.perf_counter() - t0
        good = [r for r, p in zip(results, probs) if not isinstance(r, int) and r.converged and r.m > 0
                and r.resid[: r.m].max() <= p.tol]
        lat = [r.latency for r in good]
        rec = {"completed": len(good), "failed_or_unconverged": count - len(good), "span_s": span,
               "requests_per_s": len(good) / span, "eigenpairs_per_s": sum(r.m for r in good) / span,
               "latency_p50_s": float(np.percentile(lat, 50)) if lat else None,
               "latency_p99_s": float(np.percentile(lat, 99)) if lat else None}
        if prec_name == "mixed":
            diffs = []
            for i in range(min(alone, count)):
                r = results[i]
                if isinstance(r, int):
                    continue
                a = ctx.solve_problem(probs[i], precision=prec)
                if a.m == r.m and a.m > 0:
                    diffs.append(float(np.max(np.abs(np.sort(a.lam_in) - np.sort(r.lam_in)) / np.abs(a.lam_in))))
            rec["alone_vs_stream_max_rel_eig_diff"] = max(diffs) if diffs else None
        ctx.close()
        out[prec_name] = rec
        log(f"serve {prec_name}: {rec}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 path on the same inputs")
    ap.add_argument("--fp64-steps", type=int, default=5, help="timed FP64 solves (median reported)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-full-shift", action="store_true",
                    help="also time one complete oracle inner solve at full size (minutes of host time)")
    ap.add_argument("--extras", default="c4,c2_minres",
                    help="comma-separated extra configurations solved once each ('' for none)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--basis", default="auto", choices=["auto", "shared", "per_shift", "minres"])
    ap.add_argument("--max-outer", type=int, default=0, help="cap outer iterations (profiling runs only)")
    ap.add_argument("--reorth-eta", type=float, default=0.0,
                    help="orthogonality threshold of the shared basis (0: the library's default)")
    ap.add_argument("--experiment", default="", choices=["", "matvec", "serve"],
                    help="matvec: matrix-vector product counts against m0 and nc; serve: a seeded "
                         "Poisson stream of requests (throughput, p50/p99 latency); printed instead")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); see the design notes for how the "
              "path shards across GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1706_00692_amd as pk

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.experiment == "matvec":
        print(json.dumps({"experiment": "matvec counts", **matvec_experiment(pk)}), flush=True)
        return
    if args.experiment == "serve":
        print(json.dumps({"experiment": "serving stream", **serve_experiment(pk)}), flush=True)
        return
    prob, wname, want = workload(args.workload)
    general = prob.kind == "general"
    if args.max_outer:
        prob.max_outer = args.max_outer
    basis = {"auto": pk.BASIS_AUTO, "shared": pk.BASIS_SHARED, "per_shift": pk.BASIS_PER_SHIFT,
             "minres": pk.BASIS_MINRES}[args.basis]
    shared = args.basis != "per_shift" and prob.B is None
    log(f"workload {wname}: n={prob.A.n} nnz={prob.A.nnz} m0={prob.m0} nc={prob.contour['nc']} "
        f"k={prob.max_inner} contour={prob.contour} basis={args.basis}")
    ctx = pk.Context(0)
    ctx._use_torch_stream()
    Am = ctx.matrix(prob.A)
    Bm = None if prob.B is None else ctx.matrix(prob.B)
    # inputs and outputs in HBM: the seeded initial block is uploaded once, the eigenvectors
    # stay on the device (complex for a general problem)
    X0d = torch.from_numpy(prob.x0()).cuda()
    Xout = torch.empty((prob.A.n, prob.m0 * (2 if general else 1)), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def solve(c, M, MB, prec, **kw):
        params = pk.problem_params(prob, prec, basis=basis, reorth_eta=args.reorth_eta, **kw)
        t = time.perf_counter()
        r = c.solve_dev(M, MB, prob.contour, params, X0d.data_ptr(), Xout.data_ptr())
        r.extra["wall"] = time.perf_counter() - t
        return r

    if args.warmup == 0:
        # workspace allocation and the SpMM autotune happen on the first call of a shape
        r = solve(ctx, Am, Bm, pk.PREC_MIXED, max_outer=1)
        log(f"prime (one outer iteration): {r.extra['wall']:.2f}s")
    for i in range(args.warmup):
        r = solve(ctx, Am, Bm, pk.PREC_MIXED)
        log(f"warmup {i}: converged={r.converged} m={r.m} outer={r.outer_iters} rf={r.max_resid:.2e} "
            f"time={r.solve_seconds:.3f}s")
    ctx.set_timing(True)
    torch.cuda.synchronize()
    lat = []
    res = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        r = solve(ctx, Am, Bm, pk.PREC_MIXED)
        lat.append(time.perf_counter() - ts)
        res.append(r)
        log(f"step {i}: converged={r.converged} m={r.m} outer={r.outer_iters} rf={r.max_resid:.2e} "
            f"seq_matvec={r.seq_matvec} time={r.solve_seconds:.3f}s")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    kt = kernel_table(ctx.kernel_stats())
    ctx.set_timing(False)
    ok = all(r.converged and r.m > 0 and r.resid[: r.m].max() <= prob.tol for r in res)
    pairs = sum(r.m for r in res) if ok else 0
    value = pairs / total
    for name, k in kt.items():
        log(f"kernel {name}: {k['launches']} launches, {k['seconds']:.3f}s, avg {k['avg_launch_us']:.1f}us, "
            f"{k['TFLOPs']:.1f} TFLOP/s, {k['GBs']:.0f} GB/s")

    inner_dtype = ("f32 real shared Krylov basis" if shared else "c64 per-shift Krylov bases")
    out = {"metric": "eigenpairs/s at resid<=1e-9 (mixed FP32-inner/FP64-outer IFEAST)", "value": value,
           "unit": "eigenpairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * total / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": f"{inner_dtype} (inner), f64 (outer)", "data": "synthetic",
           "config": {"workload": wname, "n": prob.A.n, "nnz": prob.A.nnz, "m0": prob.m0,
                      "nc": prob.contour["nc"], "k": prob.max_inner, "max_cycles": prob.max_cycles,
                      "basis": args.basis, "contour": {k: (float(v) if isinstance(v, (float, np.floating)) else v)
                                                       for k, v in prob.contour.items()},
                      "tol": prob.tol, "eigenpairs": res[0].m, "outer_iters": res[0].outer_iters,
                      "seq_matvec": res[0].seq_matvec, "total_matvec": res[0].total_matvec,
                      "max_outer_cap": args.max_outer or None},
           "solve_latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                               "note": "back-to-back solves of the benchmark problem"},
           "converged": ok}
    if want is not None and res[0].m == len(want):
        out["max_rel_eig_err_vs_closed_form"] = float(np.max(np.abs(np.sort(res[0].lam_in.real) - want) /
                                                             np.abs(want)))
    mixed = True
    dom = max((n for n in kt if n != "outer"), key=lambda n: kt[n]["seconds"])
    out["roofline"] = roofline_of(dom, kt[dom], mixed)
    if args.basis != "per_shift":
        out["roofline"]["traffic"] = measured_traffic(dom)
    out["roofline"]["share_of_kernel_time"] = kt[dom]["seconds"] / sum(k["seconds"] for k in kt.values())
    if "spmm" in kt:
        sec, bytes_ = spmm_burst(ctx, pk, torch, Am, Bm, prob, shared)
        ach = bytes_ / sec / 1e9
        out["spmm_roofline"] = {"kernel": "k_spmm (CSR times the basis block: " +
                                ("one real n x m0 block)" if shared else "all shifts' complex blocks)"),
                                "bound": "hbm", "achieved": ach, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                                "frac": ach / PEAK["hbm_GBs"], "traffic": None, "avg_launch_us": sec * 1e6,
                                "algorithmic_bytes_per_launch": bytes_,
                                "in_solve_avg_launch_us": kt["spmm"]["avg_launch_us"],
                                "timing": "24 back-to-back launches at the solve's shape over 4 distinct "
                                          "blocks (more than the Infinity Cache holds), one event pair"}
        log(f"spmm burst: {sec*1e6:.1f} us/launch, {ach:.0f} GB/s ({100*ach/PEAK['hbm_GBs']:.1f}% of HBM peak)")
    out["kernels"] = kt
    # the same solve with the initial block read from host memory and the eigenvectors written
    # back to it (PCIe-inclusive; not the reported value)
    X0h = X0d.cpu().numpy()
    th = time.perf_counter()
    rh = ctx.solve_resident(Am, Bm, prob.contour,
                            pk.problem_params(prob, pk.PREC_MIXED, basis=basis, reorth_eta=args.reorth_eta), X0h)
    th = time.perf_counter() - th
    okh = rh.converged and rh.resid[: rh.m].max() <= prob.tol
    out["host_io"] = {"seconds": th, "eigenpairs_per_s": (rh.m / th) if okh else 0.0,
                      "note": "initial block from host memory, eigenvectors back to host memory"}
    log(f"host io solve: {th:.3f}s")

    if not args.no_fp64:
        c64 = pk.Context(0)
        c64._use_torch_stream()
        A64 = c64.matrix(prob.A)
        B64 = None if prob.B is None else c64.matrix(prob.B)
        solve(c64, A64, B64, pk.PREC_FP64)  # warm (its own workspace)
        runs = [solve(c64, A64, B64, pk.PREC_FP64) for _ in range(max(1, args.fp64_steps))]
        walls = [r.extra["wall"] for r in runs]
        r64 = runs[int(np.argsort(walls)[len(walls) // 2])]
        log(f"fp64: converged={r64.converged} m={r64.m} outer={r64.outer_iters} median time={np.median(walls):.3f}s")
        ok64 = all(r.converged and r.m > 0 and r.resid[: r.m].max() <= prob.tol for r in runs)
        med = float(np.median(walls))
        out["fp64"] = {"eigenpairs_per_s": (r64.m / med) if ok64 else 0.0, "seconds_median": med,
                       "seconds_min": float(np.min(walls)), "seconds_max": float(np.max(walls)),
                       "timed_solves": len(walls), "outer_iters": r64.outer_iters, "converged": bool(ok64)}
        if ok64 and ok:
            a, b = np.sort_complex(res[0].lam_in), np.sort_complex(r64.lam_in)
            if len(a) == len(b):
                out["mixed_vs_fp64_max_rel_eig_diff"] = float(np.max(np.abs(a - b) / np.abs(b)))
            # both per solve: the mixed path's mean over its timed loop against the FP64 median
            out["mixed_over_fp64_speedup"] = value / out["fp64"]["eigenpairs_per_s"]
        A64.close()
        if B64 is not None:
            B64.close()
        c64.close()

    out["copy_calibration"] = copy_calibration(torch)
    log(f"copy calibration: {out['copy_calibration']}")
    Am.close()
    if Bm is not None:
        Bm.close()
    ctx.close()
    for name in [e for e in args.extras.split(",") if e and e != args.workload]:
        out[f"extra_{name}"] = extra_solve(pk, torch, name)
    if not args.no_serve:
        sv = serve_experiment(pk)
        out["serving"] = sv
        out["latency_s"] = {"p50": sv["mixed"]["latency_p50_s"], "p99": sv["mixed"]["latency_p99_s"],
                            "fp64_p50": sv["fp64"]["latency_p50_s"], "fp64_p99": sv["fp64"]["latency_p99_s"],
                            "note": "completion minus submission over a seeded Poisson stream (20 requests/s) "
                                    "of 3-D Laplacian + potential solves, sides 32-64, m0 16-64"}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, res[0], full_shift=args.cpu_full_shift)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
