"""IFEAST benchmark on one MI355X.

A step is one full IFEAST solve (Algorithm 2: initial Rayleigh-Ritz, outer
iterations of batched restarted block-GMRES shifted solves, quadrature sum,
Rayleigh-Ritz and residuals until ||R_F|| <= tol) with A already resident in
HBM.  The headline value is converged eigenpairs per second of the mixed
precision path (complex FP32 inner solves, FP64 outer iteration); the FP64
path is timed beside it on the same inputs.

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
    import workloads as W

    if name == "c1":
        return W.config1(), "lap2d_20x20_n400_m0_16_gl8_k4"
    if name == "c2":
        return W.config2(64), "lap3d_pot_64^3_n262144_m0_80_gl8_k8"
    if name.startswith("c2_"):
        N = int(name.split("_")[1])
        return W.config2(N), f"lap3d_pot_{N}^3_m0_80_gl8_k8"
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


def spmm_burst(ctx, pk, torch, Am, prob, shared, reps=24, sets=4):
    """Average duration of the solve's SpMM shape over a burst of back-to-back launches (one event
    pair around the burst, so event overhead does not inflate a short kernel).  The launches cycle
    over `sets` distinct input/output blocks whose total exceeds the 256 MB Infinity Cache, so each
    launch streams its block from HBM."""
    n, m0, ns = prob.A.n, prob.m0, prob.contour["nc"]
    if shared:
        # the shared basis multiplies one real n x m0 block: n x m0/2 complex numbers, shift 0
        z, width = np.zeros(1, dtype=complex), m0 // 2
    else:
        z, width = 1.0 + 0.05j * np.arange(1, ns + 1), m0
    bufs = [(torch.randn((n, len(z) * width), dtype=torch.complex64, device="cuda"),
             torch.empty((n, len(z) * width), dtype=torch.complex64, device="cuda")) for _ in range(sets)]
    for V, W in bufs:
        ctx.spmm_shifted(Am, None, pk.PREC_MIXED, z, width, V, W)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for r in range(reps):
        V, W = bufs[r % sets]
        ctx.spmm_shifted(Am, None, pk.PREC_MIXED, z, width, V, W)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    bytes_ = (n + 1) * 4 + prob.A.nnz * 8 + 2 * n * len(z) * width * 8
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


def cpu_baseline(prob, gpu_res, budget_s=30.0):
    """The oracle on the host cores, on a bounded sample: block GMRES of one shifted system at
    full size for k1 and then k2 block steps (the oracle solves every shift separately with its
    own basis, CGS2 and a dense least squares per step).  A per-step cost a + b (j + 1) fitted to
    the two times prices every (outer iteration, shift) inner solve the GPU ran, by the steps it
    took; the Rayleigh-Ritz steps are timed once and counted per outer iteration."""
    import threadpoolctl
    import oracle as O
    from oracle.quadrature import contour_nodes

    A = prob.A.to_scipy()
    z, w, half = contour_nodes(prob.contour)
    t0 = time.perf_counter()
    lam, X, AX, BX, _ = O.rayleigh_ritz(A, None, prob.x0())
    R, r = O.residuals(AX, BX, lam)
    t_rr = time.perf_counter() - t0
    M = O.shifted_operator(A, None, z[0])
    rhs = R / (z[0] - lam)[None, :]
    times = {}
    for k in (2, 4):
        t = time.perf_counter()
        O.block_gmres(M, rhs, k, 0.0)
        times[k] = time.perf_counter() - t
        if time.perf_counter() - t0 > budget_s:
            break
    k1, k2 = 2, max(times)
    # T(k) = a k + b k (k + 1) / 2
    if k2 > k1:
        mat = np.array([[k1, k1 * (k1 + 1) / 2], [k2, k2 * (k2 + 1) / 2]])
        a_, b_ = np.linalg.solve(mat, np.array([times[k1], times[k2]]))
        a_, b_ = max(a_, 0.0), max(b_, 0.0)
    else:
        a_, b_ = times[k1] / k1, 0.0
    hist = np.asarray(gpu_res.inner_hist, dtype=float)
    est = float(np.sum(a_ * hist + b_ * hist * (hist + 1) / 2)) + t_rr * (gpu_res.outer_iters + 1)
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    return {"value": gpu_res.m / est, "unit": "eigenpairs/s", "cores": threads, "kind": "oracle",
            "estimated_seconds": est,
            "sample": f"oracle block GMRES of one shift at full size, {k1} and {k2} steps "
                      f"({times[k1]:.1f} s, {times[k2]:.1f} s), per-step cost fitted and applied to the "
                      f"{hist.size} (outer, shift) inner solves of the GPU run; one Rayleigh-Ritz "
                      f"({t_rr:.1f} s) per outer iteration"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 path on the same inputs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--basis", default="auto", choices=["auto", "shared", "per_shift"])
    ap.add_argument("--max-outer", type=int, default=0, help="cap outer iterations (profiling runs only)")
    ap.add_argument("--reorth-eta", type=float, default=0.0,
                    help="orthogonality threshold of the shared basis (0: the library's default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); see the design notes for how the "
              "path shards across GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1706_00692_amd as pk

    assert torch.cuda.is_available(), "bench needs a GPU"
    prob, wname = workload(args.workload)
    if args.max_outer:
        prob.max_outer = args.max_outer
    basis = {"auto": pk.BASIS_AUTO, "shared": pk.BASIS_SHARED, "per_shift": pk.BASIS_PER_SHIFT}[args.basis]
    log(f"workload {wname}: n={prob.A.n} nnz={prob.A.nnz} m0={prob.m0} nc={prob.contour['nc']} "
        f"k={prob.max_inner} interval=({prob.contour['emin']}, {prob.contour['emax']}) basis={args.basis}")
    ctx = pk.Context(0)
    ctx._use_torch_stream()
    Am = ctx.matrix(prob.A)
    # inputs and outputs in HBM: the seeded initial block is uploaded once, the eigenvectors
    # stay on the device
    X0d = torch.from_numpy(prob.x0()).cuda()
    Xout = torch.empty_like(X0d)
    torch.cuda.synchronize()

    def solve(c, M, prec, **kw):
        params = pk.problem_params(prob, prec, basis=basis, reorth_eta=args.reorth_eta, **kw)
        t = time.perf_counter()
        r = c.solve_dev(M, None, prob.contour, params, X0d.data_ptr(), Xout.data_ptr())
        r.extra["wall"] = time.perf_counter() - t
        return r

    if args.warmup == 0:
        # workspace allocation and the SpMM autotune happen on the first call of a shape
        r = solve(ctx, Am, pk.PREC_MIXED, max_outer=1)
        log(f"prime (one outer iteration): {r.extra['wall']:.2f}s")
    for i in range(args.warmup):
        r = solve(ctx, Am, pk.PREC_MIXED)
        log(f"warmup {i}: converged={r.converged} m={r.m} outer={r.outer_iters} rf={r.max_resid:.2e} "
            f"time={r.solve_seconds:.3f}s")
    ctx.set_timing(True)
    torch.cuda.synchronize()
    lat = []
    res = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        r = solve(ctx, Am, pk.PREC_MIXED)
        lat.append(time.perf_counter() - ts)
        res.append(r)
        log(f"step {i}: converged={r.converged} m={r.m} outer={r.outer_iters} rf={r.max_resid:.2e} "
            f"seq_matvec={r.seq_matvec} time={r.solve_seconds:.3f}s")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    kt = kernel_table(ctx.kernel_stats())
    ctx.set_timing(False)
    ok = all(r.converged and r.resid[: r.m].max() <= prob.tol for r in res)
    pairs = sum(r.m for r in res) if ok else 0
    value = pairs / total
    for name, k in kt.items():
        log(f"kernel {name}: {k['launches']} launches, {k['seconds']:.3f}s, avg {k['avg_launch_us']:.1f}us, "
            f"{k['TFLOPs']:.1f} TFLOP/s, {k['GBs']:.0f} GB/s")

    out = {"metric": "eigenpairs/s at resid<=1e-9 (mixed FP32-inner/FP64-outer IFEAST)", "value": value,
           "unit": "eigenpairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * total / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "c64/f32-inner, f64-outer", "data": "synthetic",
           "config": {"workload": wname, "n": prob.A.n, "nnz": prob.A.nnz, "m0": prob.m0,
                      "nc": prob.contour["nc"], "k": prob.max_inner, "max_cycles": prob.max_cycles,
                      "basis": args.basis, "interval": [prob.contour["emin"], prob.contour["emax"]],
                      "tol": prob.tol, "eigenpairs": res[0].m, "outer_iters": res[0].outer_iters,
                      "seq_matvec": res[0].seq_matvec, "total_matvec": res[0].total_matvec,
                      "max_outer_cap": args.max_outer or None},
           "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
           "converged": ok}
    mixed = True
    dom = max((n for n in kt if n != "outer"), key=lambda n: kt[n]["seconds"])
    out["roofline"] = roofline_of(dom, kt[dom], mixed)
    if args.basis != "per_shift":
        out["roofline"]["traffic"] = measured_traffic(dom)
    out["roofline"]["share_of_kernel_time"] = kt[dom]["seconds"] / sum(k["seconds"] for k in kt.values())
    if "spmm" in kt:
        shared = args.basis != "per_shift"
        sec, bytes_ = spmm_burst(ctx, pk, torch, Am, prob, shared)
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
    rh = ctx.solve_resident(Am, None, prob.contour,
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
        solve(c64, A64, pk.PREC_FP64)  # warm (its own workspace)
        r64 = solve(c64, A64, pk.PREC_FP64)
        log(f"fp64: converged={r64.converged} m={r64.m} outer={r64.outer_iters} time={r64.extra['wall']:.3f}s")
        ok64 = r64.converged and r64.resid[: r64.m].max() <= prob.tol
        out["fp64"] = {"eigenpairs_per_s": (r64.m / r64.extra["wall"]) if ok64 else 0.0,
                       "seconds": r64.extra["wall"], "outer_iters": r64.outer_iters, "converged": bool(ok64)}
        if ok64 and ok:
            a, b = np.sort(res[0].lam_in), np.sort(r64.lam_in)
            if len(a) == len(b):
                out["mixed_vs_fp64_max_rel_eig_diff"] = float(np.max(np.abs(a - b) / np.abs(b)))
            out["mixed_over_fp64_speedup"] = value / out["fp64"]["eigenpairs_per_s"]
        A64.close()
        c64.close()

    out["copy_calibration"] = copy_calibration(torch)
    log(f"copy calibration: {out['copy_calibration']}")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, res[0])
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
