"""ctypes binding of libifeast (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass, field

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_HEADER = os.path.join(os.path.dirname(_PKG), "include", "ifeast.h")

PREC_FP64, PREC_MIXED = 0, 1
CONTOUR_HALF, CONTOUR_CIRCLE, CONTOUR_EXPLICIT = 0, 1, 2
RULE_GL, RULE_TRAP = 0, 1
PROBLEM_SYMMETRIC, PROBLEM_GENERAL = 0, 1
GUESS_RITZ, GUESS_ZERO = 0, 1
INNER_GLOBAL, INNER_COLUMN = 0, 1
FLAG_INSIDE, FLAG_SPURIOUS = 1, 2
STATUS = {
    0: "OK", 1: "WARN_NOT_CONVERGED", 2: "WARN_M0_TOO_SMALL", 3: "WARN_NO_EIG_IN_CONTOUR",
    -1: "ERR_INVALID_ARG", -2: "ERR_OOM", -3: "ERR_DEVICE", -4: "ERR_NUMERICAL", -5: "ERR_REJECTED",
    -6: "ERR_UNKNOWN_TICKET", -7: "ERR_UNSUPPORTED",
}


class CSRStruct(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("colind", C.c_void_p),
                ("val", C.c_void_p)]


class ContourStruct(C.Structure):
    _fields_ = [("kind", C.c_int), ("rule", C.c_int), ("nc", C.c_int), ("emin", C.c_double), ("emax", C.c_double),
                ("c_re", C.c_double), ("c_im", C.c_double), ("r", C.c_double), ("z", C.c_void_p),
                ("w", C.c_void_p), ("half", C.c_int)]


class ParamsStruct(C.Structure):
    _fields_ = [("m0", C.c_int), ("max_outer", C.c_int), ("max_inner", C.c_int), ("max_cycles", C.c_int),
                ("alpha", C.c_double), ("tol", C.c_double), ("spurious_tau", C.c_double),
                ("reorth_eta", C.c_double), ("precision", C.c_int),
                ("problem", C.c_int), ("inner_guess", C.c_int), ("inner_rule", C.c_int), ("basis", C.c_int),
                ("seed", C.c_uint64)]


class ResultStruct(C.Structure):
    _fields_ = [("m", C.c_int), ("outer_iters", C.c_int), ("converged", C.c_int), ("total_matvec", C.c_int64),
                ("seq_matvec", C.c_int64), ("max_resid", C.c_double), ("solve_seconds", C.c_double),
                ("eval_re", C.c_void_p), ("eval_im", C.c_void_p), ("evec", C.c_void_p), ("resid", C.c_void_p),
                ("flags", C.c_void_p), ("rf_hist", C.c_void_p), ("inner_hist", C.c_void_p)]


class IFeastError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class KernelStatStruct(C.Structure):
    _fields_ = [("launches", C.c_int64), ("seconds", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


BASIS_AUTO, BASIS_SHARED, BASIS_PER_SHIFT, BASIS_MINRES = 0, 1, 2, 3
KERNEL_SPMM, KERNEL_GRAM, KERNEL_UPDATE, KERNEL_QACC, KERNEL_OUTER = 0, 1, 2, 3, 4
KERNEL_NAMES = {KERNEL_SPMM: "spmm", KERNEL_GRAM: "gram", KERNEL_UPDATE: "update", KERNEL_QACC: "qacc",
                KERNEL_OUTER: "outer"}


def library_path() -> str:
    return os.environ.get("IFEAST_LIBRARY", os.path.join(_PKG, "libifeast.so"))


_LIB = None


def load_library():
    """Load libifeast.so; raises if it is missing (build it first)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"libifeast.so not found at {path}; run python -m paper_1706_00692_amd.build")
    lib = C.CDLL(path)
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double
    sig = {
        "ifeast_create": (i32, [C.POINTER(vp), i32, u64]),
        "ifeast_destroy": (i32, [vp]),
        "ifeast_set_stream": (i32, [vp, vp]),
        "ifeast_status_str": (C.c_char_p, [i32]),
        "ifeast_last_error": (C.c_char_p, [vp]),
        "ifeast_version": (C.c_char_p, []),
        "ifeast_matrix_create": (i32, [vp, C.POINTER(CSRStruct), C.POINTER(vp)]),
        "ifeast_matrix_destroy": (i32, [vp, vp]),
        "ifeast_matrix_n": (i64, [vp]),
        "ifeast_footprint": (i32, [i64, i64, i64, C.POINTER(ContourStruct), C.POINTER(ParamsStruct),
                                   C.POINTER(u64)]),
        "ifeast_solve_resident": (i32, [vp, vp, vp, C.POINTER(ContourStruct), C.POINTER(ParamsStruct), vp,
                                        C.POINTER(ResultStruct)]),
        "ifeast_solve_dev": (i32, [vp, vp, vp, C.POINTER(ContourStruct), C.POINTER(ParamsStruct), vp, vp,
                                   C.POINTER(ResultStruct)]),
        "ifeast_solve": (i32, [vp, C.POINTER(CSRStruct), C.POINTER(CSRStruct), C.POINTER(ContourStruct),
                               C.POINTER(ParamsStruct), vp, C.POINTER(ResultStruct)]),
        "ifeast_submit": (i32, [vp, C.POINTER(CSRStruct), C.POINTER(CSRStruct), C.POINTER(ContourStruct),
                                C.POINTER(ParamsStruct), vp, C.POINTER(u64)]),
        "ifeast_poll": (i32, [vp, u64, C.POINTER(i32)]),
        "ifeast_wait": (i32, [vp, u64, C.POINTER(ResultStruct), C.POINTER(dbl)]),
        "ifeast_spmm_shifted_dev": (i32, [vp, vp, vp, i32, i32, vp, i32, vp, vp]),
        "ifeast_filter_dev": (i32, [vp, vp, vp, C.POINTER(ContourStruct), C.POINTER(ParamsStruct), vp, vp, vp, dbl,
                                    vp, vp]),
        "ifeast_rayleigh_ritz_dev": (i32, [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]),
        "ifeast_rayleigh_ritz_general_dev": (i32, [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]),
        "ifeast_rayleigh_ritz_dev_noalloc": (i32, [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]),
        "ifeast_set_timing": (i32, [vp, i32]),
        "ifeast_kernel_stats": (i32, [vp, i32, C.POINTER(KernelStatStruct)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def exported_symbols():
    """Names the header declares (for ABI checks)."""
    text = open(_HEADER).read()
    return sorted(set(re.findall(r"\b(ifeast_[a-z_0-9]+)\s*\(", text)))


def _csr_struct(csr):
    rp = np.ascontiguousarray(csr.rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(csr.colind, dtype=np.int32)
    va = np.ascontiguousarray(csr.val, dtype=np.float64)
    s = CSRStruct(int(csr.n), int(len(ci)), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
    return s, (rp, ci, va)


def contour_struct(c: dict):
    """ifeast_contour from a dict: {"kind": "half", "emin", "emax", "rule": "gl"|"trap", "nc"},
    {"kind": "circle", "c", "r", "nc"} or {"kind": "explicit", "z", "w", "half", "emin", "emax"}."""
    keep = []
    s = ContourStruct()
    s.nc = int(c["nc"]) if "nc" in c else len(c["z"])
    if c["kind"] == "half":
        s.kind = CONTOUR_HALF
        s.rule = RULE_GL if c.get("rule", "gl") == "gl" else RULE_TRAP
        s.emin, s.emax = float(c["emin"]), float(c["emax"])
    elif c["kind"] == "circle":
        s.kind = CONTOUR_CIRCLE
        s.rule = RULE_TRAP
        cc = complex(c["c"])
        s.c_re, s.c_im, s.r = cc.real, cc.imag, float(c["r"])
    else:
        s.kind = CONTOUR_EXPLICIT
        z = np.ascontiguousarray(np.asarray(c["z"], dtype=np.complex128).view(np.float64))
        w = np.ascontiguousarray(np.asarray(c["w"], dtype=np.complex128).view(np.float64))
        keep += [z, w]
        s.z, s.w = z.ctypes.data, w.ctypes.data
        s.half = int(bool(c.get("half", True)))
        s.emin, s.emax = float(c.get("emin", 0.0)), float(c.get("emax", 0.0))
    return s, keep


def params_struct(m0, max_outer=50, max_inner=8, max_cycles=20, alpha=1e-2, tol=1e-9, tau=0.5,
                  precision=PREC_FP64, problem=PROBLEM_SYMMETRIC, inner_guess=GUESS_RITZ, inner_rule=INNER_COLUMN,
                  seed=0, reorth_eta=0.0, basis=0):
    return ParamsStruct(int(m0), int(max_outer), int(max_inner), int(max_cycles), float(alpha), float(tol),
                        float(tau), float(reorth_eta), int(precision), int(problem), int(inner_guess),
                        int(inner_rule), int(basis), int(seed))


def _params_from(p, precision):
    """ParamsStruct from a workloads.Problem-like object."""
    return params_struct(p.m0, p.max_outer, p.max_inner, p.max_cycles, p.alpha, p.tol, p.tau, precision,
                         PROBLEM_SYMMETRIC if p.kind == "symmetric" else PROBLEM_GENERAL, GUESS_RITZ,
                         INNER_COLUMN if p.inner_rule == "column" else INNER_GLOBAL)


def problem_params(prob, precision=PREC_FP64, **overrides) -> ParamsStruct:
    """The ifeast_params of a workloads.Problem, with field overrides."""
    params = _params_from(prob, precision)
    for k, v in overrides.items():
        setattr(params, k, v)
    return params


def _solved_systems(cs, params) -> int:
    """Shifted systems solved per outer iteration: nc, or nc / 2 for a general problem (the
    upper half of a rule symmetric about the real axis)."""
    return cs.nc // 2 if params.problem == PROBLEM_GENERAL else cs.nc


def footprint(n, nnzA, nnzB, contour: dict, params: ParamsStruct) -> int:
    lib = load_library()
    cs, keep = contour_struct(contour)
    out = C.c_uint64(0)
    st = lib.ifeast_footprint(int(n), int(nnzA), int(nnzB), C.byref(cs), C.byref(params), C.byref(out))
    if st < 0:
        raise IFeastError(st, lib.ifeast_last_error(None).decode())
    return int(out.value)


@dataclass
class Result:
    status: int
    m: int
    outer_iters: int
    converged: bool
    total_matvec: int
    seq_matvec: int
    max_resid: float
    solve_seconds: float
    lam: np.ndarray
    X: np.ndarray
    resid: np.ndarray
    flags: np.ndarray
    rf_hist: np.ndarray
    inner_hist: np.ndarray
    latency: float = float("nan")
    extra: dict = field(default_factory=dict)

    @property
    def lam_in(self):
        return self.lam[: self.m]

    @property
    def X_in(self):
        return self.X[:, : self.m]


class _ResultBuffers:
    def __init__(self, n, m0, max_outer, nc, host_evec=True, general=False):
        self.general = general
        self.eval_re = np.zeros(m0)
        self.eval_im = np.zeros(m0)
        self.evec = (np.zeros((n, m0), dtype=np.complex128 if general else np.float64) if host_evec else None)
        self.resid = np.zeros(m0)
        self.flags = np.zeros(m0, dtype=np.int32)
        self.rf_hist = np.zeros(max_outer)
        self.inner_hist = np.zeros(max_outer * nc, dtype=np.int32)
        self.s = ResultStruct()
        for name in ("eval_re", "eval_im", "evec", "resid", "flags", "rf_hist", "inner_hist"):
            arr = getattr(self, name)
            setattr(self.s, name, None if arr is None else arr.ctypes.data)

    def result(self, status, nc, latency=float("nan")):
        s = self.s
        k = s.outer_iters
        lam = self.eval_re + 1j * self.eval_im if self.general else self.eval_re.copy()
        return Result(status, s.m, s.outer_iters, bool(s.converged), s.total_matvec, s.seq_matvec, s.max_resid,
                      s.solve_seconds, lam, self.evec, self.resid.copy(), self.flags.copy(),
                      self.rf_hist[:k].copy(), self.inner_hist[: k * nc].reshape(k, nc).copy(), latency)


class Matrix:
    """A CSR matrix resident in HBM (ifeast_matrix)."""

    def __init__(self, ctx: "Context", csr):
        self.ctx = ctx
        self.n = int(csr.n)
        self.nnz = int(csr.nnz)
        s, keep = _csr_struct(csr)
        h = C.c_void_p()
        ctx._check(ctx.lib.ifeast_matrix_create(ctx.h, C.byref(s), C.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            self.ctx.lib.ifeast_matrix_destroy(self.ctx.h, self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One GPU and one stream (ifeast_ctx)."""

    def __init__(self, device: int = 0, budget: int = 0):
        self.lib = load_library()
        h = C.c_void_p()
        st = self.lib.ifeast_create(C.byref(h), int(device), int(budget))
        if st < 0:
            raise IFeastError(st, self.lib.ifeast_last_error(None).decode())
        self.h = h
        self.device = device

    def _check(self, st):
        if st < 0:
            raise IFeastError(st, self.lib.ifeast_last_error(self.h).decode())
        return st

    def close(self):
        if self.h:
            self.lib.ifeast_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def matrix(self, csr) -> Matrix:
        return Matrix(self, csr)

    def set_stream(self, stream_handle):
        self._check(self.lib.ifeast_set_stream(self.h, C.c_void_p(stream_handle) if stream_handle else None))

    def _use_torch_stream(self):
        import torch

        self.set_stream(torch.cuda.current_stream().cuda_stream)

    # --------------------------------------------------------- full solves
    def solve_resident(self, A: Matrix, B: Matrix | None, contour: dict, params: ParamsStruct, X0=None) -> Result:
        cs, keep = contour_struct(contour)
        bufs = _ResultBuffers(A.n, params.m0, params.max_outer, cs.nc, general=params.problem == PROBLEM_GENERAL)
        x0 = None if X0 is None else np.ascontiguousarray(X0, dtype=np.float64)
        st = self._check(self.lib.ifeast_solve_resident(self.h, A.h, None if B is None else B.h, C.byref(cs),
                                                         C.byref(params), None if x0 is None else x0.ctypes.data,
                                                         C.byref(bufs.s)))
        return bufs.result(st, _solved_systems(cs, params))

    def solve_dev(self, A: Matrix, B: Matrix | None, contour: dict, params: ParamsStruct, X0_ptr: int,
                  evec_ptr: int | None = None) -> Result:
        """ifeast_solve_dev: X0_ptr / evec_ptr are device addresses of n x m0 FP64 row-major
        blocks (e.g. torch tensors' data_ptr()); the result's evec is None (it is in evec_ptr)."""
        cs, keep = contour_struct(contour)
        bufs = _ResultBuffers(A.n, params.m0, params.max_outer, cs.nc, host_evec=False,
                              general=params.problem == PROBLEM_GENERAL)
        st = self._check(self.lib.ifeast_solve_dev(self.h, A.h, None if B is None else B.h, C.byref(cs),
                                                   C.byref(params), C.c_void_p(X0_ptr),
                                                   None if evec_ptr is None else C.c_void_p(evec_ptr),
                                                   C.byref(bufs.s)))
        return bufs.result(st, _solved_systems(cs, params))

    def solve(self, A, B, contour: dict, params: ParamsStruct, X0=None) -> Result:
        a, ka = _csr_struct(A)
        b, kb = (None, None) if B is None else _csr_struct(B)
        cs, keep = contour_struct(contour)
        bufs = _ResultBuffers(int(A.n), params.m0, params.max_outer, cs.nc,
                              general=params.problem == PROBLEM_GENERAL)
        x0 = None if X0 is None else np.ascontiguousarray(X0, dtype=np.float64)
        st = self._check(self.lib.ifeast_solve(self.h, C.byref(a), None if b is None else C.byref(b), C.byref(cs),
                                               C.byref(params), None if x0 is None else x0.ctypes.data,
                                               C.byref(bufs.s)))
        return bufs.result(st, _solved_systems(cs, params))

    def solve_problem(self, prob, precision=PREC_FP64, resident=None, **overrides) -> Result:
        """Solve a workloads.Problem (matrices uploaded unless given as resident Matrix objects)."""
        params = problem_params(prob, precision, **overrides)
        if resident is not None:
            A, B = resident
            return self.solve_resident(A, B, prob.contour, params, prob.x0())
        return self.solve(prob.A, prob.B, prob.contour, params, prob.x0())

    # --------------------------------------------------------- serving loop
    def submit(self, A, B, contour: dict, params: ParamsStruct, X0=None) -> int:
        a, ka = _csr_struct(A)
        b, kb = (None, None) if B is None else _csr_struct(B)
        cs, keep = contour_struct(contour)
        x0 = None if X0 is None else np.ascontiguousarray(X0, dtype=np.float64)
        t = C.c_uint64(0)
        self._check(self.lib.ifeast_submit(self.h, C.byref(a), None if b is None else C.byref(b), C.byref(cs),
                                           C.byref(params), None if x0 is None else x0.ctypes.data, C.byref(t)))
        return int(t.value)

    def poll(self, ticket: int) -> bool:
        d = C.c_int(0)
        self._check(self.lib.ifeast_poll(self.h, C.c_uint64(ticket), C.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int, n: int, m0: int, max_outer: int, nc: int, general: bool = False) -> Result:
        """nc: the shifted systems solved per outer iteration (nc / 2 for a general problem's circle)."""
        bufs = _ResultBuffers(n, m0, max_outer, nc, general=general)
        lat = C.c_double(0.0)
        st = self._check(self.lib.ifeast_wait(self.h, C.c_uint64(ticket), C.byref(bufs.s), C.byref(lat)))
        return bufs.result(st, nc, lat.value)

    # ------------------------------------------------- device-pointer steps
    def set_timing(self, enable: bool = True):
        """Reset the per-kernel-class totals and time later compute calls (HIP events on the stream)."""
        self._check(self.lib.ifeast_set_timing(self.h, int(bool(enable))))

    def kernel_stats(self) -> dict:
        """{class name: {launches, seconds, flops, bytes}} accumulated since set_timing(True)."""
        out = {}
        for k, name in KERNEL_NAMES.items():
            st = KernelStatStruct()
            self._check(self.lib.ifeast_kernel_stats(self.h, k, C.byref(st)))
            out[name] = {"launches": int(st.launches), "seconds": st.seconds, "flops": st.flops, "bytes": st.bytes}
        return out

    def spmm_shifted(self, A: Matrix, B: Matrix | None, precision: int, z, m0: int, V, W):
        """W = z_s B V_s - A V_s for all shifts (torch tensors on the device, complex64/complex128)."""
        self._use_torch_stream()
        zz = np.ascontiguousarray(np.asarray(z, dtype=np.complex128).view(np.float64))
        self._check(self.lib.ifeast_spmm_shifted_dev(self.h, A.h, None if B is None else B.h, int(precision),
                                                     len(z), zz.ctypes.data, int(m0), V.data_ptr(), W.data_ptr()))

    def filter(self, A: Matrix, B: Matrix | None, contour: dict, params: ParamsStruct, X, lam, R, rf, Q):
        """Q = X rho_hat(Lambda) + sum_k w_k D_k (device tensors, FP64); returns per-shift block iterations."""
        self._use_torch_stream()
        cs, keep = contour_struct(contour)
        iters = np.zeros(cs.nc, dtype=np.int32)
        self._check(self.lib.ifeast_filter_dev(self.h, A.h, None if B is None else B.h, C.byref(cs),
                                               C.byref(params), X.data_ptr(), lam.data_ptr(), R.data_ptr(),
                                               float(rf), Q.data_ptr(), iters.ctypes.data))
        return iters

    def rayleigh_ritz_noalloc(self, A: Matrix, B: Matrix | None, Q, lam, X, R, resid, eta):
        """Rayleigh-Ritz on span(Q) with no device allocation (scratch from the library's array)."""
        self._use_torch_stream()
        self._check(self.lib.ifeast_rayleigh_ritz_dev_noalloc(self.h, A.h, None if B is None else B.h,
                                                              int(Q.shape[1]), Q.data_ptr(), lam.data_ptr(),
                                                              X.data_ptr(), R.data_ptr(), resid.data_ptr(),
                                                              eta.data_ptr()))

    def rayleigh_ritz_general(self, A: Matrix, Q, Xprev, lam, lam_im, X, R, resid, eta):
        """Non-Hermitian Rayleigh-Ritz on span(Q) (device tensors, FP64; pair-format outputs)."""
        self._use_torch_stream()
        self._check(self.lib.ifeast_rayleigh_ritz_general_dev(
            self.h, A.h, int(Q.shape[1]), Q.data_ptr(), None if Xprev is None else Xprev.data_ptr(),
            lam.data_ptr(), lam_im.data_ptr(), X.data_ptr(), R.data_ptr(), resid.data_ptr(), eta.data_ptr()))

    def rayleigh_ritz(self, A: Matrix, B: Matrix | None, Q, lam, X, R, resid, eta):
        """Rayleigh-Ritz on span(Q) (device tensors, FP64)."""
        self._use_torch_stream()
        self._check(self.lib.ifeast_rayleigh_ritz_dev(self.h, A.h, None if B is None else B.h, int(Q.shape[1]),
                                                      Q.data_ptr(), lam.data_ptr(), X.data_ptr(), R.data_ptr(),
                                                      resid.data_ptr(), eta.data_ptr()))
