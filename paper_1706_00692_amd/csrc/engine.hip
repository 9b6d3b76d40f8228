// IFEAST engine (Algorithm 2) on one GPU.
//
// Outer iteration (FP64): Rayleigh-Ritz on span(Q), residuals, membership.
// Inner solve (complex T = float for the mixed precision path, double for the
// FP64 path): for all nc shifted systems at once, restarted block GMRES from
// the Ritz initial guess, i.e. on the right-hand side R (z_s - Lambda)^{-1},
// accumulating the quadrature sum directly into the FP64 Q:
//     Q = X rho_hat(Lambda) + sum_s wf_s V_s y_s      (wf = 2w, real part, on half contours)
// Batched layout: basis block j of all shifts is one n x (nc*m0) complex
// row-major array, so the shifted SpMM of a step is a single launch and each
// shift's block is the column slice [s*m0, (s+1)*m0).
#include "engine.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <cstdio>
#include <cstdlib>

namespace ifeast {

DevBuf::DevBuf(size_t b) : bytes(b) {
  if (b > 0) IF_HIP(hipMalloc(&p, b));
}
DevBuf::~DevBuf() {
  if (p) (void)hipFree(p);
}
DevBuf& DevBuf::operator=(DevBuf&& o) noexcept {
  if (this != &o) {
    if (p) (void)hipFree(p);
    p = o.p;
    bytes = o.bytes;
    o.p = nullptr;
    o.bytes = 0;
  }
  return *this;
}

// ------------------------------------------------------------ quadrature
// Gauss-Legendre nodes/weights on [-1, 1] by Newton's method on P_n, with
// the three-term recurrence for P_n and P_n' (ascending nodes).
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wt) {
  x.assign(n, 0.0);
  wt.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double t = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = t;
        p0 = 1.0;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (t * p1 - p0) / (t * t - 1.0);
    const double w = 2.0 / ((1.0 - t * t) * dp * dp);
    x[i] = -t;
    x[n - 1 - i] = t;
    wt[i] = wt[n - 1 - i] = w;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

Nodes make_nodes(const ifeast_contour& C) {
  Nodes nd;
  const double pi = 3.14159265358979323846;
  const cd I(0.0, 1.0);
  if (C.kind == IFEAST_CONTOUR_HALF) {
    const double c = 0.5 * (C.emin + C.emax), r = 0.5 * (C.emax - C.emin);
    nd.half = true;
    if (C.rule == IFEAST_RULE_GAUSS_LEGENDRE) {
      // theta = (pi/2)(1 - x): x in [-1, 1] onto the upper half circle
      std::vector<double> x, g;
      gauss_legendre(C.nc, x, g);
      for (int k = 0; k < C.nc; ++k) {
        const double th = 0.5 * pi * (1.0 - x[k]);
        const cd e = std::exp(I * th);
        nd.z.push_back(c + r * e);
        nd.w.push_back(g[k] * r * e / 4.0);
      }
    } else {
      // upper half of the 2nc-point trapezoidal rule
      for (int k = 1; k <= C.nc; ++k) {
        const double th = pi * (k - 0.5) / C.nc;
        const cd e = std::exp(I * th);
        nd.z.push_back(c + r * e);
        nd.w.push_back(r * e / (2.0 * C.nc));
      }
    }
  } else if (C.kind == IFEAST_CONTOUR_CIRCLE) {
    nd.half = false;
    const cd c(C.c_re, C.c_im);
    for (int k = 1; k <= C.nc; ++k) {
      const double th = 2.0 * pi * (k - 0.5) / C.nc;
      const cd e = std::exp(I * th);
      nd.z.push_back(c + C.r * e);
      nd.w.push_back(C.r * e / (double)C.nc);
    }
  } else {
    nd.half = C.half != 0;
    for (int k = 0; k < C.nc; ++k) {
      nd.z.push_back(cd(C.z[2 * k], C.z[2 * k + 1]));
      nd.w.push_back(cd(C.w[2 * k], C.w[2 * k + 1]));
    }
  }
  return nd;
}

void validate_params(const ifeast_params& p, const ifeast_contour& C, int64_t n) {
  IF_REQUIRE(p.m0 > 0 && p.m0 % 16 == 0 && p.m0 <= 128, "m0 must be a multiple of 16 in [16, 128]");
  IF_REQUIRE(p.m0 <= n, "m0 must not exceed n");
  IF_REQUIRE(p.max_outer >= 1 && p.max_inner >= 1 && p.max_cycles >= 1, "iteration limits must be >= 1");
  IF_REQUIRE(p.alpha >= 0.0 && p.alpha < 1.0, "alpha must be in [0, 1)");
  IF_REQUIRE(p.tol > 0.0, "tol must be positive");
  IF_REQUIRE(p.reorth_eta >= 0.0, "reorth_eta must be >= 0");
  IF_REQUIRE(p.basis == IFEAST_BASIS_AUTO || p.basis == IFEAST_BASIS_SHARED || p.basis == IFEAST_BASIS_PER_SHIFT ||
                 p.basis == IFEAST_BASIS_MINRES,
             "unknown basis mode");
  if (p.basis == IFEAST_BASIS_MINRES && p.problem != IFEAST_PROBLEM_SYMMETRIC)
    throw Error{IFEAST_ERR_UNSUPPORTED, "MINRES inner solves take symmetric problems"};
  IF_REQUIRE(p.precision == IFEAST_PREC_FP64 || p.precision == IFEAST_PREC_MIXED, "unknown precision");
  IF_REQUIRE(p.inner_rule == IFEAST_INNER_GLOBAL || p.inner_rule == IFEAST_INNER_COLUMN, "unknown inner rule");
  IF_REQUIRE(p.problem == IFEAST_PROBLEM_SYMMETRIC || p.problem == IFEAST_PROBLEM_GENERAL, "unknown problem kind");
  if (p.inner_guess != IFEAST_GUESS_RITZ)
    throw Error{IFEAST_ERR_UNSUPPORTED, "only the Ritz initial guess (IFEAST_GUESS_RITZ) is implemented"};
  IF_REQUIRE(C.nc >= 1 && C.nc <= 64, "nc must be in [1, 64]");
  if (p.problem == IFEAST_PROBLEM_GENERAL) {
    // real A with a contour symmetric about the real axis: the conjugate nodes' solutions are the
    // conjugates of the upper ones, so the upper nc/2 are solved (the Ritz block stays real)
    if (C.kind != IFEAST_CONTOUR_CIRCLE)
      throw Error{IFEAST_ERR_UNSUPPORTED, "non-Hermitian problems use a CIRCLE contour"};
    if (C.c_im != 0.0)
      throw Error{IFEAST_ERR_UNSUPPORTED, "non-Hermitian problems need the circle centred on the real axis"};
    IF_REQUIRE(C.nc >= 2 && C.nc % 2 == 0, "a full-circle rule needs an even number of nodes");
    IF_REQUIRE(C.r > 0.0, "the circle radius must be positive");
    if (p.basis == IFEAST_BASIS_PER_SHIFT)
      throw Error{IFEAST_ERR_UNSUPPORTED, "non-Hermitian problems use the shared basis"};
    return;
  }
  if (C.kind == IFEAST_CONTOUR_HALF) {
    IF_REQUIRE(C.emax > C.emin, "emax must exceed emin");
    IF_REQUIRE(C.rule == IFEAST_RULE_GAUSS_LEGENDRE || C.rule == IFEAST_RULE_TRAPEZOID, "unknown rule");
  } else if (C.kind == IFEAST_CONTOUR_EXPLICIT) {
    IF_REQUIRE(C.z != nullptr && C.w != nullptr, "explicit contour needs z and w");
    IF_REQUIRE(C.half == 1, "symmetric problems need the upper half of a conjugate-symmetric rule");
    IF_REQUIRE(C.emax > C.emin, "explicit contour needs the interval for membership");
  } else {
    throw Error{IFEAST_ERR_UNSUPPORTED, "symmetric problems use a HALF or EXPLICIT contour"};
  }
}

// ------------------------------------------------------------ workspace
// Workgroup slots (of the multi-block Gram kernel's two per compute unit) that the least squares
// kernels on the side stream take while the basis kernels run
int g_lsq_slots = 48;

namespace {

// Pinned staging bytes for the small uploads of one shared inner solve.
constexpr size_t kStageBytes = 64 * 1024;

// Columns of the random sketch that estimates the shared basis' loss of orthogonality.
constexpr int kSketch = 16;


struct Layout {
  // byte sizes of every buffer of the workspace
  size_t X, Q, AQ, BQ, R, vec, mm, rrwork, colpart;
  size_t V, T1, H, Vh, tauh, g, y, u, flags, tol, gpart, gred, gw, Hr, Tinv, Racc, chol, Yq, Uc, zs;
  size_t Hm, Ss;  // shared basis: real block Hessenberg, per-shift start blocks
  size_t Us, Om;  // shared basis: sketch of the older blocks (n x kSketch), its random factors
  size_t Cf;      // shared basis: coefficients of the folded second pass (5 m0 x m0)
  size_t mrv, mrd, mrp, mrs;  // MINRES: three n x m0 blocks, two direction sets, partials, state
};

Layout layout(const Shape& s) {
  const size_t ts = s.precision == IFEAST_PREC_MIXED ? 4 : 8;
  const size_t n = (size_t)s.n, m0 = s.m0, ns = s.ns, m2 = 2 * m0;
  const size_t k = s.kb;  // basis capacity in blocks
  const size_t ldc = ns * m0, ldh = (k + 1) * m0;
  Layout L{};
  L.X = L.Q = L.R = n * m0 * 8;
  L.AQ = n * m0 * 8;
  L.BQ = s.hasB ? n * m0 * 8 : 0;
  L.vec = 4 * 128 * 8;
  L.mm = m0 * m0 * 8;
  L.rrwork = (s.general ? 10 * m0 * m0 + 16 * m0 : 4 * m0 * m0 + 4 * m0) * 8;
  L.colpart = (size_t)col_sumsq_blocks(s.n) * m0 * 8;
  // per-shift least squares (both modes)
  L.H = ns * ldh * k * m0 * 16;
  L.Vh = ns * k * m2 * m0 * 16;
  L.tauh = ns * k * m0 * 8;
  L.g = ns * ldh * m0 * 16;
  L.y = ns * k * m0 * m0 * 16;
  L.flags = 16 * 64 * 4;
  L.tol = ns * m0 * 8 * 2;
  L.Racc = ns * m0 * m0 * 16;
  L.chol = ns * 3 * m0 * m0 * 16;
  L.zs = 4 * 64 * 8;
  if (s.minres) {
    // no Krylov basis and no least squares: three Lanczos blocks and two sets of direction vectors
    L.H = L.Vh = L.tauh = L.g = L.y = L.u = L.Racc = L.chol = 0;
    L.V = L.T1 = L.gpart = L.gred = L.gw = L.Hr = L.Tinv = L.Yq = L.Uc = L.Hm = L.Ss = L.Us = L.Om = L.Cf = 0;
    L.gpart = gram_partial_bytes<double>(s.n, (int)m0, (int)m0, 1);
    L.mrv = 3 * n * m0 * ts;
    L.mrd = 2 * ns * n * m0 * 2 * ts;
    L.mrp = 2 * minres_partial_bytes(s.n, (int)m0);
    L.mrs = minres_state_bytes((int)m0, (int)ns);
    return L;
  }
  L.mrv = L.mrd = L.mrp = L.mrs = 0;
  if (s.shared) {
    // one real basis of k + 1 blocks (n x m0), real products of width m0
    L.V = (k + 1) * n * m0 * ts;
    L.T1 = n * m0 * ts;
    L.u = 16;
    size_t gp = std::max(gram_partial_bytes<double>(s.n, (int)m0, (int)m0, 1),
                         ts == 4 ? gram_partial_bytes<float>(s.n, kSketch, (int)m0, 1)
                                 : gram_partial_bytes<double>(s.n, kSketch, (int)m0, 1));
    for (size_t items = 1; items <= k; ++items)
      gp = std::max(gp, ts == 4 ? gram_partial_bytes<float>(s.n, (int)m0, (int)m0, (int)items)
                                : gram_partial_bytes<double>(s.n, (int)m0, (int)m0, (int)items));
    L.gpart = gp;
    L.gred = std::max(k, (size_t)4) * m0 * m0 * 8;
    L.gw = m0 * m0 * 8;
    L.Hr = k * m0 * m0 * ts;
    L.Cf = 5 * m0 * m0 * ts;
    L.Tinv = m0 * m0 * ts;
    L.Yq = k * m0 * m0 * ts;
    L.Uc = 16;
    L.Hm = ldh * k * m0 * 8;
    L.Ss = ns * m0 * m0 * 16;
    L.Us = n * kSketch * ts;
    L.Om = k * m0 * kSketch * ts;
    return L;
  }
  L.V = (k + 1) * n * ldc * 2 * ts;
  L.T1 = n * ldc * 2 * ts;
  L.u = L.g;
  // the split count depends on the item count: take the largest over every step's Gram
  size_t gp = gram_partial_bytes<double>(s.n, (int)m0, (int)m0, 1);
  for (size_t items = ns; items <= ns * k; items += ns)
    gp = std::max(gp, ts == 4 ? gram_partial_bytes<float>(s.n, (int)m2, (int)m2, (int)items)
                              : gram_partial_bytes<double>(s.n, (int)m2, (int)m2, (int)items));
  L.gpart = gp;
  L.gred = std::max(ns * k * m2 * m2, 2 * m0 * m0) * 8;
  L.gw = ns * m2 * m2 * 8;
  L.Hr = ns * k * m2 * m2 * ts;
  L.Tinv = ns * m2 * m2 * ts;
  L.Yq = ns * k * m2 * m0 * ts;
  L.Uc = ns * (k + 1) * m2 * m2 * ts;
  L.Hm = 0;
  L.Ss = 0;
  L.Us = 0;
  L.Om = 0;
  L.Cf = 0;
  return L;
}

size_t total(const Layout& L) {
  return 3 * L.X + L.AQ + L.BQ + L.R + 10 * L.vec + 6 * L.mm + L.rrwork + L.colpart + L.V + 2 * L.T1 + L.H + L.Vh +
         L.tauh + L.g + L.u + L.y + L.flags + L.tol + L.gpart + L.gred + L.gw + L.Hr + L.Tinv + L.Racc + L.chol + L.Yq +
         L.Uc + 3 * L.zs + L.Hm + L.Ss + L.Us + L.Om + L.Cf + L.mrv + L.mrd + L.mrp + L.mrs;
}

}  // namespace

uint64_t workspace_bytes(const Shape& s) { return (uint64_t)total(layout(s)); }

namespace {
// out[i][j] = X[i][order[j]] (n x m0 row-major): eigenvectors in the result order.
__global__ void k_gather_cols(int64_t n, int m0, const double* __restrict__ X, const int* __restrict__ order,
                              double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m0) return;
  const int64_t i = idx / m0;
  const int j = (int)(idx % m0);
  out[idx] = X[i * m0 + order[j]];
}

// out (n x m0 complex, interleaved)[i][j] = eigenvector order[j] from the pair-format block X.
__global__ void k_gather_complex(int64_t n, int m0, const double* __restrict__ X, const int* __restrict__ order,
                                 const double* __restrict__ lam_im, double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m0) return;
  const int64_t i = idx / m0;
  const int o = order[(int)(idx % m0)];
  const double li = lam_im[o];
  const double* row = X + i * m0;
  double re = row[o], im = 0.0;
  if (li < 0.0) {
    im = -row[o + 1];
  } else if (li > 0.0) {
    re = row[o - 1];
    im = row[o];
  }
  out[2 * idx] = re;
  out[2 * idx + 1] = im;
}

template <class T>
__global__ void k_scan(const T* __restrict__ p, int64_t count, unsigned int* __restrict__ bad, double* __restrict__ mx) {
  __shared__ double sm[256];
  double m = 0.0;
  unsigned int b = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)p[i];
    if (!isfinite(v)) ++b;
    else m = fmax(m, fabs(v));
  }
  sm[threadIdx.x] = m;
  if (b) atomicAdd(bad, b);
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) mx[blockIdx.x] = sm[0];
}
}  // namespace

// Stage-by-stage finiteness scan of device buffers (IFEAST_DEBUG=1 only).
struct DebugScan {
  bool on = false;
  DevBuf buf;
  explicit DebugScan() {
    const char* e = getenv("IFEAST_DEBUG");
    on = e && e[0] == '1';
    if (on) buf = DevBuf(64 * 8 + 8);
  }
  template <class T>
  void operator()(hipStream_t st, const char* what, const T* p, int64_t count, int a = -1, int b = -1) {
    if (!on || count <= 0) return;
    unsigned int* bad = reinterpret_cast<unsigned int*>(buf.as<char>() + 64 * 8);
    IF_HIP(hipMemsetAsync(bad, 0, 4, st));
    hipLaunchKernelGGL((k_scan<T>), dim3(64), dim3(256), 0, st, p, count, bad, buf.as<double>());
    IF_HIP(hipGetLastError());
    double mx[64];
    unsigned int nb = 0;
    IF_HIP(hipMemcpyAsync(mx, buf.p, 64 * 8, hipMemcpyDeviceToHost, st));
    IF_HIP(hipMemcpyAsync(&nb, bad, 4, hipMemcpyDeviceToHost, st));
    IF_HIP(hipStreamSynchronize(st));
    double m = 0.0;
    for (double v : mx) m = std::max(m, v);
    fprintf(stderr, "[ifeast-debug] %-14s a=%d b=%d max|x|=%.3e nonfinite=%u\n", what, a, b, m, nb);
  }
};

struct Engine::Impl {
  DebugScan dbg;
  Shape sh;
  hipStream_t st;
  Layout L;
  // outer, FP64
  DevBuf X, Q, Xn, AQ, BQ, R, lam, resid, eta, rho, C, GA, GB, rrwork, colpart, clsout;
  DevBuf lamI, rhoI, GX;  // non-Hermitian path: imaginary parts (pair format), Gram of the filtered block
  DevBuf TS, TA;          // non-Hermitian path: SVQB transform of a pass, accumulated transform
  DevBuf mrV, mrD, mrP, mrS, mrN;  // MINRES: Lanczos blocks, directions, partials, state, start norms
  // inner
  DevBuf V, T1, T2, H, Vh, tauh, g, y, u, flags, tol, gpart, gred, gwb, Hr, Tinv, Racc, chol, Yq, Uc, zsT, zsD, wsD;
  DevBuf Hm, Ss;             // shared basis
  DevBuf Us, Om;             // shared basis: sketch of the older blocks, its random factors
  DevBuf Cf;                 // shared basis: folded second-pass coefficients
  int* d_one = nullptr;      // a single 1 (the shared block's activity flag)
  int shared_steps = 0;      // Arnoldi steps of the last shared inner solve
  int* d_active = nullptr;  // ns
  int* d_run = nullptr;     // ns
  int* d_cont = nullptr;    // ns
  int* d_iters = nullptr;   // ns
  int* d_cdone = nullptr;   // ns
  int* d_cls = nullptr;     // m0 flags
  int* d_need = nullptr;    // ns flags: second Gram-Schmidt pass needed
  int* d_single = nullptr;  // ns flags: one Cholesky-QR pass is enough
  int* d_two = nullptr;     // ns flags: two Cholesky-QR passes
  double* d_loss = nullptr; // estimated loss of orthogonality of the shared basis' newest block,
                            // followed by that step's one-pass / two-pass Cholesky-QR flags
  int* d_single_sh = nullptr;
  int* d_two_sh = nullptr;
  int* d_act3 = nullptr;    // second local pass needed (twice: the two local blocks), then 1 (W's own term)
  int* d_cnt = nullptr;     // blocks normalised with one Cholesky-QR pass (shared basis)
  double single_gersh = 0.5;
  double dead_thr = 1e-280;
  int64_t single_steps = 0; // shift-steps normalised with one Cholesky-QR pass
  double reorth_eta = 0.1;  // keep-fraction below which a second pass runs (>= 1: always)
  int64_t reorth_steps = 0; // shift-steps that ran a second pass
  int64_t local_second = 0; // shared basis: steps whose first pass needed a second one against the local blocks
  double max_loss = 0.0;     // largest measured loss of orthogonality (shared basis, partial mode)
  int64_t ldc = 0, blk = 0;  // complex per row, reals per basis block

  // side stream of the shared-basis least squares updates, its events and host flag slots
  hipStream_t st_lsq = nullptr;
  hipEvent_t ev_main = nullptr, ev_lsq[2] = {nullptr, nullptr};
  int* h_flags = nullptr;  // pinned: 2 x 64 stop flags, then the step's check words
  char* h_stage = nullptr;  // pinned staging of the shared inner solve's small uploads
  size_t stage_off = 0;
  hipEvent_t ev_chk = nullptr;
  // stream of the sketch updates queued one step ahead, and its two events
  hipStream_t st_sk = nullptr;
  hipEvent_t ev_sk_go = nullptr, ev_sk_done = nullptr;
  // the third stream, created on first use (the FP32 shared basis only: engines of the FP64
  // basis, several of which may serve requests at once, keep to two streams)
  void third_stream() {
    if (st_sk) return;
    IF_HIP(hipStreamCreateWithFlags(&st_sk, hipStreamNonBlocking));
    IF_HIP(hipEventCreateWithFlags(&ev_sk_go, hipEventDisableTiming));
    IF_HIP(hipEventCreateWithFlags(&ev_sk_done, hipEventDisableTiming));
  }
  void side_stream() {
    if (st_lsq) return;
    IF_HIP(hipStreamCreateWithFlags(&st_lsq, hipStreamNonBlocking));
    IF_HIP(hipEventCreateWithFlags(&ev_main, hipEventDisableTiming));
    IF_HIP(hipEventCreateWithFlags(&ev_lsq[0], hipEventDisableTiming));
    IF_HIP(hipEventCreateWithFlags(&ev_lsq[1], hipEventDisableTiming));
    IF_HIP(hipEventCreateWithFlags(&ev_chk, hipEventDisableTiming));
    IF_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_flags), 4 * 64 * sizeof(int), hipHostMallocDefault));
    IF_HIP(hipHostMalloc(reinterpret_cast<void**>(&h_stage), kStageBytes, hipHostMallocDefault));
  }
  ~Impl() {
    if (st_lsq) (void)hipStreamSynchronize(st_lsq);
    if (st_sk) (void)hipStreamSynchronize(st_sk);
    if (h_flags) (void)hipHostFree(h_flags);
    if (h_stage) (void)hipHostFree(h_stage);
    for (hipEvent_t e : {ev_main, ev_lsq[0], ev_lsq[1], ev_chk, ev_sk_go, ev_sk_done})
      if (e) (void)hipEventDestroy(e);
    if (st_lsq) (void)hipStreamDestroy(st_lsq);
    if (st_sk) (void)hipStreamDestroy(st_sk);
  }
  Impl(const Impl&) = delete;
  Impl& operator=(const Impl&) = delete;

  Impl(hipStream_t s, const Shape& shape) : sh(shape), st(s), L(layout(shape)) {
    X = DevBuf(L.X);
    Q = DevBuf(L.Q);
    Xn = DevBuf(L.X);
    AQ = DevBuf(L.AQ);
    if (L.BQ) BQ = DevBuf(L.BQ);
    R = DevBuf(L.R);
    lam = DevBuf(L.vec);
    resid = DevBuf(L.vec);
    eta = DevBuf(L.vec);
    rho = DevBuf(L.vec);
    clsout = DevBuf(L.vec);
    C = DevBuf(L.mm);
    GA = DevBuf(L.mm);
    GB = DevBuf(L.mm);
    GX = DevBuf(L.mm);
    if (sh.general) {
      TS = DevBuf(L.mm);
      TA = DevBuf(L.mm);
    }
    lamI = DevBuf(L.vec);
    rhoI = DevBuf(L.vec);
    launch_fill_zero(st, lamI.p, lamI.bytes);
    launch_fill_zero(st, rhoI.p, rhoI.bytes);
    rrwork = DevBuf(L.rrwork);
    colpart = DevBuf(L.colpart);
    V = DevBuf(L.V);
    T1 = DevBuf(L.T1);
    T2 = DevBuf(L.T1);
    H = DevBuf(L.H);
    Vh = DevBuf(L.Vh);
    tauh = DevBuf(L.tauh);
    g = DevBuf(L.g);
    u = DevBuf(L.u);
    y = DevBuf(L.y);
    flags = DevBuf(L.flags);
    tol = DevBuf(L.tol);
    gpart = DevBuf(L.gpart);
    gred = DevBuf(L.gred);
    gwb = DevBuf(L.gw);
    Hr = DevBuf(L.Hr);
    Tinv = DevBuf(L.Tinv);
    Racc = DevBuf(L.Racc);
    chol = DevBuf(L.chol);
    Yq = DevBuf(L.Yq);
    Uc = DevBuf(L.Uc);
    zsT = DevBuf(L.zs);
    zsD = DevBuf(L.zs);
    wsD = DevBuf(L.zs);
    if (L.Hm) Hm = DevBuf(L.Hm);
    if (L.mrv) {
      mrV = DevBuf(L.mrv);
      mrD = DevBuf(L.mrd);
      mrP = DevBuf(L.mrp);
      mrS = DevBuf(L.mrs);
      mrN = DevBuf(L.vec);
    }
    if (L.Ss) Ss = DevBuf(L.Ss);
    if (L.Us) Us = DevBuf(L.Us);
    if (L.Cf) Cf = DevBuf(L.Cf);
    if (L.Om) {
      // fixed Gaussian factors, variance 1 / kSketch: E ||Om^T x||^2 = ||x||^2
      Om = DevBuf(L.Om);
      std::mt19937_64 gen(0x5eed5ce7c4ULL);
      std::normal_distribution<double> nd(0.0, 1.0 / std::sqrt((double)kSketch));
      const bool f32 = sh.precision == IFEAST_PREC_MIXED;
      const size_t cnt = L.Om / (f32 ? 4 : 8);
      if (!f32) {
        std::vector<double> h(cnt);
        for (auto& x : h) x = nd(gen);
        h2d(Om.p, h.data(), L.Om);
      } else {
        std::vector<float> h(cnt);
        for (auto& x : h) x = (float)nd(gen);
        h2d(Om.p, h.data(), L.Om);
      }
    }
    int* f = flags.as<int>();
    d_active = f;
    d_run = f + 64;
    d_cont = f + 128;
    d_iters = f + 192;
    d_cdone = f + 256;
    d_cls = f + 320;
    d_need = f + 448;
    d_single = f + 512;
    d_two = f + 576;
    d_one = f + 640;
    d_loss = reinterpret_cast<double*>(f + 704);
    d_single_sh = f + 706;
    d_two_sh = f + 707;
    d_act3 = f + 708;
    d_cnt = f + 720;
    ldc = (int64_t)sh.ns * sh.m0;
    blk = sh.n * ldc * 2;
    // stale basis blocks of shifts that stopped early are multiplied by zero
    // coefficients later; zero them once so they are always finite
    launch_fill_zero(st, V.p, V.bytes);
    launch_fill_zero(st, H.p, H.bytes);
    if (L.Hm) launch_fill_zero(st, Hm.p, Hm.bytes);
    const int one = 1;
    h2d(d_one, &one, sizeof(int));
  }

  // -------------------------------------------------------- Rayleigh-Ritz
  // X <- Qin C, lam, R = A X - B X Lambda, resid = ||R e_j||, eta (Algorithm 2, step 3-4)
  void rr(const ifeast_matrix* A, const ifeast_matrix* B, const double* Qin, double* Xout, double* lamv, double* Rout,
          double* residv, double* etav) {
    const int64_t n = sh.n;
    const int m0 = sh.m0;
    double* aq = AQ.as<double>();
    launch_spmm_real(st, A, m0, Qin, aq);
    const double* bq = Qin;
    if (B != nullptr) {
      launch_spmm_real(st, B, m0, Qin, BQ.as<double>());
      bq = BQ.as<double>();
    }
    GramArgs ga{n, m0, m0, 1, 1, Qin, m0, 0, 0, aq, m0, 0, 0, nullptr, GA.as<double>(), KC_OUTER};
    launch_gram<double>(st, ga, gpart.p, gpart.bytes);
    GramArgs gb{n, m0, m0, 1, 1, Qin, m0, 0, 0, bq, m0, 0, 0, nullptr, GB.as<double>(), KC_OUTER};
    launch_gram<double>(st, gb, gpart.p, gpart.bytes);
    launch_rr_small(st, m0, GA.as<double>(), GB.as<double>(), lamv, C.as<double>(), etav, rrwork.as<double>());
    // X = Q C, AX = AQ C (into R), BX = BQ C (into Xn scratch unless B = I)
    ApplyArgs ap{n, m0, m0, 1, 1, 1, Qin, m0, 0, 0, 0, C.p, 0, Xout, m0, 0, 1.0, 0.0, nullptr, nullptr, KC_OUTER};
    launch_apply<double, double>(st, ap);
    ApplyArgs aa = ap;
    aa.A = aq;
    aa.O = Rout;
    launch_apply<double, double>(st, aa);
    const double* bx = Xout;
    if (B != nullptr) {
      ApplyArgs ab = ap;
      ab.A = bq;
      ab.O = AQ.p;  // AQ is free now
      launch_apply<double, double>(st, ab);
      bx = AQ.as<double>();
    }
    launch_residual(st, n, m0, Rout, bx, lamv, Rout);
    launch_col_sumsq(st, n, m0, Rout, residv, colpart.as<double>());
  }

  // Non-Hermitian Rayleigh-Ritz (Algorithm 2, step 3, right Galerkin condition, B = I) in pair
  // format: X <- Qin C, lam + i lamI, R = A X - X Lambda_b, resid (per complex eigenvector),
  // eta from the Gram of Xprev, the block that was filtered into Qin (null: identity).  Xprev
  // may be Xout (its Gram is taken first).
  void rr_general(const ifeast_matrix* A, const double* Qin, const double* Xprev, double* Xout, double* lamv,
                  double* lamIv, double* Rout, double* residv, double* etav) {
    const int64_t n = sh.n;
    const int m0 = sh.m0;
    double* aq = AQ.as<double>();
    if (Xprev != nullptr) {
      GramArgs gx{n, m0, m0, 1, 1, Xprev, m0, 0, 0, Xprev, m0, 0, 0, nullptr, GX.as<double>(), KC_OUTER};
      launch_gram<double>(st, gx, gpart.p, gpart.bytes);
    }
    // P = Q Tacc orthonormal: three SVQB passes, P in Xn, Rout, Xn (Rout is written last)
    const double* P = Qin;
    double* pbuf[3] = {Xn.as<double>(), Rout, Xn.as<double>()};
    double* Tp = TS.as<double>();
    double* Ta = TA.as<double>();
    for (int pass = 0; pass < 3; ++pass) {
      GramArgs gb{n, m0, m0, 1, 1, P, m0, 0, 0, P, m0, 0, 0, nullptr, GB.as<double>(), KC_OUTER};
      launch_gram<double>(st, gb, gpart.p, gpart.bytes);
      launch_svqb_pass(st, m0, GB.as<double>(), Tp, Ta, pass == 0 ? 1 : 0, rrwork.as<double>());
      ApplyArgs ap{n, m0, m0, 1, 1, 1, P, m0, 0, 0, 0, Tp, 0, pbuf[pass], m0, 0, 1.0, 0.0, nullptr, nullptr,
                   KC_OUTER};
      launch_apply<double, double>(st, ap);
      P = pbuf[pass];
    }
    launch_spmm_real(st, A, m0, P, aq);
    GramArgs ga{n, m0, m0, 1, 1, P, m0, 0, 0, aq, m0, 0, 0, nullptr, GA.as<double>(), KC_OUTER};
    launch_gram<double>(st, ga, gpart.p, gpart.bytes);
    double* Wd = GB.as<double>();  // free again
    launch_rr_general(st, m0, GA.as<double>(), Ta, Xprev != nullptr ? GX.as<double>() : nullptr, lamv, lamIv, Wd,
                      C.as<double>(), etav, rrwork.as<double>());
    // X = P W, A X = (A P) W
    ApplyArgs ap{n, m0, m0, 1, 1, 1, P, m0, 0, 0, 0, Wd, 0, Xout, m0, 0, 1.0, 0.0, nullptr, nullptr, KC_OUTER};
    launch_apply<double, double>(st, ap);
    ApplyArgs aa = ap;
    aa.A = aq;
    aa.O = Rout;
    launch_apply<double, double>(st, aa);
    launch_residual_pairs(st, n, m0, Rout, Xout, lamv, lamIv, Rout);
    launch_col_sumsq(st, n, m0, Rout, residv, colpart.as<double>());
    launch_pair_norms(st, m0, lamIv, residv);
  }

  // ---------------------------------------------------------- CholQR2
  // dst_s = orthonormal basis of src_s (n x m0 complex, per shift), Racc_s = R factor.
  template <class T>
  void cholqr2(const T* src, T* tmp, T* dst, const int* act, const double* G0 = nullptr) {
    const int64_t n = sh.n;
    const int m0 = sh.m0, m2 = 2 * m0, ns = sh.ns;
    const double eps = sizeof(T) == 4 ? (double)FLT_EPSILON : DBL_EPSILON;
    const T* in = src;
    for (int pass = 0; pass < 2; ++pass) {
      T* out = pass == 0 ? tmp : dst;
      // G0: the Gram of src, already computed for every active shift
      const double* G = gred.as<double>();
      if (pass == 0 && G0 != nullptr) {
        G = G0;
      } else {
        GramArgs gg{n, m2, m2, ns, 1, in, 2 * ldc, m2, 0, in, 2 * ldc, m2, 0, act, gred.as<double>()};
        launch_gram<T>(st, gg, gpart.p, gpart.bytes);
      }
      launch_cholqr_factor<T>(st, ns, m0, G, pass == 0 ? 4.0 * m0 * eps : 0.0, act, Tinv.as<T>(),
                              Racc.as<cd>(), pass, chol.as<cd>());
      ApplyArgs ap{n, m2, m2, ns, 1, 1, in, 2 * ldc, m2, 0, 0, Tinv.p, (int64_t)m2 * m2, out, 2 * ldc, m2,
                   1.0, 0.0, act, nullptr};
      launch_apply<T, T>(st, ap);
      in = out;
    }
  }

  LsqArgs lsq_args() {
    LsqArgs a;
    a.ns = sh.ns;
    a.m0 = sh.m0;
    a.k = sh.kb;
    a.ldh = (sh.kb + 1) * sh.m0;
    a.need_u = sh.shared ? 0 : 1;
    a.H = H.as<cd>();
    a.Vh = Vh.as<cd>();
    a.tauh = tauh.as<double>();
    a.g = g.as<cd>();
    a.y = y.as<cd>();
    a.u = u.as<cd>();
    a.res = tol.as<double>() + (size_t)sh.ns * sh.m0;
    a.tol = tol.as<double>();
    a.active = d_active;
    a.iters = d_iters;
    a.cycle_done = d_cdone;
    return a;
  }

  // host-known population of a device flag array, for the kernel timer's accounting
  static void note(const int* flags, const std::vector<int>& h) {
    if (KernelTimer* kt = current_timer())
      kt->set_count(flags, (int)std::count_if(h.begin(), h.end(), [](int v) { return v != 0; }));
  }

  std::vector<int> d2h_ints(const int* d, int cnt) {
    std::vector<int> h(cnt);
    IF_HIP(hipMemcpyAsync(h.data(), d, cnt * sizeof(int), hipMemcpyDeviceToHost, st));
    IF_HIP(hipStreamSynchronize(st));
    return h;
  }
  void h2d(void* d, const void* h, size_t bytes) {
    IF_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st));
  }
  // Asynchronous upload through the pinned staging area (no wait on the host).  The area is
  // reused from the start by each shared inner solve: the previous one's uploads have
  // completed by then (its results were read back).
  void h2d_staged(void* d, const void* h, size_t bytes) {
    const size_t at = (stage_off + 255) / 256 * 256;
    if (at + bytes > kStageBytes) {
      h2d(d, h, bytes);
      return;
    }
    std::memcpy(h_stage + at, h, bytes);
    IF_HIP(hipMemcpyAsync(d, h_stage + at, bytes, hipMemcpyHostToDevice, st));
    stage_off = at + bytes;
  }

  // ------------------------------------------------- shared real basis
  // Cholesky-QR of one real n x m0 block (two passes, the first shifted); G0: its Gram.
  template <class T>
  void cholqr2_real(const T* src, T* tmp, T* dst, const double* G0 = nullptr) {
    const int64_t n = sh.n;
    const int m0 = sh.m0;
    const double eps = sizeof(T) == 4 ? (double)FLT_EPSILON : DBL_EPSILON;
    const T* in = src;
    for (int pass = 0; pass < 2; ++pass) {
      T* out = pass == 0 ? tmp : dst;
      const double* G = gred.as<double>();
      if (pass == 0 && G0 != nullptr) {
        G = G0;
      } else {
        GramArgs gg{n, m0, m0, 1, 1, in, m0, 0, 0, in, m0, 0, 0, nullptr, gred.as<double>()};
        launch_gram<T>(st, gg, gpart.p, gpart.bytes);
      }
      launch_cholqr_factor<T>(st, 1, m0, G, pass == 0 ? 4.0 * m0 * eps : 0.0, nullptr, Tinv.as<T>(), Racc.as<cd>(),
                              pass, chol.as<cd>(), true);
      ApplyArgs ap{n, m0, m0, 1, 1, 1, in, m0, 0, 0, 0, Tinv.p, 0, out, m0, 0, 1.0, 0.0, nullptr, nullptr};
      launch_apply<T, T>(st, ap);
      in = out;
    }
  }

  // Two Cholesky-QR passes, the second skipped on the device when the first Gram G0 is
  // certified well conditioned (then the first pass runs unshifted and is accurate to
  // about kappa^2 u with kappa <= (1 + g) / (1 - g), g = single_gersh).  The second pass's
  // GEMMs are left out of the kernel timer (whether they run is known on the device only).
  template <class T>
  // certified: -1 unknown on the host (the flags are set here, on the device), 1 / 0: the
  // flags d_single / d_two were set earlier and the host read them (one pass / two passes).
  // jstep >= 0: the final pass also writes the Lanczos outputs of step jstep (the subdiagonal
  // block of Hm and, with Hr_next, the next step's recurrence coefficients).
  void cholqr_adaptive_real(const T* src, T* tmp, T* dst, const double* G0, int certified = -1, int jstep = -1,
                            int ldh = 0, T* Hr_next = nullptr) {
    const int64_t n = sh.n;
    const int m0 = sh.m0;
    const double eps = sizeof(T) == 4 ? (double)FLT_EPSILON : DBL_EPSILON;
    double* hm = jstep >= 0 ? Hm.as<double>() : nullptr;
    if (certified < 0) launch_gersh_flags(st, m0, G0, single_gersh, dead_thr, d_single_sh, d_two_sh, d_cnt);
    launch_cholqr_real_ctl<T>(st, m0, G0, 4.0 * m0 * eps, Tinv.as<T>(), Racc.as<cd>(), 0, d_single_sh, 0, hm, ldh,
                              jstep, Hr_next);
    ApplyArgs a1{n, m0, m0, 1, 1, 1, src, m0, 0, 0, 0, Tinv.p, 0, dst, m0, 0, 1.0, 0.0, nullptr, nullptr};
    a1.upper0 = 1;
    launch_apply<T, T>(st, a1);
    if (certified == 1) return;
    GramArgs g2{n, m0, m0, 1, 1, dst, m0, 0, 0, dst, m0, 0, 0, d_two_sh, gred.as<double>(), -1};
    launch_gram<T>(st, g2, gpart.p, gpart.bytes);
    launch_cholqr_real_ctl<T>(st, m0, gred.as<double>(), 0.0, Tinv.as<T>(), Racc.as<cd>(), 1, d_single_sh, 1, hm,
                              ldh, jstep, Hr_next, chol.as<double>());
    ApplyArgs a2{n, m0, m0, 1, 1, 1, dst, m0, 0, 0, 0, Tinv.p, 0, tmp, m0, 0, 1.0, 0.0, d_two_sh, nullptr, -1};
    a2.upper0 = 1;
    launch_apply<T, T>(st, a2);
    launch_copy_if<T>(st, d_two_sh, n * m0, tmp, dst);
  }

  // Inner solves by batched shifted MINRES (B = I, symmetric A): one Lanczos recurrence per
  // column of R shared by every shift, minimal-residual iterates by Givens rotations of each
  // shift's complex tridiagonal, directions by three-term recurrences, Q += Re(wf_s x_s) as they
  // go.  Each (column, shift) stops by the stopping rule on its minimal residual; at most
  // k * max_cycles steps.  Returns the steps per shift.
  template <class T>
  std::vector<int> inner_minres(const ifeast_matrix* A, const Nodes& nd, const ifeast_params& p, const double* Xd,
                                const double* lamd, const double* Rd, const double* rhod,
                                const std::vector<double>& tolh, double* Qd) {
    const int64_t n = sh.n;
    const int m0 = sh.m0, ns = sh.ns, K = sh.kb;
    IF_REQUIRE(m0 % 2 == 0 && m0 <= 128, "MINRES: m0 must be even and at most 128");
    std::vector<double> zdv(2 * ns), wf(2 * ns);
    for (int s = 0; s < ns; ++s) {
      zdv[2 * s] = nd.z[s].real();
      zdv[2 * s + 1] = nd.z[s].imag();
      const cd f = nd.half ? 2.0 * nd.w[s] : nd.w[s];
      wf[2 * s] = f.real();
      wf[2 * s + 1] = f.imag();
    }
    side_stream();  // pinned host flags
    stage_off = 0;
    const std::vector<T> zero(4, (T)0);
    h2d_staged(zsT.p, zero.data(), zero.size() * sizeof(T));
    h2d_staged(zsD.p, zdv.data(), zdv.size() * sizeof(double));
    h2d_staged(wsD.p, wf.data(), wf.size() * sizeof(double));
    h2d_staged(tol.p, tolh.data(), tolh.size() * sizeof(double));
    const int64_t bs = n * m0;
    T* vb = mrV.as<T>();
    MinresRun<T> mr;
    mr.n = n;
    mr.m0 = m0;
    mr.ns = ns;
    mr.V = vb;
    mr.Vp = vb + bs;
    mr.W = vb + 2 * bs;
    mr.D1 = mrD.as<T>();
    mr.D2 = mrD.as<T>() + 2 * ns * bs;
    mr.pa = mrP.as<double>();
    mr.pb = mrP.as<double>() + minres_partial_bytes(n, m0) / sizeof(double);
    mr.state = mrS.p;
    // Q = X rho_hat(Lambda); v_1 = r / ||r|| per column
    launch_scale_cols(st, n, m0, Xd, rhod, Qd);
    launch_col_sumsq(st, n, m0, Rd, mrN.as<double>(), colpart.as<double>());
    mr.start(st, Rd, mrN.as<double>(), lamd, zsD.as<double>());
    int steps = 0;
    for (int k = 0; k < K; ++k) {
      mr.step(st, A, zsT.as<T>(), zsD.as<double>(), wsD.as<double>(), tol.as<double>(), Qd);
      steps = k + 1;
      // the pairs still iterating after step k, read one step later (the device runs on)
      IF_HIP(hipMemcpyAsync(h_flags + (k & 1) * 128, mr.column_active(), m0 * sizeof(int), hipMemcpyDeviceToHost,
                            st));
      IF_HIP(hipEventRecord(ev_lsq[k & 1], st));
      if (k >= 1) {
        IF_HIP(hipEventSynchronize(ev_lsq[(k - 1) & 1]));
        const int* hf = h_flags + ((k - 1) & 1) * 128;
        if (std::all_of(hf, hf + m0, [](int a) { return a == 0; })) break;
      }
    }
    shared_steps = steps;
    return d2h_ints(mr.shift_steps(), ns);
  }

  // Inner solves of all shifts on one real block Arnoldi of M = -A (B = I):
  //   M V_j = V_{j+1} Hm,  (z_s I - A) V_j = V_{j+1} (z_s I~ + Hm),
  // each shift's least squares min || [S0 D_s; 0] - (z_s I~ + Hm) y_s || updated per step
  // and stopped by its own rule; Q = X rho_hat(Lambda) + V Re(sum_s wf_s y_s).
  // Up to kb = k * max_cycles steps, no restarts.  Returns per-shift block iterations.
  // Non-Hermitian A (lamId != null: the Ritz block in pair format, rho + i rhoId its filter
  // values): the recurrence has no block-tridiagonal structure, so every step projects against
  // every block twice and the least squares keep the whole block Hessenberg matrix.
  template <class T>
  std::vector<int> inner_shared(const ifeast_matrix* A, const Nodes& nd, const ifeast_params& p, const double* Xd,
                                const double* lamd, const double* Rd, const double* rhod,
                                const std::vector<double>& tolh, double* Qd, const double* lamId = nullptr,
                                const double* rhoId = nullptr) {
    const bool nonsym = lamId != nullptr;
    const int64_t n = sh.n;
    const int m0 = sh.m0, ns = sh.ns, K = sh.kb, ldh = (K + 1) * m0;
    const int64_t bs = n * m0;  // elements per basis block
    T* Vb = V.as<T>();
    T* t1 = T1.as<T>();
    T* t2 = T2.as<T>();
    std::vector<double> zdv(2 * ns), wf(2 * ns);
    for (int s = 0; s < ns; ++s) {
      zdv[2 * s] = nd.z[s].real();
      zdv[2 * s + 1] = nd.z[s].imag();
      const cd f = nd.half ? 2.0 * nd.w[s] : nd.w[s];
      wf[2 * s] = f.real();
      wf[2 * s + 1] = f.imag();
    }
    side_stream();
    stage_off = 0;
    const std::vector<T> zero(4, (T)0);
    h2d_staged(zsT.p, zero.data(), zero.size() * sizeof(T));
    h2d_staged(zsD.p, zdv.data(), zdv.size() * sizeof(double));
    h2d_staged(wsD.p, wf.data(), wf.size() * sizeof(double));
    h2d_staged(tol.p, tolh.data(), tolh.size() * sizeof(double));
    // A is symmetric, so in exact arithmetic A V_j has components along V_{j-1} and V_j only
    // (block Lanczos).  Each step projects W against those two blocks twice, and the second
    // pass projects against every block when W has lost more than reorth_eta of
    // orthogonality to the older ones: ||[V_0..V_{j-2}]^T w|| / ||w|| over the columns w,
    // estimated from a Gaussian sketch U = sum_i V_i Om_i of those blocks (kSketch columns,
    // E ||U^T w||^2 = ||[V_0..]^T w||^2), so that the estimate reads n x kSketch numbers
    // instead of the whole basis.  reorth_eta >= 1 projects against every block in both passes.
    // non-Hermitian A: every pass projects against every block; the second pass runs only when
    // the sketched loss of orthogonality after the first exceeds the threshold (reorth_eta >= 1:
    // always two passes)
    const bool full_always = p.reorth_eta >= 1.0;
    const bool always = full_always || nonsym;
    const bool nonsym_sel = nonsym && !full_always;
    // default: a tenth of the inner tolerance factor for an FP32 basis (the loss then stays an
    // order of magnitude below the accuracy the inner solves ask for), near FP64 rounding for
    // an FP64 one
    const double thr = p.reorth_eta > 0.0 ? p.reorth_eta : (sizeof(T) == 4 ? std::max(1e-4, 0.1 * p.alpha) : 1e-12);
    reorth_eta = thr;
    // one Cholesky-QR pass when the block's Gram certifies kappa <= 9 in FP32 (orthonormal to
    // ~81 u, far below the orthogonality threshold) and kappa <= 3 in FP64
    single_gersh = sizeof(T) == 4 ? 0.8 : 0.5;
    dead_thr = sizeof(T) == 4 ? 1e-30 : 1e-280;
    // Q = X rho_hat(Lambda); V_0 S0 = R
    if (nonsym)
      launch_scale_pairs(st, n, m0, Xd, rhod, rhoId, lamId, Qd);
    else
      launch_scale_cols(st, n, m0, Xd, rhod, Qd);
    launch_to_T<T>(st, bs, Rd, t1);
    cholqr2_real<T>(t1, t2, Vb);
    if (nonsym)
      launch_start_rhs_pairs(st, ns, m0, Racc.as<cd>(), lamd, lamId, zsD.as<double>(), Ss.as<cd>());
    else
      launch_start_rhs(st, ns, m0, Racc.as<cd>(), lamd, zsD.as<double>(), Ss.as<cd>());
    std::vector<int> all(ns, 1);
    h2d_staged(d_active, all.data(), ns * sizeof(int));
    h2d_staged(d_run, all.data(), ns * sizeof(int));
    note(d_active, all);
    LsqArgs la = lsq_args();
    // for symmetric A, Hm is block tridiagonal up to rounding, so the least squares problems
    // keep one block above the diagonal
    la.band = nonsym ? 0 : 1;
    launch_lsq_init(st, la, Ss.as<cd>());
    // G = [V_lo..V_{lo+nb-1}]^T W
    // G = [V_lo..V_{lo+nb-1}]^T W into gred (from item 0 at gred + off items), its reduction
    // also writing block column j of Hm (block rows lo..) and the update factors Hr
    auto gram = [&](int j, int lo, int nb, int accumulate, int off = 0) {
      GramArgs gg{n, m0, m0, 1, nb, Vb + (int64_t)lo * bs, m0, 0, bs, t1, m0, 0, 0, nullptr,
                  gred.as<double>() + (int64_t)off * m0 * m0};
      gg.cmb = GramCombine{Hm.as<double>(), ldh, j, lo, accumulate, Hr.as<T>() + (int64_t)off * m0 * m0};
      launch_gram<T>(st, gg, gpart.p, gpart.bytes);
    };
    // W -= [V_lo..V_{lo+nb-1}] Hr (lower0: Hr's first block is the recurrence's R^T, lower triangular)
    auto project = [&](int lo, int nb, int lower0 = 0) {
      ApplyArgs ap{n, m0, m0, 1, nb, nb, Vb + (int64_t)lo * bs, m0, 0, 0, bs, Hr.p, 0, t1, m0, 0, -1.0, 1.0, nullptr,
                   nullptr};
      ap.lower0 = lower0;
      launch_apply<T, T>(st, ap);
    };
    GramArgs gw{n, m0, m0, 1, 1, t1, m0, 0, 0, t1, m0, 0, 0, nullptr, gwb.as<double>()};
    T* U = Us.as<T>();
    if (sizeof(T) == 4) {
      // a sketch update still queued on the third stream (a solve that ended early on an error)
      // finishes before U is cleared
      third_stream();
      IF_HIP(hipStreamWaitEvent(st, ev_sk_done, 0));
    }
    if (!always || nonsym_sel) launch_fill_zero(st, Us.p, Us.bytes);
    bool force_next = false;  // the step after a triggered third pass takes one too
    int skip_checks = 0;      // steps left before the next orthogonality estimate
    int sk_queued = -1;       // the step whose sketch update is already queued on st_sk
    const int zero_cnt = 0;
    h2d_staged(d_cnt, &zero_cnt, sizeof(int));
    side_stream();
    int jdone = 0;
    // W = M V_j = -A V_j: the shifted product with one zero shift on the block viewed as
    // n x m0/2 complex numbers (A is real, so it acts on real and imaginary parts alike).
    // Step j + 1's product is queued before the host reads the stop flags of step j - 1, so
    // the device does not wait for that read (once per solve it is not used).
    auto spmm_step = [&](int j) {
      launch_spmm_shifted<T>(st, A, nullptr, 1, m0 / 2, zsT.as<T>(), nullptr, Vb + (int64_t)j * bs, t1);
    };
    spmm_step(0);
    for (int j = 0; j < K; ++j) {
      if (nonsym_sel) {
        // one classical Gram-Schmidt pass against every block; V_j joins the sketch U of the
        // basis, and the loss of orthogonality of the projected block is estimated from U^T W
        gram(j, 0, j + 1, 0);
        project(0, j + 1);
        ApplyArgs au{n, m0, kSketch, 1, 1, 1, Vb + (int64_t)j * bs, m0, 0, 0, 0,
                     Om.as<T>() + (int64_t)j * m0 * kSketch, 0, U, kSketch, 0, 1.0, 1.0, nullptr, nullptr};
        launch_apply<T, T>(st, au);
        double* gsk = GA.as<double>();  // the outer Gram buffer is free during the inner solve
        GramArgs gs{n, kSketch, m0, 1, 1, U, kSketch, 0, 0, t1, m0, 0, 0, nullptr, gsk, KC_GRAM, 1};
        launch_gram<T>(st, gs, gpart.p, gpart.bytes);
        launch_gram<T>(st, gw, gpart.p, gpart.bytes);
        launch_sketch_check_real(st, kSketch, m0, gsk, gwb.as<double>(), d_loss);
        // one Cholesky-QR pass when the Gram certifies it; the margin covers a second pass
        launch_gersh_flags(st, m0, gwb.as<double>(), single_gersh - 4.0 * thr, dead_thr, d_single_sh, d_two_sh,
                           d_cnt);
        double* hchk = reinterpret_cast<double*>(h_flags + 128);
        IF_HIP(hipMemcpyAsync(hchk, d_loss, sizeof(double) + 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        IF_HIP(hipEventRecord(ev_chk, st));
        IF_HIP(hipEventSynchronize(ev_chk));
        max_loss = std::max(max_loss, hchk[0]);
        const int certified = h_flags[130] != 0 ? 1 : 0;
        if (!(hchk[0] <= thr)) {
          gram(j, 0, j + 1, 1);
          project(0, j + 1);
          launch_gram<T>(st, gw, gpart.p, gpart.bytes);
          ++reorth_steps;
        }
        cholqr_adaptive_real<T>(t1, t2, Vb + (int64_t)(j + 1) * bs, gwb.as<double>(), certified, j, ldh, nullptr);
      } else {
        const int lo = always ? 0 : std::max(0, j - 1), nl = j + 1 - lo;
        if (!always && j >= 1) {
          // first pass: the coefficients against V_{j-1} are those of the recurrence,
          // V_{j-1}^T M V_j = (M V_{j-1})^T V_j = Hm(j, j-1)^T, so only V_j^T W is formed (the
          // previous step's Cholesky-QR wrote Hm(j, j-1)^T into Hm and the coefficient buffer)
          gram(j, j, 1, 0, 1);
        } else {
          gram(j, lo, nl, 0);
        }
        project(lo, nl, !always && j >= 1 ? 1 : 0);
        bool full = always || lo == 0;
        int certified = -1;
        bool folded = false;  // V_{j+1} already formed (the second pass folded into the normalisation)
        if (!full) {
          const int64_t mm0 = (int64_t)m0 * m0;
          double* gwf = gred.as<double>() + nl * mm0;        // W^T W: the combined Gram's last item
          double* gsk = gred.as<double>() + (nl + 1) * mm0;  // the sketch product, beside it
          // V_{j-2} joins the older blocks: U += V_{j-2} Om_{j-2}; then the estimate from U^T W
          auto sketch_update = [&](hipStream_t s, int i) {
            ApplyArgs au{n, m0, kSketch, 1, 1, 1, Vb + (int64_t)(i - 2) * bs, m0, 0, 0, 0,
                         Om.as<T>() + (int64_t)(i - 2) * m0 * kSketch, 0, U, kSketch, 0, 1.0, 1.0, nullptr, nullptr};
            // untimed off the main stream: the event timer synchronises when the stream changes
            if (s != st) au.kclass = -1;
            launch_apply<T, T>(s, au);
          };
          if (sk_queued == j)
            IF_HIP(hipStreamWaitEvent(st, ev_sk_done, 0));
          else
            sketch_update(st, j);
          // 16 x 16 tiles: the sketch is read once per tile column, the block once.  Far below
          // the threshold the estimate is left out for a few steps: the loss grows by well under
          // a factor 2 per step (measured: at most about 1.5)
          const bool check = skip_checks == 0;
          if (check) {
            GramArgs gs{n, kSketch, m0, 1, 1, U, kSketch, 0, 0, t1, m0, 0, 0, nullptr, gsk, KC_GRAM, 1};
            launch_gram<T>(st, gs, gpart.p, gpart.bytes);
          } else {
            --skip_checks;
          }
          // the second pass's coefficients G2 = [V_{j-1}, V_j]^T W and the block's own Gram
          // W^T W in one sweep over W: items 0..nl of [V_{j-1}, V_j, W]^T W
          GramArgs g3{n, m0, m0, 1, nl + 1, Vb + (int64_t)lo * bs, m0, 0, bs, t1, m0, 0, 0, nullptr, gred.as<double>()};
          g3.A_last = t1;
          // the least squares kernels of the previous step run beside it: its row split leaves
          // their workgroup slots free
          g3.reserve = g_lsq_slots;
          launch_gram<T>(st, g3, gpart.p, gpart.bytes);
          // in one launch: the sketched estimate; the Gershgorin certificate for one Cholesky-QR
          // pass (the second Gram-Schmidt pass changes the block by rounding only, or (a full
          // pass) by at most reorth_eta per column, which the margin on the bound covers); the
          // measured loss of orthogonality the first pass left against the local blocks (the
          // second pass runs only when it exceeds a hundredth of the loss tolerated against the
          // older blocks)
          launch_step_checks(st, kSketch, m0, check ? gsk : nullptr, gwf, single_gersh - 4.0 * thr, dead_thr,
                             d_single_sh, d_two_sh, d_cnt, nl * m0, gred.as<double>(), 0.01 * thr, d_act3, d_loss);
          // the estimate and the flags in one copy.  With the FP32 basis it goes to the third
          // stream, so that the main stream goes on at once (the words are next written by step
          // j + 1's checks, which the host queues only after reading them), and step j + 1's
          // sketch update, U += V_{j-1} Om_{j-1}, follows it there, beside the single-workgroup
          // Cholesky-QR: V_{j-1} is final and this step's reads of U are queued before the event;
          // step j + 1 waits for it before its sketch product.  Measured per solve: 0.7 % and
          // 0.4 % faster in FP32, 0.65 % and 1.6 % slower with the FP64 basis, which keeps both on
          // the main stream.
          double* hchk = reinterpret_cast<double*>(h_flags + 128);
          const bool third = sizeof(T) == 4;
          hipStream_t cs = third ? st_sk : st;
          if (third) {
            IF_HIP(hipEventRecord(ev_sk_go, st));
            IF_HIP(hipStreamWaitEvent(st_sk, ev_sk_go, 0));
          }
          IF_HIP(hipMemcpyAsync(hchk, d_loss, sizeof(double) + 3 * sizeof(int), hipMemcpyDeviceToHost, cs));
          IF_HIP(hipEventRecord(ev_chk, cs));
          if (third && j + 1 < K) {
            sketch_update(st_sk, j + 1);
            IF_HIP(hipEventRecord(ev_sk_done, st_sk));
            sk_queued = j + 1;
          }
          // the common case (no pass against the older blocks) runs while the host waits: the
          // second pass, when needed, folded into the normalisation, V_{j+1} = (W - V G2) R^{-1}
          // from the Gram W^T W - G2^T G2 (the pass removes little, so the downdate loses nothing
          // to cancellation) as W R^{-1} + [V_{j-1}, V_j] (-G2 R^{-1})
          launch_gram_downdate(st, nl * m0, m0, gred.as<double>(), gwf, d_act3);
          const double eps = sizeof(T) == 4 ? (double)FLT_EPSILON : DBL_EPSILON;
          T* hr_next = j + 1 < K ? Hr.as<T>() : nullptr;
          launch_cholqr_real_ctl<T>(st, m0, gwf, 4.0 * m0 * eps, Tinv.as<T>(), Racc.as<cd>(), 0, d_single_sh, 0,
                                    Hm.as<double>(), ldh, j, hr_next);
          T* cf = Cf.as<T>();
          T* g2t = cf + (nl + 1) * mm0;
          launch_fold_second_pass<T>(st, m0, nl, gred.as<double>(), Tinv.as<T>(), cf, g2t, Hm.as<double>(), ldh, j,
                                     lo, d_act3);
          T* dst = Vb + (int64_t)(j + 1) * bs;
          ApplyArgs aw{n, m0, m0, 1, 1, 1, t1, m0, 0, 0, 0, cf + nl * mm0, 0, dst, m0, 0, 1.0, 0.0, nullptr, nullptr};
          aw.upper0 = 1;  // R^{-1}
          launch_apply<T, T>(st, aw);
          // the second pass's term (skipped on the device when not needed; left out of the timer,
          // as whether it runs is known on the device only)
          ApplyArgs av{n, m0, m0, 1, nl, nl, Vb + (int64_t)lo * bs, m0, 0, 0, bs, cf, 0, dst, m0, 0, 1.0, 1.0, d_act3,
                       nullptr, -1};
          launch_apply<T, T>(st, av);
          IF_HIP(hipEventSynchronize(ev_chk));
          const bool second = h_flags[132] != 0;
          if (second) ++local_second;
          // a third pass cleans the new block, but the block before it still carries the loss
          // into the next step's product: that step takes a third pass too, after which both
          // parents of the recurrence are clean (Simon's partial reorthogonalisation does the same)
          full = force_next || (check && !(hchk[0] <= thr));
          force_next = full && !force_next;
          if (check) {
            max_loss = std::max(max_loss, hchk[0]);
            // steps that cannot reach the threshold even if the loss doubled every step
            double e = hchk[0] * 2.0;
            while (skip_checks < 8 && e * 2.0 < thr) {
              e *= 2.0;
              ++skip_checks;
            }
          }
          if (full) skip_checks = 0;
          certified = h_flags[130] != 0 ? 1 : 0;
          if (full) {
            // the folded block is discarded: the second pass as a projection, then a third pass
            // against every block (the local blocks again: their coefficients are rounding-sized),
            // the block's Gram afresh and its normalisation
            ApplyArgs ap{n, m0, m0, 1, nl, nl, Vb + (int64_t)lo * bs, m0, 0, 0, bs, g2t, 0, t1, m0, 0, -1.0, 1.0,
                         nullptr, nullptr};
            if (second) launch_apply<T, T>(st, ap);
            gram(j, 0, j + 1, 1);
            project(0, j + 1);
            launch_gram<T>(st, gw, gpart.p, gpart.bytes);
            ++reorth_steps;
            cholqr_adaptive_real<T>(t1, t2, dst, gwb.as<double>(), certified, j, ldh, hr_next);
          } else if (certified == 0) {
            // the second Cholesky-QR pass (the first ran shifted)
            GramArgs g2{n, m0, m0, 1, 1, dst, m0, 0, 0, dst, m0, 0, 0, d_two_sh, gred.as<double>(), -1};
            launch_gram<T>(st, g2, gpart.p, gpart.bytes);
            launch_cholqr_real_ctl<T>(st, m0, gred.as<double>(), 0.0, Tinv.as<T>(), Racc.as<cd>(), 1, d_single_sh, 1,
                                      Hm.as<double>(), ldh, j, hr_next, chol.as<double>());
            ApplyArgs a2{n, m0, m0, 1, 1, 1, dst, m0, 0, 0, 0, Tinv.p, 0, t2, m0, 0, 1.0, 0.0, d_two_sh, nullptr, -1};
            a2.upper0 = 1;
            launch_apply<T, T>(st, a2);
            launch_copy_if<T>(st, d_two_sh, n * m0, t2, dst);
          }
          folded = true;
        } else {
          gram(j, lo, nl, 1);
          project(lo, nl);
          launch_gram<T>(st, gw, gpart.p, gpart.bytes);
        }
        T* dst = Vb + (int64_t)(j + 1) * bs;
        if (always) {
          cholqr2_real<T>(t1, t2, dst, gwb.as<double>());
          launch_subdiag_real(st, m0, j, ldh, Racc.as<cd>(), Hm.as<double>());
        } else if (!folded) {
          cholqr_adaptive_real<T>(t1, t2, dst, gwb.as<double>(), certified, j, ldh,
                                  j + 1 < K ? Hr.as<T>() : nullptr);
        }
      }
      // the shifts' least squares updates of step j run on the side stream, beside step
      // j + 1's basis work; their stop flags are read one step later
      IF_HIP(hipEventRecord(ev_main, st));
      IF_HIP(hipStreamWaitEvent(st_lsq, ev_main, 0));
      launch_shift_column(st_lsq, ns, m0, j, ldh, K, zsD.as<double>(), d_active, Hm.as<double>(), H.as<cd>(),
                          la.band);
      launch_lsq_step(st_lsq, la, j);
      IF_HIP(hipMemcpyAsync(h_flags + (j & 1) * 64, d_active, ns * sizeof(int), hipMemcpyDeviceToHost, st_lsq));
      IF_HIP(hipEventRecord(ev_lsq[j & 1], st_lsq));
      jdone = j + 1;
      if (j + 1 < K) spmm_step(j + 1);
      if (j >= 1) {
        // every shift had stopped after step j - 1: step j's update left the least squares
        // problems as they were (it skips stopped shifts), so the solution uses j blocks
        IF_HIP(hipEventSynchronize(ev_lsq[(j - 1) & 1]));
        const int* hf = h_flags + ((j - 1) & 1) * 64;
        const std::vector<int> act(hf, hf + ns);
        note(d_active, act);
        if (std::none_of(act.begin(), act.end(), [](int a) { return a != 0; })) {
          jdone = j;
          break;
        }
      }
    }
    IF_HIP(hipEventRecord(ev_lsq[0], st_lsq));
    IF_HIP(hipStreamWaitEvent(st, ev_lsq[0], 0));
    // a sketch update queued for a step that did not run: U is cleared by the next solve
    if (sk_queued >= 0) IF_HIP(hipStreamWaitEvent(st, ev_sk_done, 0));
    shared_steps = jdone;
    single_steps += d2h_ints(d_cnt, 1)[0];
    launch_lsq_finish(st, la, jdone);
    launch_sum_y<T>(st, ns, m0, K, jdone, y.as<cd>(), wsD.as<double>(), Yq.as<T>());
    ApplyArgs aq{n, m0, m0, 1, jdone, jdone, Vb, m0, 0, 0, bs, Yq.p, 0, Qd, m0, 0, 1.0, 1.0, nullptr, nullptr,
                 KC_QACC};
    launch_apply<T, double>(st, aq);
    return d2h_ints(d_iters, ns);
  }

  // --------------------------------------------------------- inner solve
  // Q = X rho_hat(Lambda) + sum_s wf_s V_s y_s over all GMRES(k) cycles.
  // tolh: ns x m0 host stopping thresholds.  Returns per-shift block iterations.
  template <class T>
  std::vector<int> inner(const ifeast_matrix* A, const ifeast_matrix* B, const Nodes& nd, const ifeast_params& p,
                         const double* Xd, const double* lamd, const double* Rd, const double* rhod,
                         const std::vector<double>& tolh, double* Qd) {
    const int64_t n = sh.n;
    const int m0 = sh.m0, m2 = 2 * m0, ns = sh.ns, k = sh.k, ldh = (k + 1) * m0;
    T* Vb = V.as<T>();
    T* t1 = T1.as<T>();
    T* t2 = T2.as<T>();
    // shifts (device, type T and FP64) and quadrature factors
    std::vector<T> zt(2 * ns);
    std::vector<double> zdv(2 * ns), wf(2 * ns);
    for (int s = 0; s < ns; ++s) {
      zt[2 * s] = (T)nd.z[s].real();
      zt[2 * s + 1] = (T)nd.z[s].imag();
      zdv[2 * s] = nd.z[s].real();
      zdv[2 * s + 1] = nd.z[s].imag();
      const cd f = nd.half ? 2.0 * nd.w[s] : nd.w[s];
      wf[2 * s] = f.real();
      wf[2 * s + 1] = f.imag();
    }
    h2d(zsT.p, zt.data(), zt.size() * sizeof(T));
    h2d(zsD.p, zdv.data(), zdv.size() * sizeof(double));
    h2d(wsD.p, wf.data(), wf.size() * sizeof(double));
    h2d(tol.p, tolh.data(), tolh.size() * sizeof(double));
    // Q = X rho_hat(Lambda); start blocks R (z_s - Lambda)^{-1}
    launch_scale_cols(st, n, m0, Xd, rhod, Qd);
    launch_rhs_build<T>(st, n, m0, ns, Rd, lamd, zsD.as<double>(), t1);
    dbg(st, "rhs", t1, n * ldc * 2);
    std::vector<int> run(ns, 1), total_iters(ns, 0);
    LsqArgs la = lsq_args();
    reorth_eta = p.reorth_eta > 0.0 ? p.reorth_eta : 0.1;
    // one Cholesky-QR pass leaves the basis orthonormal to about kappa^2 u: kappa <= 9 in FP32
    // (GMRES steps that stop at a relative residual of alpha), kappa <= 3 in FP64
    single_gersh = sizeof(T) == 4 ? 0.8 : 0.5;
    dead_thr = sizeof(T) == 4 ? 1e-30 : 1e-280;
    for (int cyc = 0; cyc < p.max_cycles; ++cyc) {
      h2d(d_run, run.data(), ns * sizeof(int));
      h2d(d_active, run.data(), ns * sizeof(int));
      note(d_run, run);
      note(d_active, run);
      // V_1 S = qr(start block)
      cholqr2<T>(t1, t2, Vb, d_run);
      dbg(st, "V0", Vb, n * ldc * 2, cyc);
      dbg(st, "S", reinterpret_cast<double*>(Racc.p), (int64_t)ns * m0 * m0 * 2, cyc);
      launch_lsq_init(st, la, Racc.as<cd>());
      int jdone = 0;
      for (int j = 0; j < k; ++j) {
        T* Vj = Vb + (int64_t)j * blk;
        // W = z_s V_j - A V_j (all shifts in one launch)
        launch_spmm_shifted<T>(st, A, B, ns, m0, zsT.as<T>(), d_active, Vj, t1);
        dbg(st, "W=MV", t1, n * ldc * 2, cyc, j);
        // classical Gram-Schmidt against V_0..V_j; the second pass runs only for the shifts
        // whose block kept less than the fraction reorth_eta of some column's norm
        auto cgs_pass = [&](const int* act, int accumulate) {
          GramArgs gg{n, m2, m2, ns, j + 1, Vb, 2 * ldc, m2, blk, t1, 2 * ldc, m2, 0, act, gred.as<double>()};
          launch_gram<T>(st, gg, gpart.p, gpart.bytes);
          launch_cgs_combine<T>(st, ns, j + 1, m0, j, ldh, gred.as<double>(), act, H.as<cd>(), Hr.as<T>(),
                                accumulate);
          ApplyArgs ap{n,   m2,  m2,  ns,     j + 1,         j + 1, Vb, 2 * ldc, m2,      0,        blk,
                       Hr.p, (int64_t)(j + 1) * m2 * m2, t1, 2 * ldc, m2, -1.0, 1.0, act, nullptr};
          launch_apply<T, T>(st, ap);
        };
        cgs_pass(d_active, 0);
        const bool always = reorth_eta >= 1.0;
        if (always) {
          cgs_pass(d_active, 1);
          reorth_steps += ns;
        }
        // Gram of the projected block (its own buffer: a second pass reuses gred); it is the
        // first Cholesky-QR Gram of every shift that needs no second Gram-Schmidt pass
        GramArgs gw{n, m2, m2, ns, 1, t1, 2 * ldc, m2, 0, t1, 2 * ldc, m2, 0, d_active, gwb.as<double>()};
        launch_gram<T>(st, gw, gpart.p, gpart.bytes);
        launch_orth_check(st, ns, m0, j, ldh, always ? 0.0 : reorth_eta, always ? -1.0 : single_gersh, dead_thr,
                          gwb.as<double>(), d_active, H.as<cd>(), d_need, d_single, d_two);
        const std::vector<int> fl = d2h_ints(d_need, 3 * 64);
        const std::vector<int> need(fl.begin(), fl.begin() + ns), single(fl.begin() + 64, fl.begin() + 64 + ns),
            two(fl.begin() + 128, fl.begin() + 128 + ns);
        auto count = [](const std::vector<int>& v) { return (int)std::count_if(v.begin(), v.end(), [](int x) { return x != 0; }); };
        if (count(need) > 0) {
          note(d_need, need);
          cgs_pass(d_need, 1);
          GramArgs gn = gw;
          gn.active = d_need;
          launch_gram<T>(st, gn, gpart.p, gpart.bytes);
          reorth_steps += count(need);
        }
        // V_{j+1} H_{j+1,j} = qr(W): one unshifted Cholesky-QR pass where the Gram is certified
        // well conditioned, two passes (the first shifted) elsewhere
        T* dst = Vb + (int64_t)(j + 1) * blk;
        dbg(st, "W_cgs", t1, n * ldc * 2, cyc, j);
        if (count(single) > 0) {
          note(d_single, single);
          launch_cholqr_factor<T>(st, ns, m0, gwb.as<double>(), 0.0, d_single, Tinv.as<T>(), Racc.as<cd>(), 0,
                                  chol.as<cd>());
          ApplyArgs ap{n, m2, m2, ns, 1, 1, t1, 2 * ldc, m2, 0, 0, Tinv.p, (int64_t)m2 * m2, dst, 2 * ldc, m2,
                       1.0, 0.0, d_single, nullptr};
          launch_apply<T, T>(st, ap);
          single_steps += count(single);
        }
        if (count(two) > 0) {
          note(d_two, two);
          cholqr2<T>(t1, t2, dst, d_two, gwb.as<double>());
        }
        dbg(st, "V_j+1", Vb + (int64_t)(j + 1) * blk, n * ldc * 2, cyc, j);
        dbg(st, "Hsub", reinterpret_cast<double*>(Racc.p), (int64_t)ns * m0 * m0 * 2, cyc, j);
        launch_store_subdiag(st, ns, m0, j, ldh, d_active, Racc.as<cd>(), H.as<cd>());
        launch_lsq_step(st, la, j);
        dbg(st, "lsq_res", la.res, (int64_t)ns * m0, cyc, j);
        jdone = j + 1;
        const std::vector<int> act = d2h_ints(d_active, ns);
        note(d_active, act);
        if (std::none_of(act.begin(), act.end(), [](int a) { return a != 0; })) break;
      }
      launch_lsq_finish(st, la);
      dbg(st, "y", reinterpret_cast<double*>(y.p), (int64_t)ns * k * m0 * m0 * 2, cyc);
      dbg(st, "u", reinterpret_cast<double*>(u.p), (int64_t)ns * ldh * m0 * 2, cyc);
      launch_make_coefs<T>(st, la, wsD.as<double>(), jdone, Yq.as<T>(), Uc.as<T>(), 0);
      dbg(st, "Yq", Yq.as<T>(), (int64_t)ns * jdone * m2 * m0, cyc);
      // Q += Re sum_s V_s[0..jdone) Yq_s
      ApplyArgs aq{n,  m2, m0, 1, ns * jdone, jdone, Vb, 2 * ldc, 0, m2, blk, Yq.p, 0, Qd, m0, 0,
                   1.0, 1.0, nullptr, d_run, KC_QACC};
      launch_apply<T, double>(st, aq);
      dbg(st, "Q", Qd, n * m0, cyc);
      const std::vector<int> it = d2h_ints(d_iters, ns);
      const std::vector<int> cd_ = d2h_ints(d_cdone, ns);
      std::vector<int> cont(ns, 0);
      bool any = false;
      for (int s = 0; s < ns; ++s) {
        if (!run[s]) continue;
        total_iters[s] += it[s];
        cont[s] = (cd_[s] == 0 && cyc + 1 < p.max_cycles) ? 1 : 0;
        any = any || cont[s];
      }
      if (!any) break;
      // restart residual: T1_s = sum_b V_s[b] u_s[b], b = 0..jdone
      h2d(d_cont, cont.data(), ns * sizeof(int));
      note(d_cont, cont);
      ApplyArgs ar{n, m2, m2, ns, jdone + 1, jdone + 1, Vb, 2 * ldc, m2, 0, blk, Uc.p,
                   (int64_t)(jdone + 1) * m2 * m2, t1, 2 * ldc, m2, 1.0, 0.0, d_cont, nullptr};
      launch_apply<T, T>(st, ar);
      dbg(st, "restart", t1, n * ldc * 2, cyc);
      run = cont;
    }
    return total_iters;
  }
};

Engine::Engine(hipStream_t st, const Shape& shape) : shape_(shape), st_(st), impl_(new Impl(st, shape)) {}
Engine::~Engine() = default;

namespace {

// Stopping thresholds of the inner solves (ns x m0).  Per-column rule: alpha times the start
// residual of column j, ||r_j|| / |z_s - lambda_j|; for a conjugate pair in pair format the
// columns mix both eigenvalues, and the bound (1/|z - lambda| + 1/|z - conj(lambda)|) / 2 times
// the pair's residual is used for both.
std::vector<double> inner_tolerances(const Nodes& nd, const ifeast_params& p, const std::vector<double>& lam,
                                     const std::vector<double>& lam_im, const std::vector<double>& resid, double rf,
                                     int m0) {
  const int ns = (int)nd.z.size();
  std::vector<double> t((size_t)ns * m0 * 2, 0.0);
  for (int s = 0; s < ns; ++s)
    for (int j = 0; j < m0; ++j) {
      double v;
      if (p.inner_rule == IFEAST_INNER_GLOBAL) {
        v = p.alpha * rf;
      } else if (lam_im[j] == 0.0) {
        v = p.alpha * resid[j] / std::abs(nd.z[s] - lam[j]);
      } else {
        const cd l(lam[j], std::fabs(lam_im[j]));
        v = p.alpha * resid[j] * 0.5 * (1.0 / std::abs(nd.z[s] - l) + 1.0 / std::abs(nd.z[s] - std::conj(l)));
      }
      t[(size_t)s * m0 + j] = v;
    }
  return t;
}

// Nodes of a conjugate-symmetric rule in the upper half plane, summed as 2 Re.
Nodes upper_half(const Nodes& nd) {
  Nodes u;
  u.half = true;
  for (size_t k = 0; k < nd.z.size(); ++k)
    if (nd.z[k].imag() > 0.0) {
      u.z.push_back(nd.z[k]);
      u.w.push_back(nd.w[k]);
    }
  return u;
}

ClassifyArgs classify_args(const ifeast_contour& C, const Nodes& nd, int m0, double tau, const double* zd,
                           const double* wd) {
  ClassifyArgs a;
  a.m0 = m0;
  a.nc = (int)nd.z.size();
  a.half = nd.half ? 1 : 0;
  a.kind = C.kind;
  a.emin = C.emin;
  a.emax = C.emax;
  a.c_re = C.c_re;
  a.c_im = C.c_im;
  a.r = C.r;
  a.tau = tau;
  a.z = zd;
  a.w = wd;
  return a;
}

__global__ void k_rho(int m0, int nc, int half, const double* __restrict__ z, const double* __restrict__ w,
                      const double* __restrict__ lam, double* __restrict__ rho) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m0) return;
  double rr = 0.0, ri = 0.0;
  const double l = lam[j];
  for (int k = 0; k < nc; ++k) {
    const double zr = z[2 * k] - l, zi = z[2 * k + 1];
    const double d = zr * zr + zi * zi;
    rr += (w[2 * k] * zr + w[2 * k + 1] * zi) / d;
    ri += (w[2 * k + 1] * zr - w[2 * k] * zi) / d;
  }
  rho[j] = half ? 2.0 * rr : rr;
}

}  // namespace

void Engine::rayleigh_ritz(const ifeast_matrix* A, const ifeast_matrix* B, const double* Q, double* lam, double* X,
                           double* R, double* resid, double* eta) {
  impl_->rr(A, B, Q, X, lam, R, resid, eta);
}

void Engine::rayleigh_ritz_general(const ifeast_matrix* A, const double* Q, const double* Xprev, double* lam,
                                   double* lam_im, double* X, double* R, double* resid, double* eta) {
  impl_->rr_general(A, Q, Xprev, X, lam, lam_im, R, resid, eta);
}

void Engine::filter(const ifeast_matrix* A, const ifeast_matrix* B, const ifeast_contour& C, const ifeast_params& p,
                    const double* X, const double* lam, const double* R, double rf, double* Q,
                    std::vector<int>* iters) {
  Impl& I = *impl_;
  const int m0 = shape_.m0;
  const Nodes nd = make_nodes(C);
  std::vector<double> zd(2 * nd.z.size()), wd(2 * nd.z.size());
  for (size_t s = 0; s < nd.z.size(); ++s) {
    zd[2 * s] = nd.z[s].real();
    zd[2 * s + 1] = nd.z[s].imag();
    wd[2 * s] = nd.w[s].real();
    wd[2 * s + 1] = nd.w[s].imag();
  }
  DevBuf zb(zd.size() * 8), wb(wd.size() * 8);
  I.h2d(zb.p, zd.data(), zd.size() * 8);
  I.h2d(wb.p, wd.data(), wd.size() * 8);
  hipLaunchKernelGGL(k_rho, dim3(1), dim3(128), 0, st_, m0, (int)nd.z.size(), nd.half ? 1 : 0, zb.as<double>(),
                     wb.as<double>(), lam, I.rho.as<double>());
  IF_HIP(hipGetLastError());
  std::vector<double> lamh(m0), residh(m0);
  IF_HIP(hipMemcpyAsync(lamh.data(), lam, m0 * 8, hipMemcpyDeviceToHost, st_));
  launch_col_sumsq(st_, shape_.n, m0, R, I.resid.as<double>(), I.colpart.as<double>());
  IF_HIP(hipMemcpyAsync(residh.data(), I.resid.p, m0 * 8, hipMemcpyDeviceToHost, st_));
  IF_HIP(hipStreamSynchronize(st_));
  IF_REQUIRE(!shape_.general, "the step-level filter takes symmetric problems");
  const std::vector<double> tolh = inner_tolerances(nd, p, lamh, std::vector<double>(m0, 0.0), residh, rf, m0);
  std::vector<int> it;
  if (shape_.minres)
    it = shape_.precision == IFEAST_PREC_MIXED
             ? I.inner_minres<float>(A, nd, p, X, lam, R, I.rho.as<double>(), tolh, Q)
             : I.inner_minres<double>(A, nd, p, X, lam, R, I.rho.as<double>(), tolh, Q);
  else if (shape_.shared)
    it = shape_.precision == IFEAST_PREC_MIXED
             ? I.inner_shared<float>(A, nd, p, X, lam, R, I.rho.as<double>(), tolh, Q)
             : I.inner_shared<double>(A, nd, p, X, lam, R, I.rho.as<double>(), tolh, Q);
  else
    it = shape_.precision == IFEAST_PREC_MIXED
             ? I.inner<float>(A, B, nd, p, X, lam, R, I.rho.as<double>(), tolh, Q)
             : I.inner<double>(A, B, nd, p, X, lam, R, I.rho.as<double>(), tolh, Q);
  IF_HIP(hipStreamSynchronize(st_));
  if (iters) *iters = it;
}

int Engine::solve(const ifeast_matrix* A, const ifeast_matrix* B, const ifeast_contour& C, const ifeast_params& p,
                  const double* X0_in, ifeast_result* res, bool x0_on_device, double* evec_dev) {
  Impl& I = *impl_;
  const int64_t n = shape_.n;
  const int m0 = shape_.m0;
  const bool gen = shape_.general;
  // nd: the whole rule (the filter rho_hat and membership); nd_in: the systems solved.  For a
  // non-Hermitian problem on a circle centred on the real axis these are the nodes in the upper
  // half with 2 Re of their sum (the lower half's solutions are the conjugates: A, X and R are real)
  const Nodes nd = make_nodes(C);
  const Nodes nd_in = gen ? upper_half(nd) : nd;
  const int ncl = (int)nd.z.size();
  IF_REQUIRE((int)nd_in.z.size() == shape_.ns, "contour and workspace shape differ");
  std::vector<double> zd(2 * ncl), wd(2 * ncl);
  for (int s = 0; s < ncl; ++s) {
    zd[2 * s] = nd.z[s].real();
    zd[2 * s + 1] = nd.z[s].imag();
    wd[2 * s] = nd.w[s].real();
    wd[2 * s + 1] = nd.w[s].imag();
  }
  DevBuf zb(zd.size() * 8), wb(wd.size() * 8), outh(16);
  I.h2d(zb.p, zd.data(), zd.size() * 8);
  I.h2d(wb.p, wd.data(), wd.size() * 8);
  // initial block
  if (x0_on_device) {
    IF_HIP(hipMemcpyAsync(I.Q.p, X0_in, (size_t)n * m0 * 8, hipMemcpyDeviceToDevice, st_));
  } else {
    std::vector<double> x0;
    const double* X0_host = X0_in;
    if (X0_host == nullptr) {
      std::mt19937_64 gen(p.seed);
      std::normal_distribution<double> nrm(0.0, 1.0);
      x0.resize((size_t)n * m0);
      for (auto& v : x0) v = nrm(gen);
      X0_host = x0.data();
    }
    I.h2d(I.Q.p, X0_host, (size_t)n * m0 * 8);
  }

  hipEvent_t e0, e1;
  IF_HIP(hipEventCreate(&e0));
  IF_HIP(hipEventCreate(&e1));
  IF_HIP(hipEventRecord(e0, st_));

  double* X = I.X.as<double>();
  double* Q = I.Q.as<double>();
  double* lam = I.lam.as<double>();
  double* resid = I.resid.as<double>();
  double* eta = I.eta.as<double>();
  double* R = I.R.as<double>();
  SolveStats stats;
  double* lamI = I.lamI.as<double>();
  std::vector<double> lamh(m0), lamIh(m0, 0.0), residh(m0), cls(3);
  int geo_count = 0;  // Ritz values inside the contour, counted or not
  std::vector<int> flagh(m0);

  auto classify = [&](double tau) {
    const ClassifyArgs ca = classify_args(C, nd, m0, tau, zb.as<double>(), wb.as<double>());
    launch_classify(st_, ca, lam, gen ? lamI : nullptr, resid, eta, I.d_cls, I.clsout.as<double>());
    if (gen) {
      launch_rho_pairs(st_, m0, ncl, zb.as<double>(), wb.as<double>(), lam, lamI, I.rho.as<double>(),
                       I.rhoI.as<double>());
      IF_HIP(hipMemcpyAsync(lamIh.data(), lamI, m0 * 8, hipMemcpyDeviceToHost, st_));
    } else {
      hipLaunchKernelGGL(k_rho, dim3(1), dim3(128), 0, st_, m0, ncl, nd.half ? 1 : 0, zb.as<double>(),
                         wb.as<double>(), lam, I.rho.as<double>());
      IF_HIP(hipGetLastError());
    }
    IF_HIP(hipMemcpyAsync(cls.data(), I.clsout.p, 24, hipMemcpyDeviceToHost, st_));
    IF_HIP(hipMemcpyAsync(lamh.data(), lam, m0 * 8, hipMemcpyDeviceToHost, st_));
    IF_HIP(hipMemcpyAsync(residh.data(), resid, m0 * 8, hipMemcpyDeviceToHost, st_));
    IF_HIP(hipMemcpyAsync(flagh.data(), I.d_cls, m0 * 4, hipMemcpyDeviceToHost, st_));
    IF_HIP(hipStreamSynchronize(st_));
    for (int j = 0; j < m0; ++j)
      if (!std::isfinite(lamh[j]) || !std::isfinite(residh[j]))
        throw Error{IFEAST_ERR_NUMERICAL, "non-finite Ritz value or residual"};
    stats.rf = cls[0];
    stats.m = (int)cls[1];
    geo_count = (int)cls[2];
  };

  const char* vb = getenv("IFEAST_VERBOSE");
  const bool verbose = vb && (vb[0] == '1' || vb[0] == '2');
  const bool verbose2 = vb && vb[0] == '2';
  // initial Rayleigh-Ritz on X0 gives Lambda, R and the exact initial ||R_F||
  if (gen)
    I.rr_general(A, Q, nullptr, X, lam, lamI, R, resid, eta);
  else
    I.rr(A, B, Q, X, lam, R, resid, eta);
  classify(0.0);
  if (verbose) fprintf(stderr, "[ifeast] start rf=%.3e m=%d\n", stats.rf, stats.m);
  int status = IFEAST_WARN_NOT_CONVERGED;
  for (int it = 0; it < p.max_outer; ++it) {
    const std::vector<double> tolh = inner_tolerances(nd_in, p, lamh, lamIh, residh, stats.rf, m0);
    std::vector<int> iters;
    const double* lamId = gen ? lamI : nullptr;
    const double* rhoId = gen ? I.rhoI.as<double>() : nullptr;
    if (shape_.minres)
      iters = shape_.precision == IFEAST_PREC_MIXED
                  ? I.inner_minres<float>(A, nd_in, p, X, lam, R, I.rho.as<double>(), tolh, Q)
                  : I.inner_minres<double>(A, nd_in, p, X, lam, R, I.rho.as<double>(), tolh, Q);
    else if (shape_.shared)
      iters = shape_.precision == IFEAST_PREC_MIXED
                  ? I.inner_shared<float>(A, nd_in, p, X, lam, R, I.rho.as<double>(), tolh, Q, lamId, rhoId)
                  : I.inner_shared<double>(A, nd_in, p, X, lam, R, I.rho.as<double>(), tolh, Q, lamId, rhoId);
    else
      iters = shape_.precision == IFEAST_PREC_MIXED
                  ? I.inner<float>(A, B, nd_in, p, X, lam, R, I.rho.as<double>(), tolh, Q)
                  : I.inner<double>(A, B, nd_in, p, X, lam, R, I.rho.as<double>(), tolh, Q);
    if (gen)
      I.rr_general(A, Q, X, X, lam, lamI, R, resid, eta);
    else
      I.rr(A, B, Q, X, lam, R, resid, eta);
    classify(p.spurious_tau);
    stats.outer = it + 1;
    stats.rf_hist.push_back(stats.rf);
    // matrix-vector products: one real block of m0 columns per shared Arnoldi step, or one
    // complex block per shift and step
    int mx = 0;
    for (int s = 0; s < shape_.ns; ++s) {
      stats.inner_hist.push_back(iters[s]);
      if (!shape_.shared && !shape_.minres) stats.total_matvec += (int64_t)iters[s] * m0;
      mx = std::max(mx, iters[s]);
    }
    if (shape_.shared || shape_.minres) {
      stats.total_matvec += (int64_t)I.shared_steps * m0;
      mx = I.shared_steps;
    }
    stats.seq_matvec += mx;
    if (verbose) {
      float ms_now = 0.f;
      hipEvent_t en;
      if (hipEventCreate(&en) == hipSuccess) {
        (void)hipEventRecord(en, st_);
        (void)hipEventSynchronize(en);
        (void)hipEventElapsedTime(&ms_now, e0, en);
        (void)hipEventDestroy(en);
      }
      fprintf(stderr,
              "[ifeast] outer %d rf=%.3e m=%d max_inner=%d reorth=%lld local2=%lld single=%lld loss=%.1e t=%.2fs\n",
              it + 1, stats.rf, stats.m, mx, (long long)I.reorth_steps, (long long)I.local_second,
              (long long)I.single_steps, I.max_loss, ms_now * 1e-3);
      if (verbose2) {
        std::vector<double> etah(m0), rhoh(m0);
        IF_HIP(hipMemcpyAsync(etah.data(), eta, m0 * 8, hipMemcpyDeviceToHost, st_));
        IF_HIP(hipMemcpyAsync(rhoh.data(), I.rho.p, m0 * 8, hipMemcpyDeviceToHost, st_));
        IF_HIP(hipStreamSynchronize(st_));
        const double w = 0.1 * (C.emax - C.emin);
        for (int j = 0; j < m0; ++j)
          if (lamh[j] > C.emin - w && lamh[j] < C.emax + w)
            fprintf(stderr, "   pair %2d lam=%.8f r=%.2e eta/rho=%.3f flags=%d\n", j, lamh[j], residh[j],
                    etah[j] / std::max(1e-300, std::fabs(rhoh[j])), flagh[j]);
      }
      fflush(stderr);
    }
    if (stats.m > 0 && stats.rf <= p.tol) {
      stats.converged = 1;
      status = stats.m >= m0 ? IFEAST_WARN_M0_TOO_SMALL : IFEAST_OK;
      break;
    }
    // the premise of Algorithm 2 ("Start with"): fewer than m0 eigenvalues inside the contour
    // and at least one.  After a filter application, every Ritz value inside means the subspace
    // has no room for the eigenvalues outside; none inside means the contour holds none
    if (geo_count >= m0) {
      status = IFEAST_WARN_M0_TOO_SMALL;
      break;
    }
    if (geo_count == 0) {
      status = IFEAST_WARN_NO_EIG_IN_CONTOUR;
      break;
    }
  }
  IF_HIP(hipEventRecord(e1, st_));
  IF_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  IF_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  stats.seconds = ms * 1e-3;

  // outputs: counted pairs first (ascending), then the rest (ascending)
  std::vector<int> order;
  for (int j = 0; j < m0; ++j)
    if (flagh[j] & IFEAST_FLAG_INSIDE) order.push_back(j);
  for (int j = 0; j < m0; ++j)
    if (!(flagh[j] & IFEAST_FLAG_INSIDE)) order.push_back(j);
  res->m = stats.m;
  res->outer_iters = stats.outer;
  res->converged = stats.converged;
  res->total_matvec = stats.total_matvec;
  res->seq_matvec = stats.seq_matvec;
  res->max_resid = stats.rf;
  res->solve_seconds = stats.seconds;
  for (int j = 0; j < m0; ++j) {
    if (res->eval_re) res->eval_re[j] = lamh[order[j]];
    if (res->eval_im) res->eval_im[j] = lamIh[order[j]];
    if (res->resid) res->resid[j] = residh[order[j]];
    if (res->flags) res->flags[j] = flagh[order[j]];
  }
  if (res->rf_hist)
    for (size_t i = 0; i < stats.rf_hist.size(); ++i) res->rf_hist[i] = stats.rf_hist[i];
  if (res->inner_hist)
    for (size_t i = 0; i < stats.inner_hist.size(); ++i) res->inner_hist[i] = stats.inner_hist[i];
  if (evec_dev) {
    DevBuf ob(m0 * sizeof(int));
    I.h2d(ob.p, order.data(), m0 * sizeof(int));
    const int64_t tot = n * m0;
    if (gen)
      hipLaunchKernelGGL(k_gather_complex, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st_, n, m0, X,
                         ob.as<int>(), lamI, evec_dev);
    else
      hipLaunchKernelGGL(k_gather_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st_, n, m0, X,
                         ob.as<int>(), evec_dev);
    IF_HIP(hipGetLastError());
    IF_HIP(hipStreamSynchronize(st_));
  }
  if (res->evec) {
    std::vector<double> xh((size_t)n * m0);
    IF_HIP(hipMemcpyAsync(xh.data(), X, xh.size() * 8, hipMemcpyDeviceToHost, st_));
    IF_HIP(hipStreamSynchronize(st_));
    if (gen) {
      // complex eigenvectors, interleaved: a pair's columns hold Re x and Im x of a + ib
      for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < m0; ++j) {
          const int o = order[j];
          const double* row = xh.data() + i * m0;
          double re = row[o], im = 0.0;
          if (lamIh[o] < 0.0) im = -row[o + 1];
          else if (lamIh[o] > 0.0) re = row[o - 1], im = row[o];
          res->evec[2 * (i * m0 + j)] = re;
          res->evec[2 * (i * m0 + j) + 1] = im;
        }
    } else {
      for (int64_t i = 0; i < n; ++i)
        for (int j = 0; j < m0; ++j) res->evec[i * m0 + j] = xh[i * m0 + order[j]];
    }
  }
  return status;
}

}  // namespace ifeast
