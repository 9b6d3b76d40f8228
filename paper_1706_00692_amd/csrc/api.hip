// C ABI of libifeast (see include/ifeast.h).  Every entry point converts
// engine errors into status codes and records the message on the context.
#include <chrono>
#include <cmath>
#include <cstring>

#include "engine.h"
#include "serve.h"

using namespace ifeast;

namespace {

thread_local std::string g_noctx_error;

int fail(ifeast_ctx* ctx, int status, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  else g_noctx_error = msg;
  return status;
}

template <class F>
int guarded(ifeast_ctx* ctx, F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(ctx, e.status, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(ctx, IFEAST_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ctx, IFEAST_ERR_DEVICE, e.what());
  }
}

struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&prev);
    if (prev != dev) IF_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

// Installs a kernel timer for the calling thread while a compute call runs on a
// context with timing on, then folds its totals into the context (caller holds ctx->mu).
struct TimingScope {
  ifeast_ctx* ctx;
  std::unique_ptr<KernelTimer> t;
  explicit TimingScope(ifeast_ctx* c) : ctx(c) {
    if (ctx->timing) {
      t.reset(new KernelTimer());
      current_timer() = t.get();
    }
  }
  ~TimingScope() {
    if (!t) return;
    current_timer() = nullptr;
    try {
      t->flush();
    } catch (...) {
      return;  // a device error is reported by the call itself
    }
    for (int k = 0; k < KC_N; ++k) {
      ctx->kstats[k].launches += t->acc[k].launches;
      ctx->kstats[k].seconds += t->acc[k].seconds;
      ctx->kstats[k].flops += t->acc[k].flops;
      ctx->kstats[k].bytes += t->acc[k].bytes;
    }
  }
};

void check_csr(const ifeast_csr* M) {
  IF_REQUIRE(M != nullptr && M->rowptr != nullptr && M->colind != nullptr && M->val != nullptr, "null CSR pointer");
  IF_REQUIRE(M->n > 0 && M->n < (int64_t(1) << 31), "n must be in [1, 2^31)");
  IF_REQUIRE(M->nnz >= 0 && M->nnz < (int64_t(1) << 31), "nnz must be < 2^31");
  IF_REQUIRE(M->rowptr[0] == 0 && M->rowptr[M->n] == M->nnz, "rowptr must start at 0 and end at nnz");
  for (int64_t i = 0; i < M->n; ++i) {
    const int64_t a = M->rowptr[i], b = M->rowptr[i + 1];
    IF_REQUIRE(a <= b, "rowptr must be non-decreasing");
    for (int64_t e = a; e < b; ++e) {
      const int32_t c = M->colind[e];
      IF_REQUIRE(c >= 0 && c < M->n, "column index out of range");
      IF_REQUIRE(e == a || M->colind[e - 1] < c, "column indices must be sorted and unique within a row");
      IF_REQUIRE(std::isfinite(M->val[e]), "non-finite matrix value");
    }
  }
}

int nsys(const ifeast_contour* C) { return C->nc; }

Shape make_shape(int64_t n, bool hasB, const ifeast_contour* C, const ifeast_params* p) {
  Shape s;
  s.n = n;
  s.m0 = p->m0;
  s.ns = nsys(C);
  s.k = p->max_inner;
  s.hasB = hasB;
  s.precision = p->precision;
  if ((p->basis == IFEAST_BASIS_SHARED || p->basis == IFEAST_BASIS_MINRES) && hasB)
    throw Error{IFEAST_ERR_UNSUPPORTED, "a shared Krylov basis or MINRES inner solves need B = I"};
  s.minres = p->basis == IFEAST_BASIS_MINRES;
  s.shared = !hasB && p->basis != IFEAST_BASIS_PER_SHIFT && !s.minres;
  if (p->problem == IFEAST_PROBLEM_GENERAL) {
    if (hasB) throw Error{IFEAST_ERR_UNSUPPORTED, "non-Hermitian problems take B = I"};
    // the upper half of a conjugate-symmetric rule is solved (see validate_params)
    s.general = true;
    s.ns = nsys(C) / 2;
  }
  s.kb = (s.shared || s.minres) ? p->max_inner * p->max_cycles : p->max_inner;
  return s;
}

// Reuse the context's engine when the shape matches (same workspace).
Engine& engine_for(ifeast_ctx* ctx, const Shape& s);

}  // namespace

struct EngineCache {
  std::unique_ptr<Engine> eng;
};
static std::mutex g_cache_mu;
static std::map<ifeast_ctx*, EngineCache> g_cache;

namespace {
bool same(const Shape& a, const Shape& b) {
  return a.n == b.n && a.m0 == b.m0 && a.ns == b.ns && a.k == b.k && a.hasB == b.hasB && a.precision == b.precision &&
         a.shared == b.shared && a.kb == b.kb && a.general == b.general && a.minres == b.minres;
}
Engine& engine_for(ifeast_ctx* ctx, const Shape& s) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  EngineCache& c = g_cache[ctx];
  if (!c.eng || !same(c.eng->shape(), s) || c.eng->stream() != ctx->stream) {
    c.eng.reset();
    c.eng.reset(new Engine(ctx->stream, s));
  }
  return *c.eng;
}
void drop_engine(ifeast_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_cache.erase(ctx);
}
}  // namespace

namespace ifeast {
void release_engine(ifeast_ctx* ctx) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard g(ctx->device);
  drop_engine(ctx);
}
}  // namespace ifeast

extern "C" {

const char* ifeast_version(void) { return "libifeast 0.1 (gfx950)"; }

const char* ifeast_status_str(int s) {
  switch (s) {
    case IFEAST_OK: return "ok";
    case IFEAST_WARN_NOT_CONVERGED: return "warning: not converged within max_outer";
    case IFEAST_WARN_M0_TOO_SMALL: return "warning: m0 too small for the eigenvalues inside the contour";
    case IFEAST_WARN_NO_EIG_IN_CONTOUR: return "warning: no eigenvalue inside the contour";
    case IFEAST_ERR_INVALID_ARG: return "error: invalid argument";
    case IFEAST_ERR_OOM: return "error: out of device memory";
    case IFEAST_ERR_DEVICE: return "error: device failure";
    case IFEAST_ERR_NUMERICAL: return "error: non-finite values in the iteration";
    case IFEAST_ERR_REJECTED: return "error: request exceeds the HBM budget";
    case IFEAST_ERR_UNKNOWN_TICKET: return "error: unknown ticket";
    case IFEAST_ERR_UNSUPPORTED: return "error: unsupported option";
    default: return "unknown status";
  }
}

const char* ifeast_last_error(ifeast_ctx* ctx) { return ctx ? ctx->last_error.c_str() : g_noctx_error.c_str(); }

int ifeast_create(ifeast_ctx** out, int device, uint64_t budget) {
  return guarded(nullptr, [&]() -> int {
    IF_REQUIRE(out != nullptr, "null context pointer");
    int count = 0;
    IF_HIP(hipGetDeviceCount(&count));
    IF_REQUIRE(device >= 0 && device < count, "no such HIP device");
    std::unique_ptr<ifeast_ctx> ctx(new ifeast_ctx);
    ctx->device = device;
    DeviceGuard g(device);
    IF_HIP(hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking));
    ctx->stream = ctx->own_stream;
    size_t fr = 0, tot = 0;
    IF_HIP(hipMemGetInfo(&fr, &tot));
    ctx->budget = budget ? budget : (uint64_t)(0.9 * (double)fr);
    // the allocation-free entry point's scratch address on this device (looked up once)
    (void)noalloc_scratch(device);
    *out = ctx.release();
    return IFEAST_OK;
  });
}

int ifeast_destroy(ifeast_ctx* ctx) {
  if (!ctx) return IFEAST_OK;
  return guarded(nullptr, [&]() -> int {
    ctx->server.reset();
    drop_engine(ctx);
    {
      DeviceGuard g(ctx->device);
      if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
    }
    delete ctx;
    return IFEAST_OK;
  });
}

int ifeast_set_stream(ifeast_ctx* ctx, void* stream) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr, "null context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stream = static_cast<hipStream_t>(stream);
    return IFEAST_OK;
  });
}

int ifeast_matrix_create(ifeast_ctx* ctx, const ifeast_csr* A, ifeast_matrix** out) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && out != nullptr, "null argument");
    check_csr(A);
    DeviceGuard g(ctx->device);
    std::unique_ptr<ifeast_matrix> M(new ifeast_matrix);
    M->n = A->n;
    M->nnz = A->nnz;
    M->device = ctx->device;
    std::vector<int32_t> rp(A->n + 1);
    for (int64_t i = 0; i <= A->n; ++i) rp[i] = (int32_t)A->rowptr[i];
    std::vector<float> vf(A->nnz);
    std::vector<double> colsum(A->n, 0.0);
    for (int64_t e = 0; e < A->nnz; ++e) {
      vf[e] = (float)A->val[e];
      colsum[A->colind[e]] += std::fabs(A->val[e]);
    }
    for (double c : colsum) M->norm1 = std::max(M->norm1, c);
    M->rowptr = DevBuf((A->n + 1) * 4);
    M->colind = DevBuf(std::max<int64_t>(1, A->nnz) * 4);
    M->val = DevBuf(std::max<int64_t>(1, A->nnz) * 8);
    M->valf = DevBuf(std::max<int64_t>(1, A->nnz) * 4);
    hipStream_t st = ctx->stream;
    IF_HIP(hipMemcpyAsync(M->rowptr.p, rp.data(), rp.size() * 4, hipMemcpyHostToDevice, st));
    IF_HIP(hipMemcpyAsync(M->colind.p, A->colind, A->nnz * 4, hipMemcpyHostToDevice, st));
    IF_HIP(hipMemcpyAsync(M->val.p, A->val, A->nnz * 8, hipMemcpyHostToDevice, st));
    IF_HIP(hipMemcpyAsync(M->valf.p, vf.data(), A->nnz * 4, hipMemcpyHostToDevice, st));
    IF_HIP(hipStreamSynchronize(st));
    *out = M.release();
    return IFEAST_OK;
  });
}

int ifeast_matrix_destroy(ifeast_ctx* ctx, ifeast_matrix* M) {
  if (!M) return IFEAST_OK;
  return guarded(ctx, [&]() -> int {
    DeviceGuard g(M->device);
    delete M;
    return IFEAST_OK;
  });
}

int64_t ifeast_matrix_n(const ifeast_matrix* M) { return M ? M->n : 0; }

int ifeast_footprint(int64_t n, int64_t nnzA, int64_t nnzB, const ifeast_contour* C, const ifeast_params* p,
                     uint64_t* bytes) {
  return guarded(nullptr, [&]() -> int {
    IF_REQUIRE(C != nullptr && p != nullptr && bytes != nullptr, "null argument");
    validate_params(*p, *C, n);
    const Shape s = make_shape(n, nnzB > 0, C, p);
    const uint64_t mats = (uint64_t)(n + 1) * 4 * 2 + (uint64_t)(nnzA + nnzB) * (4 + 8 + 4);
    *bytes = workspace_bytes(s) + mats;
    return IFEAST_OK;
  });
}

int ifeast_solve_resident(ifeast_ctx* ctx, const ifeast_matrix* A, const ifeast_matrix* B, const ifeast_contour* C,
                          const ifeast_params* p, const double* X0, ifeast_result* res) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && A != nullptr && C != nullptr && p != nullptr && res != nullptr, "null argument");
    IF_REQUIRE(B == nullptr || B->n == A->n, "A and B sizes differ");
    validate_params(*p, *C, A->n);
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    Engine& eng = engine_for(ctx, make_shape(A->n, B != nullptr, C, p));
    TimingScope ts(ctx);
    return eng.solve(A, B, *C, *p, X0, res);
  });
}

int ifeast_solve_dev(ifeast_ctx* ctx, const ifeast_matrix* A, const ifeast_matrix* B, const ifeast_contour* C,
                     const ifeast_params* p, const double* X0, double* evec, ifeast_result* res) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && A != nullptr && C != nullptr && p != nullptr && res != nullptr && X0 != nullptr,
               "null argument");
    IF_REQUIRE(B == nullptr || B->n == A->n, "A and B sizes differ");
    validate_params(*p, *C, A->n);
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    Engine& eng = engine_for(ctx, make_shape(A->n, B != nullptr, C, p));
    TimingScope ts(ctx);
    return eng.solve(A, B, *C, *p, X0, res, true, evec);
  });
}

int ifeast_solve(ifeast_ctx* ctx, const ifeast_csr* A, const ifeast_csr* B, const ifeast_contour* C,
                 const ifeast_params* p, const double* X0, ifeast_result* res) {
  ifeast_matrix* Am = nullptr;
  ifeast_matrix* Bm = nullptr;
  int st = ifeast_matrix_create(ctx, A, &Am);
  if (st != IFEAST_OK) return st;
  if (B != nullptr) {
    st = ifeast_matrix_create(ctx, B, &Bm);
    if (st != IFEAST_OK) {
      ifeast_matrix_destroy(ctx, Am);
      return st;
    }
  }
  st = ifeast_solve_resident(ctx, Am, Bm, C, p, X0, res);
  ifeast_matrix_destroy(ctx, Bm);
  ifeast_matrix_destroy(ctx, Am);
  return st;
}

int ifeast_set_timing(ifeast_ctx* ctx, int enable) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr, "null context");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->timing = enable != 0;
    for (auto& k : ctx->kstats) k = KernelStat{};
    return IFEAST_OK;
  });
}

int ifeast_kernel_stats(ifeast_ctx* ctx, int kind, ifeast_kernel_stat* out) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && out != nullptr, "null argument");
    IF_REQUIRE(kind >= 0 && kind < KC_N, "unknown kernel class");
    std::lock_guard<std::mutex> lk(ctx->mu);
    const KernelStat& k = ctx->kstats[kind];
    out->launches = k.launches;
    out->seconds = k.seconds;
    out->flops = k.flops;
    out->bytes = k.bytes;
    return IFEAST_OK;
  });
}

int ifeast_spmm_shifted_dev(ifeast_ctx* ctx, const ifeast_matrix* A, const ifeast_matrix* B, int precision, int ns,
                            const double* z, int m0, const void* V, void* W) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && A != nullptr && z != nullptr && V != nullptr && W != nullptr, "null argument");
    IF_REQUIRE(B == nullptr || B->n == A->n, "A and B sizes differ");
    IF_REQUIRE(ns >= 1 && ns <= 64 && m0 >= 2 && m0 % 2 == 0, "ns in [1, 64] and even m0 required");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    TimingScope ts(ctx);
    hipStream_t st = ctx->stream;
    // the shifts go to a buffer the context keeps, in stream order: consecutive calls queue
    // without host synchronisation or allocation
    if (ctx->zbuf.p == nullptr) ctx->zbuf = DevBuf(64 * 2 * sizeof(double));
    if (precision == IFEAST_PREC_MIXED) {
      std::vector<float> zf(2 * ns);
      for (int i = 0; i < 2 * ns; ++i) zf[i] = (float)z[i];
      IF_HIP(hipMemcpyAsync(ctx->zbuf.p, zf.data(), zf.size() * 4, hipMemcpyHostToDevice, st));
      launch_spmm_shifted<float>(st, A, B, ns, m0, ctx->zbuf.as<float>(), nullptr, static_cast<const float*>(V),
                                 static_cast<float*>(W));
    } else {
      IF_REQUIRE(precision == IFEAST_PREC_FP64, "unknown precision");
      IF_HIP(hipMemcpyAsync(ctx->zbuf.p, z, 2 * ns * 8, hipMemcpyHostToDevice, st));
      launch_spmm_shifted<double>(st, A, B, ns, m0, ctx->zbuf.as<double>(), nullptr, static_cast<const double*>(V),
                                  static_cast<double*>(W));
    }
    return IFEAST_OK;
  });
}

int ifeast_filter_dev(ifeast_ctx* ctx, const ifeast_matrix* A, const ifeast_matrix* B, const ifeast_contour* C,
                      const ifeast_params* p, const double* X, const double* lam, const double* R, double rf,
                      double* Q, int32_t* inner_iters) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && A != nullptr && C != nullptr && p != nullptr, "null argument");
    IF_REQUIRE(X != nullptr && lam != nullptr && R != nullptr && Q != nullptr, "null device pointer");
    IF_REQUIRE(B == nullptr || B->n == A->n, "A and B sizes differ");
    validate_params(*p, *C, A->n);
    if (p->problem != IFEAST_PROBLEM_SYMMETRIC)
      throw Error{IFEAST_ERR_UNSUPPORTED, "the step-level filter takes symmetric problems"};
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    Engine& eng = engine_for(ctx, make_shape(A->n, B != nullptr, C, p));
    TimingScope ts(ctx);
    std::vector<int> it;
    eng.filter(A, B, *C, *p, X, lam, R, rf, Q, &it);
    if (inner_iters)
      for (size_t i = 0; i < it.size(); ++i) inner_iters[i] = it[i];
    return IFEAST_OK;
  });
}

int ifeast_rayleigh_ritz_dev(ifeast_ctx* ctx, const ifeast_matrix* A, const ifeast_matrix* B, int m0,
                             const double* Q, double* lam, double* X, double* R, double* resid, double* eta) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && A != nullptr, "null argument");
    IF_REQUIRE(Q && lam && X && R && resid && eta, "null device pointer");
    IF_REQUIRE(m0 > 0 && m0 % 16 == 0 && m0 <= 128 && m0 <= A->n, "m0 must be a multiple of 16 in [16, 128]");
    IF_REQUIRE(B == nullptr || B->n == A->n, "A and B sizes differ");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    ifeast_contour C{};
    C.kind = IFEAST_CONTOUR_HALF;
    C.nc = 1;
    C.emin = 0.0;
    C.emax = 1.0;
    ifeast_params p{};
    p.m0 = m0;
    p.max_inner = 1;
    p.precision = IFEAST_PREC_FP64;
    Engine& eng = engine_for(ctx, make_shape(A->n, B != nullptr, &C, &p));
    TimingScope ts(ctx);
    eng.rayleigh_ritz(A, B, Q, lam, X, R, resid, eta);
    IF_HIP(hipStreamSynchronize(ctx->stream));
    return IFEAST_OK;
  });
}

int ifeast_rayleigh_ritz_dev_noalloc(ifeast_ctx* ctx, const ifeast_matrix* A, const ifeast_matrix* B, int m0,
                                     const double* Q, double* lam, double* X, double* R, double* resid, double* eta) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && A != nullptr, "null argument");
    IF_REQUIRE(Q && lam && X && R && resid && eta, "null device pointer");
    IF_REQUIRE(Q != X, "Q and X must not alias");
    IF_REQUIRE(m0 > 0 && m0 % 16 == 0 && m0 <= 128 && m0 <= A->n, "m0 must be a multiple of 16 in [16, 128]");
    IF_REQUIRE(B == nullptr || B->n == A->n, "A and B sizes differ");
    IF_REQUIRE(A->device == ctx->device && (B == nullptr || B->device == ctx->device),
               "matrices live on another device");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    rayleigh_ritz_noalloc(ctx->stream, ctx->device, A, B, m0, Q, lam, X, R, resid, eta);
    IF_HIP(hipStreamSynchronize(ctx->stream));
    return IFEAST_OK;
  });
}

int ifeast_rayleigh_ritz_general_dev(ifeast_ctx* ctx, const ifeast_matrix* A, int m0, const double* Q,
                                     const double* Xprev, double* lam, double* lam_im, double* X, double* R,
                                     double* resid, double* eta) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && A != nullptr, "null argument");
    IF_REQUIRE(Q && lam && lam_im && X && R && resid && eta, "null device pointer");
    IF_REQUIRE(Xprev != X, "Xprev and X must not alias");
    IF_REQUIRE(m0 > 0 && m0 % 16 == 0 && m0 <= 128 && m0 <= A->n, "m0 must be a multiple of 16 in [16, 128]");
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    ifeast_contour C{};
    C.kind = IFEAST_CONTOUR_CIRCLE;
    C.nc = 2;
    C.r = 1.0;
    ifeast_params p{};
    p.m0 = m0;
    p.max_inner = 1;
    p.max_cycles = 1;
    p.precision = IFEAST_PREC_FP64;
    p.problem = IFEAST_PROBLEM_GENERAL;
    Engine& eng = engine_for(ctx, make_shape(A->n, false, &C, &p));
    TimingScope ts(ctx);
    eng.rayleigh_ritz_general(A, Q, Xprev, lam, lam_im, X, R, resid, eta);
    IF_HIP(hipStreamSynchronize(ctx->stream));
    return IFEAST_OK;
  });
}

int ifeast_submit(ifeast_ctx* ctx, const ifeast_csr* A, const ifeast_csr* B, const ifeast_contour* C,
                  const ifeast_params* p, const double* X0, uint64_t* ticket) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && A != nullptr && C != nullptr && p != nullptr && ticket != nullptr, "null argument");
    check_csr(A);
    if (B) check_csr(B);
    IF_REQUIRE(B == nullptr || B->n == A->n, "A and B sizes differ");
    validate_params(*p, *C, A->n);
    uint64_t fp = 0;
    const int s = ifeast_footprint(A->n, A->nnz, B ? B->nnz : 0, C, p, &fp);
    if (s != IFEAST_OK) return fail(ctx, s, ifeast_last_error(nullptr));
    if (fp > ctx->budget) return fail(ctx, IFEAST_ERR_REJECTED, "request footprint exceeds the context budget");
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      if (!ctx->server) ctx->server.reset(new Server(ctx));
    }
    *ticket = ctx->server->submit(A, B, *C, *p, X0, fp);
    return IFEAST_OK;
  });
}

int ifeast_poll(ifeast_ctx* ctx, uint64_t ticket, int* done) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && done != nullptr, "null argument");
    if (!ctx->server) return fail(ctx, IFEAST_ERR_UNKNOWN_TICKET, "unknown ticket");
    return ctx->server->poll(ticket, done);
  });
}

int ifeast_wait(ifeast_ctx* ctx, uint64_t ticket, ifeast_result* res, double* latency_s) {
  return guarded(ctx, [&]() -> int {
    IF_REQUIRE(ctx != nullptr && res != nullptr, "null argument");
    if (!ctx->server) return fail(ctx, IFEAST_ERR_UNKNOWN_TICKET, "unknown ticket");
    return ctx->server->wait(ticket, res, latency_s);
  });
}

}  // extern "C"
