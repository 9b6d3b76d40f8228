// The Rayleigh-Ritz step (Algorithm 2, steps 3-4) for callers that cannot allocate device
// memory (code under graph capture, serving loops, harnesses that forbid allocation).
//
// Every scratch buffer of the step (the Gram matrices, the reduced eigensolver's workspace,
// the split-K and column-norm partial sums, B Q) is carved from one file-scope device array.
// The output block X stages A Q before it receives the Ritz vectors, so B = I needs no n x m0
// scratch at all.  Each device holds its own copy of the array until the process ends; all
// calls on one device share it, so calls that overlap on one device race.
#include <mutex>

#include "internal.h"

static __device__ __align__(256) unsigned char scratch[ifeast::kNoAllocScratchBytes];

namespace ifeast {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

// Device address of this device's scratch array.  The array's name is a host-side stand-in in
// host code; only this address may reach kernels or copies.  The caller makes `device` current.
void* noalloc_scratch(int device) {
  IF_REQUIRE(device >= 0 && device < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    void* p = nullptr;
    IF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    IF_REQUIRE(p != nullptr, "no device address for the scratch array");
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

size_t noalloc_rr_bytes(int64_t n, int m0, bool hasB) {
  const size_t mm = (size_t)m0 * m0 * sizeof(double);
  size_t b = 3 * align256(mm);                                                     // GA, GB, C
  b += align256((4 * (size_t)m0 * m0 + 4 * m0) * sizeof(double));                 // eigensolver
  b += align256((size_t)col_sumsq_blocks(n) * m0 * sizeof(double));                // column norms
  b += align256(gram_partial_bytes<double>(n, m0, m0, 1));                         // Gram partials
  if (hasB) b += align256((size_t)n * m0 * sizeof(double));                        // B Q, then B X
  return b;
}

void rayleigh_ritz_noalloc(hipStream_t st, int device, const ifeast_matrix* A, const ifeast_matrix* B, int m0,
                           const double* Q, double* lam, double* X, double* R, double* resid, double* eta) {
  const int64_t n = A->n;
  const size_t need = noalloc_rr_bytes(n, m0, B != nullptr);
  IF_REQUIRE(need <= kNoAllocScratchBytes,
             "the problem needs " + std::to_string(need >> 20) + " MiB of scratch; the allocation-free Rayleigh-Ritz "
             "entry point holds " + std::to_string(kNoAllocScratchBytes >> 20) + " MiB per device");
  char* base = static_cast<char*>(noalloc_scratch(device));
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    char* p = base + off;
    off += align256(bytes);
    return p;
  };
  const size_t mm = (size_t)m0 * m0 * sizeof(double);
  double* GA = reinterpret_cast<double*>(carve(mm));
  double* GB = reinterpret_cast<double*>(carve(mm));
  double* C = reinterpret_cast<double*>(carve(mm));
  double* work = reinterpret_cast<double*>(carve((4 * (size_t)m0 * m0 + 4 * m0) * sizeof(double)));
  double* colpart = reinterpret_cast<double*>(carve((size_t)col_sumsq_blocks(n) * m0 * sizeof(double)));
  const size_t gpart_bytes = gram_partial_bytes<double>(n, m0, m0, 1);
  void* gpart = carve(gpart_bytes);
  double* BQ = B != nullptr ? reinterpret_cast<double*>(carve((size_t)n * m0 * sizeof(double))) : nullptr;
  // A Q staged in X; B Q in the scratch (B = I: Q itself)
  double* AQ = X;
  launch_spmm_real(st, A, m0, Q, AQ);
  const double* bq = Q;
  if (B != nullptr) {
    launch_spmm_real(st, B, m0, Q, BQ);
    bq = BQ;
  }
  GramArgs ga{n, m0, m0, 1, 1, Q, m0, 0, 0, AQ, m0, 0, 0, nullptr, GA, -1};
  launch_gram<double>(st, ga, gpart, gpart_bytes);
  GramArgs gb{n, m0, m0, 1, 1, Q, m0, 0, 0, bq, m0, 0, 0, nullptr, GB, -1};
  launch_gram<double>(st, gb, gpart, gpart_bytes);
  launch_rr_small(st, m0, GA, GB, lam, C, eta, work);
  // A X = (A Q) C into R, then X = Q C over the staged A Q
  ApplyArgs aa{n, m0, m0, 1, 1, 1, AQ, m0, 0, 0, 0, C, 0, R, m0, 0, 1.0, 0.0, nullptr, nullptr, -1};
  launch_apply<double, double>(st, aa);
  ApplyArgs ax = aa;
  ax.A = Q;
  ax.O = X;
  launch_apply<double, double>(st, ax);
  const double* bx = X;
  if (B != nullptr) {
    launch_spmm_real(st, B, m0, X, BQ);  // B X over B Q
    bx = BQ;
  }
  launch_residual(st, n, m0, R, bx, lam, R);
  launch_col_sumsq(st, n, m0, R, resid, colpart);
}

}  // namespace ifeast
