// IFEAST engine: Algorithm 2 with restarted block-GMRES inner solves, all
// arithmetic in device kernels; the host only sequences launches and reads
// a few status words per step.
#pragma once

#include "internal.h"

namespace ifeast {

// Quadrature nodes and weights (Eq. contour_int_quad) and whether the sum is
// taken as 2 Re over the upper half of a conjugate-symmetric rule.
struct Nodes {
  std::vector<cd> z, w;
  bool half = true;
};
Nodes make_nodes(const ifeast_contour& C);
void validate_params(const ifeast_params& p, const ifeast_contour& C, int64_t n);

// Sizes of one solve's device workspace.
struct Shape {
  int64_t n;
  int m0, ns, k;
  bool hasB;
  int precision;
  bool shared = false;  // one real Krylov basis for all shifts (B = I)
  int kb = 0;           // basis capacity in blocks: k (per shift) or k * max_cycles (shared)
  bool general = false; // non-Hermitian A (real, B = I): Ritz block in pair format, full Arnoldi
  bool minres = false;  // batched shifted MINRES (B = I, symmetric): kb = the step cap
};
uint64_t workspace_bytes(const Shape& s);

struct SolveStats {
  int outer = 0, m = 0, converged = 0;
  int64_t total_matvec = 0, seq_matvec = 0;
  double rf = 0.0, seconds = 0.0;
  std::vector<double> rf_hist;
  std::vector<int> inner_hist;  // outer-major, ns per outer
};

// One solve's state: workspace, iterate, nodes.  Reused across calls with the
// same shape (the serving loop keeps one per resident request).
class Engine {
 public:
  Engine(hipStream_t st, const Shape& shape);
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  const Shape& shape() const { return shape_; }
  hipStream_t stream() const { return st_; }

  // Full solve; X0 host n x m0 row-major (FP64).  Results written to res.
  // X0: n x m0 initial block, host memory (NULL: seeded normal block) or, with x0_on_device,
  // device memory.  evec_dev: device n x m0 output of the eigenvectors (NULL: none), in the
  // order of the result arrays; res->evec (host) is filled when non-NULL.
  int solve(const ifeast_matrix* A, const ifeast_matrix* B, const ifeast_contour& C, const ifeast_params& p,
            const double* X0, ifeast_result* res, bool x0_on_device = false, double* evec_dev = nullptr);

  // Step entry points on device data (for the step-level ABI).
  void filter(const ifeast_matrix* A, const ifeast_matrix* B, const ifeast_contour& C, const ifeast_params& p,
              const double* X, const double* lam, const double* R, double rf, double* Q, std::vector<int>* iters);
  void rayleigh_ritz(const ifeast_matrix* A, const ifeast_matrix* B, const double* Q, double* lam, double* X,
                     double* R, double* resid, double* eta);
  // Non-Hermitian Rayleigh-Ritz (pair format); Xprev: the filtered block for the gains (may be null).
  void rayleigh_ritz_general(const ifeast_matrix* A, const double* Q, const double* Xprev, double* lam,
                             double* lam_im, double* X, double* R, double* resid, double* eta);

  struct Impl;

 private:
  Shape shape_;
  hipStream_t st_;
  std::unique_ptr<Impl> impl_;
};

}  // namespace ifeast
