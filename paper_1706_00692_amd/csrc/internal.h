// Internal declarations of libifeast: device matrices, the context, and the
// host-side launchers of every kernel.  Kernels are written for gfx950
// (CDNA4: 64-lane wavefronts, MFMA, 160 KiB LDS per CU, 8 XCDs).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <complex>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ifeast.h"

namespace ifeast {

using cd = std::complex<double>;

// Error carried from deep inside the engine up to the C ABI.
struct Error {
  int status;
  std::string msg;
};

#define IF_HIP(call)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::ifeast::Error{e_ == hipErrorOutOfMemory ? IFEAST_ERR_OOM : IFEAST_ERR_DEVICE,  \
                            std::string(#call) + ": " + hipGetErrorString(e_)};              \
  } while (0)

#define IF_REQUIRE(cond, msg)                                                                \
  do {                                                                                       \
    if (!(cond)) throw ::ifeast::Error{IFEAST_ERR_INVALID_ARG, (msg)};                       \
  } while (0)

// Device buffer with RAII release.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t b);
  ~DevBuf();
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept;
  template <class T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace ifeast

namespace ifeast {
// Autotuned shifted-SpMM schedule key: block width (complex columns), element size, B present.
struct SpmmKey {
  int width, elem;
  bool hasB;
  bool operator<(const SpmmKey& o) const {
    return width != o.width ? width < o.width : elem != o.elem ? elem < o.elem : hasB < o.hasB;
  }
};
}  // namespace ifeast

struct ifeast_matrix {
  int64_t n = 0, nnz = 0;
  ifeast::DevBuf rowptr, colind, val, valf;  // int32, int32, double, float
  double norm1 = 0.0;                        // max column sum of |a_ij|
  int device = 0;
  mutable std::mutex tune_mu;                        // guards sched
  mutable std::map<ifeast::SpmmKey, int> sched;      // autotuned SpMM schedule per product shape
};

namespace ifeast {
// Per-kernel-class timing with HIP events on the launching stream.  When a
// timer is installed for the calling thread, the launchers bracket each
// launch of the classes below with two events and account its algorithmic
// FLOPs and HBM bytes (active shifts only, from the host-known population of
// each device flag array registered with set_count).
enum KClass { KC_SPMM = 0, KC_GRAM = 1, KC_UPDATE = 2, KC_QACC = 3, KC_OUTER = 4, KC_N = 5 };
struct KernelStat {
  int64_t launches = 0;
  double seconds = 0.0, flops = 0.0, bytes = 0.0;
};
struct KernelTimer {
  KernelStat acc[KC_N];
  std::map<const int*, int> counts;
  struct Pending {
    int ev;  // index of the start event; ev + 1 ends it
    int cls;
    double flops, bytes;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pend;
  int next = 0;
  ~KernelTimer();
  int begin(hipStream_t st);
  void end(int tok, int cls, double flops, double bytes);
  void flush();
  void set_count(const int* flags, int cnt) { counts[flags] = cnt; }
  int count(const int* flags, int full) const {
    if (flags == nullptr) return full;
    auto it = counts.find(flags);
    return it == counts.end() ? full : it->second;
  }
  hipStream_t stream = nullptr;
};
KernelTimer*& current_timer();
const char* spmm_schedule_name(int idx);
}  // namespace ifeast

namespace ifeast {
struct Server;  // serving loop (serve.cpp)
}

struct ifeast_ctx {
  int device = 0;
  bool timing = false;
  ifeast::KernelStat kstats[ifeast::KC_N];
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  uint64_t budget = 0;
  std::string last_error;
  std::mutex mu;  // serialises solves on this context
  std::unique_ptr<ifeast::Server> server;
  ifeast::DevBuf zbuf;  // shifts of the step-level SpMM (64 complex FP64)
};

namespace ifeast {

// ------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return immediately.

// W[:, s] = z_s B V[:, s] - A V[:, s] for the ns*m0 complex columns (T = float|double).
template <class T>
void launch_spmm_shifted(hipStream_t st, const ifeast_matrix* A, const ifeast_matrix* B, int ns, int m0,
                         const T* zs /*device, 2*ns*/, const int* active /*device ns or null*/,
                         const T* V, T* W);

// Y = M X for real FP64 n x m blocks (row-major, leading dimension m).
void launch_spmm_real(hipStream_t st, const ifeast_matrix* M, int m, const double* X, double* Y);

// Tall-skinny Gram products on real views, batched:
//   G[item] = sum_rows A_item^T B_item,  A_item (n x PW), B_item (n x QW).
// item = s*ni + i addresses A = A0 + s*a_s + i*a_i, B = B0 + s*b_s (+ i*b_i).
// Partial sums over row splits are reduced in FP64 into G (double, item-major, PW x QW).
// Optional output of a Gram's reduction for one real shift (shared basis): G also goes to
// block column j of Hm (FP64, column-major ldh, block rows i0 + item; added when accumulate)
// and to Hr (type T, G's layout), as the Gram-Schmidt update needs them.
struct GramCombine {
  double* Hm = nullptr;
  int ldh = 0, j = 0, i0 = 0, accumulate = 0;
  void* Hr = nullptr;
};

struct GramArgs {
  int64_t n;
  int PW, QW;
  int ns, ni;  // items = ns * ni
  const void* A;
  int64_t lda, a_s, a_i;  // in elements
  const void* B;
  int64_t ldb, b_s, b_i;
  const int* active;  // per s, may be null
  double* G;          // ns*ni*PW*QW
  int kclass = KC_GRAM;  // timing class (KC_GRAM or KC_OUTER; < 0: not timed)
  int tb_cap = 0;        // > 0: largest square tile, in 16-column blocks (narrow-by-wide products)
  GramCombine cmb;       // optional (cmb.Hm != null): Hm and Hr written by the reduction
  const void* A_last = nullptr;  // optional: block ni - 1 of each shift read from A_last + s * a_s instead
  int reserve = 0;  // multi-block kernel: workgroup slots left to concurrent work when sizing the row split
};
template <class T>
void launch_gram(hipStream_t st, const GramArgs& g, void* partial, size_t partial_bytes);
template <class T>
size_t gram_partial_bytes(int64_t n, int PW, int QW, int items);

// Tall-skinny products on real views, batched over items (z):
//   O_item = beta O_item + alpha sum_b A_{item,b} (n x KW) * Bm_{item,b} (KW x OW)
// with b = 0..nb-1 split as (sb, ib) = (b / nbi, b % nbi):
//   A = A0 + item*a_item + sb*a_s + ib*a_i,  Bm = B0 + item*bm_item + b*KW*OW,
//   O = O0 + item*o_item.  Blocks whose shift flag (active[sb] or active[item]) is 0 are skipped.
struct ApplyArgs {
  int64_t n;
  int KW, OW;
  int items, nb, nbi;
  const void* A;
  int64_t lda, a_item, a_s, a_i;
  const void* Bm;  // same type as A
  int64_t bm_item;
  void* O;         // TO
  int64_t ldo, o_item;
  double alpha, beta;
  const int* active_item;  // per item, may be null
  const int* active_sb;    // per sb, may be null
  int kclass = KC_UPDATE;  // timing class (KC_UPDATE or KC_QACC; < 0: not timed)
  const void* A_last = nullptr;  // optional: block nb - 1 read from A_last + item * a_item instead
  int lower0 = 0;  // 1: block 0's coefficient (KW x OW) is lower triangular; its zero tiles are skipped
  int upper0 = 0;  // 1: block 0's coefficient is upper triangular (a triangular factor's inverse)
};
template <class T, class TO>
void launch_apply(hipStream_t st, const ApplyArgs& a);

// ---- small dense kernels (one workgroup per shift / per solve), FP64
// CholQR factor from the Gram of the block: per shift s,
//   G (2m0 x 2m0 real view of W^H W) -> column scaling, optional shift,
//   Cholesky -> Tinv (real-ified, type T, 2m0 x 2m0) and Rf (complex m0 x m0,
//   W = W_new Rf); if `accumulate`, Racc = Rf * Racc_prev.  real: G is the m0 x m0
//   Gram of a real block and Tinv real m0 x m0 (Rf then has zero imaginary parts).
// The blocked real factor (one block, m0 <= 128; scratch: m0 x m0 doubles of global memory for
// the previous R when it does not fit in LDS beside the factor) steered by a device flag: single[0] != 0
// makes the first pass (role 0) unshifted and the second (role 1) a no-op.  Hm != null: the
// final pass writes Hm(jstep+1, jstep) = R; Hr_next != null: also its transpose into block
// column jstep+1 (rows of block jstep) and into Hr_next (m0 x m0, Gram layout).
template <class T>
void launch_cholqr_real_ctl(hipStream_t st, int m0, const double* G, double shift_rel, T* Tinv, cd* Racc,
                            int accumulate, const int* single, int role, double* Hm = nullptr, int ldh = 0,
                            int jstep = 0, T* Hr_next = nullptr, double* scratch = nullptr);
// single[0] / two[0]: one Cholesky-QR pass is enough for the block with Gram G (m0 x m0, real)
// or not; count[0] (may be null) counts the certified blocks
void launch_gersh_flags(hipStream_t st, int m0, const double* G, double gersh, double dead_thr, int* single, int* two,
                        int* count);
// dst = src (count elements) when flag[0] != 0
template <class T>
void launch_copy_if(hipStream_t st, const int* flag, int64_t count, const T* src, T* dst);
template <class T>
void launch_cholqr_factor(hipStream_t st, int ns, int m0, const double* G, double shift_rel, const int* active,
                          T* Tinv, cd* Racc, int accumulate, cd* work /*ns x 3 m0^2*/, bool real = false);

// CGS combine: for items (s, i), i < ni: C = complex(G) -> H[s](i-block rows, j-block col) = C
// (+= C when accumulate), Hr[s, i] = real-ified C (type T) for the update W -= V Hr.
template <class T>
void launch_cgs_combine(hipStream_t st, int ns, int ni, int m0, int j, int ldh, const double* G,
                        const int* active, cd* H, T* Hr, int accumulate);

// Per shift s, from the Gram G of the block after one Gram-Schmidt pass (real view) and
// that pass's coefficients (column block j of Hbar): need[s] = a second pass is needed
// (some column kept less than eta of its norm); single[s] = one unshifted Cholesky-QR pass
// is enough (no second pass, no negligible column, Gershgorin radius of the scaled Gram
// <= gersh); twopass[s] = active and not single.
void launch_orth_check(hipStream_t st, int ns, int m0, int j, int ldh, double eta, double gersh, double dead_thr,
                       const double* G, const int* active, const cd* H, int* need, int* single, int* twopass);

// Write Racc (m0 x m0 complex) into H[s] at block (row j+1, col j).
void launch_store_subdiag(hipStream_t st, int ns, int m0, int j, int ldh, const int* active, const cd* Racc, cd* H);

// Block-GMRES least squares, incremental Householder QR on Hbar.
struct LsqArgs {
  int ns, m0, k, ldh;
  cd* H;        // ns x [ldh x k*m0] column-major, (k+1)*m0 rows used
  cd* Vh;       // ns x k x [2m0 x m0] Householder vectors (column-major)
  double* tauh; // ns x k x m0 scalars 2/(v^H v)
  cd* g;        // ns x [(k+1)*m0 x m0] column-major transformed right-hand side
  cd* y;        // ns x [k*m0 x m0] column-major solution
  cd* u;        // ns x [(k+1)*m0 x m0] column-major residual coefficients
  double* res;  // ns x m0 current per-column residual norms
  const double* tol;  // ns x m0 stopping thresholds
  int* active;        // ns: shift still iterating in this cycle
  int* iters;         // ns: block iterations in this cycle
  int* cycle_done;    // ns: 1 if the shift met its tolerance
  int need_u = 1;     // lsq_finish also forms u (restart residual coefficients)
  int band = 0;       // > 0: block column j of Hbar is zero above block row j - band (and R above
                      // block row j - band - 1), so only the reflectors of steps >= j - band - 1 act on it
};
// ---- shared-basis inner solve (shared.hip): Arnoldi of M = -A on real blocks
template <class T>
void launch_to_T(hipStream_t st, int64_t count, const double* X, T* Y);
// out[0] = max over columns b of ||G[:, b]|| / ||w_b|| (G = U^T W, nk x m0; gw = W^T W)
void launch_sketch_check_real(hipStream_t st, int nk, int m0, const double* G, const double* gw, double* out);
// gw -= C^T C (C: rows x m0): the Gram of a block after projecting out orthonormal directions
// active (may be null): skipped when active[0] == 0
void launch_gram_downdate(hipStream_t st, int rows, int m0, const double* C, double* gw,
                          const int* active = nullptr);
// act[0..1] = the loss of orthogonality max_b ||G2[:, b]|| / ||w_b|| a first Gram-Schmidt pass
// left against the local blocks exceeds eta (G2: rows x m0, gw = W^T W); act[2] = 1
void launch_local_loss(hipStream_t st, int rows, int m0, const double* G2, const double* gw, double eta, int* act);
// The sketch estimate (Gsk may be null: skipped), the Gershgorin flags of gw and the local loss in
// one launch (launch_sketch_check_real, launch_gersh_flags and launch_local_loss in turn)
void launch_step_checks(hipStream_t st, int nk, int m0, const double* Gsk, const double* gw, double gersh,
                        double dead_thr, int* single, int* two, int* count, int rows, const double* G2, double eta,
                        int* act, double* out);
// The second Gram-Schmidt pass folded into the Cholesky-QR product: from G2 (nl blocks m0 x m0,
// FP64) and Tinv, Cf = [-G2_0 Tinv; ..; -G2_{nl-1} Tinv; Tinv], G2T = G2 in type T, and
// Hm(lo + b, j) += G2_b; with need[0] == 0 (no second pass) only Cf[nl] = Tinv.
template <class T>
void launch_fold_second_pass(hipStream_t st, int m0, int nl, const double* G2, const T* Tinv, T* Cf, T* G2T,
                             double* Hm, int ldh, int j, int lo, const int* need);
void launch_subdiag_real(hipStream_t st, int m0, int j, int ldh, const cd* Racc, double* Hm);
// block column j of Hbar_s = z_s I~ + Hm for every active shift (per-shift complex H, capacity kcap)
void launch_shift_column(hipStream_t st, int ns, int m0, int j, int ldh, int kcap, const double* z, const int* active,
                         const double* Hm, cd* H, int band);
// S_s = S0 diag(1 / (z_s - lambda)) (ns x m0 x m0 row-major)
void launch_start_rhs(hipStream_t st, int ns, int m0, const cd* S0, const double* lam, const double* z, cd* S);
// Yr[b] = Re sum_s wf_s y_s block b (b < jmax), m0 x m0 each, type T
template <class T>
void launch_sum_y(hipStream_t st, int ns, int m0, int kcap, int jmax, const cd* y, const double* wf, T* Yr);

void launch_lsq_init(hipStream_t st, const LsqArgs& a, const cd* S /*ns x m0 x m0 row-major*/);
void launch_lsq_step(hipStream_t st, const LsqArgs& a, int j);
// jmax: host-known bound on the shifts' block iterations (-1: unknown)
void launch_lsq_finish(hipStream_t st, const LsqArgs& a, int jmax = -1);
// Real-ified coefficient blocks from y and u for the tall-skinny products:
//   Yq[s][b] (2m0 x m0, T): Q += Re(V_b (wfac_s y_b))  (wfac = 2w for HALF contours, w otherwise)
//   Uc[s][b] (2m0 x 2m0, T): T1_s = sum_b V_b u_b
template <class T>
void launch_make_coefs(hipStream_t st, const LsqArgs& a, const double* wfac /*2*ns*/, int jmax, T* Yq, T* Uc,
                       int complex_out);

// Rayleigh-Ritz small eigensolve (symmetric): from GA = Q^T A Q, GB = Q^T B Q
// produce lam (ascending), C (m0 x m0 row-major, X = Q C), eta = 1/||c_l||.
// work: 4 m0^2 + 4 m0 doubles.
void launch_rr_small(hipStream_t st, int m0, const double* GA, const double* GB, double* lam, double* C,
                     double* eta, double* work);

// ---- non-Hermitian path (nonsym.hip): Ritz blocks in pair format (a conjugate pair a -+ ib,
// b > 0, owns adjacent columns j, j+1 = Re x, Im x of the eigenvector of a + ib, with
// lam_im[j] = -b, lam_im[j+1] = +b)
// One SVQB pass from the Gram G = P^T P of a block: T (m0 x m0) with P T orthonormal on the
// resolved directions; Tacc <- Tacc T (first: Tacc = T).  work: 3 m0^2 doubles.
void launch_svqb_pass(hipStream_t st, int m0, const double* G, double* T, double* Tacc, int first, double* work);
// Reduced problem of the right-Galerkin Rayleigh-Ritz step on an orthonormal basis P = Q Tacc:
// from GA = P^T A P and GX = X^T X of the filtered block (null: identity): lam, lam_im, W
// (X = P W, unit 2-norm eigenvectors), C = Tacc W, eta.  work: 4 m0^2 doubles.  NaN in lam[0]
// when the Schur iteration fails.
void launch_rr_general(hipStream_t st, int m0, const double* GA, const double* Tacc, const double* GX, double* lam,
                       double* lam_im, double* W, double* C, double* eta, double* work);
// R = A X - X Lambda_b (AX may alias R)
void launch_residual_pairs(hipStream_t st, int64_t n, int m, const double* AX, const double* X, const double* lam,
                           const double* lam_im, double* R);
// resid of a pair's two columns := sqrt(r_j^2 + r_{j+1}^2)
void launch_pair_norms(hipStream_t st, int m, const double* lam_im, double* resid);
// rho_hat at each column's eigenvalue over all nc nodes (z, w device, 2*nc): rho + i rho_im
void launch_rho_pairs(hipStream_t st, int m0, int nc, const double* z, const double* w, const double* lam,
                      const double* lam_im, double* rho, double* rho_im);
// Y = X rho_hat(Lambda_b)
void launch_scale_pairs(hipStream_t st, int64_t n, int m, const double* X, const double* rho, const double* rho_im,
                        const double* lam_im, double* Y);
// S_s = S0 (z_s - Lambda_b)^{-1} (ns x m0 x m0 row-major)
void launch_start_rhs_pairs(hipStream_t st, int ns, int m0, const cd* S0, const double* lam, const double* lam_im,
                            const double* z, cd* S);

// Membership, spurious test and ||R_F|| (Algorithm 2, step 4) on device:
// flags[j] = IFEAST_FLAG_* bits; out[0] = ||R_F||, out[1] = m (as double), out[2] = Ritz
// values inside the contour whether counted or not.  lam_im (may be null): imaginary parts.
struct ClassifyArgs {
  int m0, nc, half, kind;  // kind: IFEAST_CONTOUR_*
  double emin, emax, c_re, c_im, r, tau;
  const double* z;  // device 2*nc
  const double* w;  // device 2*nc
};
void launch_classify(hipStream_t st, const ClassifyArgs& a, const double* lam, const double* lam_im,
                     const double* resid, const double* eta, int* flags, double* out);

// ---- batched shifted MINRES (minres.hip): one Lanczos recurrence per column of R shared by all
// shifts, minimal-residual iterates by Givens rotations of each shift's tridiagonal, direction
// vectors by a three-term recurrence accumulated straight into Q.  Buffers belong to the caller:
// V, Vp, W: n x m0 (T); D1, D2: ns x n x m0 complex (T, interleaved); pa, pb: partial sums
// (minres_partial_bytes each); state: minres_state_bytes.
size_t minres_state_bytes(int m0, int ns);
size_t minres_partial_bytes(int64_t n, int m0);
template <class T>
struct MinresRun {
  int64_t n;
  int m0, ns;
  T *V, *Vp, *W, *D1, *D2;
  double *pa, *pb;
  void* state;
  int k = 0;
  // v_1 = R / rnorm per column (R: n x m0 FP64, rnorm its column norms), zero directions, and
  // g_1 = rnorm / (z_s - lambda_c) per (column, shift); z: device 2 ns doubles
  int start(hipStream_t st, const double* R, const double* rnorm, const double* lam, const double* z);
  // one Lanczos step for every column and one MINRES update for every active (column, shift):
  // zeroshift: device complex 0 of type T; z, wf: device 2 ns doubles (nodes, quadrature factors
  // of Q += Re(wf x)); tol: device ns x m0 stopping thresholds on the minimal residual
  void step(hipStream_t st, const ifeast_matrix* A, const T* zeroshift, const double* z, const double* wf,
            const double* tol, double* Q);
  const int* column_active() const;  // device m0: pairs of each column still iterating
  const int* shift_steps() const;    // device ns: steps in which each shift iterated
};

// ---- allocation-free Rayleigh-Ritz (noalloc.hip)
// Size of the per-device scratch array the allocation-free entry point draws every buffer from.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// Device address of `device`'s scratch array, looked up once per device (the device must be current).
void* noalloc_scratch(int device);
// Scratch bytes one allocation-free Rayleigh-Ritz step needs.
size_t noalloc_rr_bytes(int64_t n, int m0, bool hasB);
// Rayleigh-Ritz and residuals (as Engine::rayleigh_ritz) with no device allocation: buffers from
// the scratch array, A Q staged in the output X.  INVALID_ARG when the scratch is too small.
void rayleigh_ritz_noalloc(hipStream_t st, int device, const ifeast_matrix* A, const ifeast_matrix* B, int m0,
                           const double* Q, double* lam, double* X, double* R, double* resid, double* eta);

// ---- elementwise / reductions
void launch_col_sumsq(hipStream_t st, int64_t n, int m, const double* X, double* out /*m*/, double* partial);
void launch_scale_cols(hipStream_t st, int64_t n, int m, const double* X, const double* f, double* Y);
void launch_residual(hipStream_t st, int64_t n, int m, const double* AX, const double* BX, const double* lam,
                     double* R);
template <class T>
void launch_rhs_build(hipStream_t st, int64_t n, int m0, int ns, const double* R, const double* lam,
                      const double* z /*2*ns*/, T* out);
void launch_col_sumsq_finish(hipStream_t st, int nblocks, int m, const double* partial, double* out, int do_sqrt);
int col_sumsq_blocks(int64_t n);
void launch_fill_zero(hipStream_t st, void* p, size_t bytes);

}  // namespace ifeast
