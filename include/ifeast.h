/*
 * ifeast.h -- C ABI of libifeast, an MI355X (gfx950) implementation of the
 * IFEAST eigensolver: FEAST contour integration with inexact block-GMRES
 * solves of the shifted systems (Gavin & Polizzi, arXiv 1706.00692).
 *
 * Problem (Eq. eigenvalueproblem; generalized form Eq. generalized_linsys):
 *   find the eigenpairs A x = lambda B x with lambda inside a contour C,
 *   A, B real sparse (CSR), B symmetric positive definite or the identity.
 *   Non-Hermitian problems (Sec. 1.1: the results extend to them): A real
 *   nonsymmetric, B = I, C a circle centred on the real axis; the Ritz
 *   problem is solved with the right Galerkin condition.
 * Method (Algorithm 2): starting from an n x m0 block X, each outer
 * iteration solves the nc shifted systems (z_k B - A) Y_k = B X inexactly
 * with block GMRES (one real Krylov basis shared by all shifts when B = I,
 * restarted per-shift bases otherwise), forms Q = sum_k w_k Y_k (Eq. contour_int_quad),
 * and runs Rayleigh-Ritz on span(Q) (Algorithm 2, step 3) until the
 * eigenvector residual ||R_F|| = max ||A x_j - lambda_j B x_j|| over the pairs
 * inside C falls below tol (Algorithm 2, step 4).
 *
 * Conventions
 *   - Every call returns an int status: IFEAST_OK (0), a warning (> 0: the
 *     outputs are valid but flagged) or an error (< 0: outputs untouched or
 *     partial).  No C++ exception crosses this interface.  After an error
 *     ifeast_last_error(ctx) describes it.
 *   - Host pointers are owned by the caller and only read during the call
 *     (ifeast_submit copies them before returning).  Device pointers
 *     (the *_dev entry points) must be device memory on the context's device
 *     and stay valid until the call returns; work is ordered on the context's
 *     stream (see ifeast_set_stream).
 *   - Dense blocks are row-major: element (i, j) of an n x m block is at
 *     i*m + j.  Complex numbers are interleaved (re, im) pairs.
 *   - Matrices are 0-based CSR with sorted, duplicate-free column indices
 *     within each row; nnz must be < 2^31.
 *   - m0 must be a multiple of 16 in [16, 128].
 */
#ifndef IFEAST_H
#define IFEAST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
enum {
  IFEAST_OK = 0,
  IFEAST_WARN_NOT_CONVERGED = 1,   /* max_outer reached; results are the last iterate */
  IFEAST_WARN_M0_TOO_SMALL = 2,    /* after an outer iteration all m0 Ritz values lie inside C (the premise of
                                      Algorithm 2, fewer than m0 eigenvalues inside, fails); the solve stops */
  IFEAST_WARN_NO_EIG_IN_CONTOUR = 3, /* after an outer iteration no Ritz value lies inside C; the solve stops */
  IFEAST_ERR_INVALID_ARG = -1,
  IFEAST_ERR_OOM = -2,
  IFEAST_ERR_DEVICE = -3,
  IFEAST_ERR_NUMERICAL = -4,       /* NaN/Inf met in the iteration */
  IFEAST_ERR_REJECTED = -5,        /* request footprint exceeds the context's HBM budget */
  IFEAST_ERR_UNKNOWN_TICKET = -6,
  IFEAST_ERR_UNSUPPORTED = -7
};

/* ----------------------------------------------------------------- inputs */
typedef struct ifeast_ctx ifeast_ctx;       /* one GPU, one stream, owns device memory */
typedef struct ifeast_matrix ifeast_matrix; /* a CSR matrix resident in HBM */

typedef struct {
  int64_t n;              /* rows = columns */
  int64_t nnz;
  const int64_t *rowptr;  /* n+1 entries, rowptr[0] = 0, rowptr[n] = nnz */
  const int32_t *colind;  /* nnz entries, sorted within each row */
  const double *val;      /* nnz entries */
} ifeast_csr;

enum { IFEAST_CONTOUR_HALF = 0,      /* real symmetric pencil: nc nodes on the upper half of the
                                        circle through emin and emax, Q = 2 Re sum (Sec. 4.1) */
       IFEAST_CONTOUR_CIRCLE = 1,    /* nc trapezoidal nodes around |z - c| = r */
       IFEAST_CONTOUR_EXPLICIT = 2 };/* caller-given nodes and weights */
enum { IFEAST_RULE_GAUSS_LEGENDRE = 0, IFEAST_RULE_TRAPEZOID = 1 };

typedef struct {
  int kind;                /* IFEAST_CONTOUR_* */
  int rule;                /* IFEAST_RULE_* (HALF only; CIRCLE is always trapezoidal) */
  int nc;                  /* number of shifted systems solved */
  double emin, emax;       /* HALF: the search interval (open); EXPLICIT: the interval for membership */
  double c_re, c_im, r;    /* CIRCLE: centre and radius */
  const double *z;         /* EXPLICIT: nc complex nodes, interleaved */
  const double *w;         /* EXPLICIT: nc complex weights, interleaved */
  int half;                /* EXPLICIT: 1 if the nodes are the upper half of a conjugate-symmetric rule */
} ifeast_contour;

enum { IFEAST_PREC_FP64 = 0,   /* FP64 inner solves and outer iteration */
       IFEAST_PREC_MIXED = 1 };/* FP32 inner solves (the shared basis: one real FP32 Krylov basis; the
                                  per-shift basis: complex FP32 blocks), FP64 outer iteration */
enum { IFEAST_PROBLEM_SYMMETRIC = 0, /* A symmetric, B SPD or NULL: HALF or EXPLICIT contours */
       IFEAST_PROBLEM_GENERAL = 1 };  /* A nonsymmetric, B NULL, a CIRCLE contour with c_im = 0 and an
                                         even nc (the rule is symmetric about the real axis, so the
                                         nc/2 systems of the upper half are solved and the lower
                                         half's solutions are their conjugates); shared basis only */
enum { IFEAST_GUESS_RITZ = 0,  /* inner initial guess X (z - Lambda)^{-1} */
       IFEAST_GUESS_ZERO = 1 };/* zero initial guess, right-hand side B X (Algorithm 2 as printed) */
enum { IFEAST_BASIS_AUTO = 0,      /* shared for B = I, per shift otherwise */
       IFEAST_BASIS_SHARED = 1,    /* one real block Arnoldi of A serves every shift (B = I only): the shifted
                                      block Krylov spaces from R (z_s - Lambda)^{-1} coincide, so up to
                                      max_inner * max_cycles block steps run without restarts and only the
                                      small least-squares problems are per shift */
       IFEAST_BASIS_PER_SHIFT = 2, /* per shift complex block GMRES(max_inner), restarted up to max_cycles */
       IFEAST_BASIS_MINRES = 3 };  /* B = I, symmetric A: MINRES per column (the paper's inner solver, Sec. 2), one
                                      Lanczos recurrence per column of R serving every shift, directions by
                                      three-term recurrences added straight into Q, no Krylov basis stored; at
                                      most max_inner * max_cycles steps */
enum { IFEAST_INNER_GLOBAL = 0,/* stop when every column residual <= alpha ||R_F|| (Algorithm 2, step 1) */
       IFEAST_INNER_COLUMN = 1 };/* column j stops when its residual fell by alpha (Eq. alpha with alpha_j = alpha) */

typedef struct {
  int m0;              /* search subspace size, multiple of 16, at most 128 */
  int max_outer;       /* outer (subspace) iterations */
  int max_inner;       /* k: block-GMRES iterations per restart cycle (basis of k+1 blocks) */
  int max_cycles;      /* restart cycles per shifted solve and outer iteration */
  double alpha;        /* inner tolerance factor, 0 <= alpha < 1 */
  double tol;          /* eigen-residual tolerance on ||R_F|| */
  double spurious_tau; /* a Ritz pair inside C counts when its filter gain >= tau |rho_hat(lambda)| */
  double reorth_eta;   /* block Gram-Schmidt in the Arnoldi step.  Per-shift bases: a second classical
                          pass runs for a shift when some column kept less than this fraction of its
                          norm in the first one, and the block is normalised by one Cholesky-QR pass
                          when its Gram is certified well conditioned (two passes otherwise); 0
                          selects 0.1.  Shared basis: both passes project against the two newest
                          blocks, and the second also against every older block when the loss of
                          orthogonality to them, max over columns w of ||[V_0..]^T w|| / ||w||
                          estimated from a 16-column random sketch, exceeds this value; 0 selects
                          max(1e-4, alpha / 10) for an FP32 basis and 1e-12 for an FP64 one.
                          >= 1: always two full passes and two Cholesky-QR passes */
  int precision;       /* IFEAST_PREC_* */
  int problem;         /* IFEAST_PROBLEM_* */
  int inner_guess;     /* IFEAST_GUESS_* */
  int inner_rule;      /* IFEAST_INNER_* */
  int basis;           /* IFEAST_BASIS_* */
  uint64_t seed;       /* seed of the initial block when X0 is NULL */
} ifeast_params;

/* ---------------------------------------------------------------- outputs */
enum { IFEAST_FLAG_INSIDE = 1,    /* counted eigenpair inside C */
       IFEAST_FLAG_SPURIOUS = 2 };/* inside C but with an inconsistent filter gain */

typedef struct {
  /* filled by the library */
  int m;                   /* counted eigenpairs inside C (they come first, ascending) */
  int outer_iters;
  int converged;
  int64_t total_matvec;    /* columns multiplied by A: per-shift bases, sum over shifts of block iterations
                              times m0 (complex columns); shared basis, Arnoldi steps times m0 (real) */
  int64_t seq_matvec;      /* sum over outer iterations of the sequential block products: the largest
                              per-shift block-iteration count, or the shared basis's Arnoldi steps */
  double max_resid;        /* ||R_F|| of the final iterate */
  double solve_seconds;    /* device time of the solve, CSR upload excluded */
  /* caller-allocated arrays (may be NULL to skip) */
  double *eval_re;         /* m0 */
  double *eval_im;         /* m0 (zeros for symmetric problems) */
  double *evec;            /* n x m0 row-major, B-normalised; PROBLEM_GENERAL: n x m0 complex
                              (interleaved re, im: 2 n m0 doubles), unit 2-norm */
  double *resid;           /* m0 residual norms ||A x_j - lambda_j B x_j|| */
  int32_t *flags;          /* m0 IFEAST_FLAG_* bits */
  double *rf_hist;         /* max_outer entries: ||R_F|| after each outer iteration */
  int32_t *inner_hist;     /* max_outer * nc entries: block iterations per shift per outer iteration */
} ifeast_result;

/* ------------------------------------------------------------ contexts */
/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory of resident requests in the serving loop (0 = 90% of free). */
int ifeast_create(ifeast_ctx **ctx, int device, uint64_t hbm_budget_bytes);
/* Free the context.  Serving requests still queued end with
 * IFEAST_ERR_DEVICE (a thread blocked in ifeast_wait on one returns that
 * status); running ones finish first.  No other call may start on the
 * context once destroy has begun (such a call races with the free). */
int ifeast_destroy(ifeast_ctx *ctx);
/* Order the context's later work on a caller stream (a hipStream_t passed as
 * void*; NULL is the default (null) stream).  Until this is called a context
 * uses a stream of its own.  The stream must outlive its use. */
int ifeast_set_stream(ifeast_ctx *ctx, void *stream);
const char *ifeast_status_str(int status);
const char *ifeast_last_error(ifeast_ctx *ctx);
/* Library version string. */
const char *ifeast_version(void);

/* ------------------------------------------------------------ matrices */
/* Validate a CSR matrix and copy it to HBM (FP64 values plus an FP32 copy
 * for the mixed-precision inner solves).  Errors: INVALID_ARG on unsorted or
 * out-of-range indices, non-finite values or nnz >= 2^31. */
int ifeast_matrix_create(ifeast_ctx *ctx, const ifeast_csr *A, ifeast_matrix **out);
int ifeast_matrix_destroy(ifeast_ctx *ctx, ifeast_matrix *M);
int64_t ifeast_matrix_n(const ifeast_matrix *M);

/* ---------------------------------------------------------------- solve */
/* Device bytes one solve needs (workspace + matrices) for these inputs. */
int ifeast_footprint(int64_t n, int64_t nnzA, int64_t nnzB, const ifeast_contour *C,
                     const ifeast_params *p, uint64_t *bytes);

/* Solve with matrices already resident in HBM.  B may be NULL (identity).
 * X0: host n x m0 row-major initial block, NULL = seeded normal block.
 * Returns OK, a warning, or an error. */
int ifeast_solve_resident(ifeast_ctx *ctx, const ifeast_matrix *A, const ifeast_matrix *B,
                          const ifeast_contour *C, const ifeast_params *p, const double *X0,
                          ifeast_result *res);

/* As ifeast_solve_resident with the big arrays in HBM: X0 is a device n x m0
 * row-major initial block (required), evec a device n x m0 row-major output
 * for the eigenvectors in the order of res's arrays (NULL: not written;
 * PROBLEM_GENERAL: n x m0 complex, 2 n m0 doubles interleaved).  The
 * small host arrays of res are filled as in ifeast_solve_resident; res->evec,
 * when non-NULL, is filled too.  Both device buffers belong to the caller and
 * are used on the context's stream; the call returns when the solve is done. */
int ifeast_solve_dev(ifeast_ctx *ctx, const ifeast_matrix *A, const ifeast_matrix *B,
                     const ifeast_contour *C, const ifeast_params *p, const double *X0,
                     double *evec, ifeast_result *res);

/* Upload, solve, free: ifeast_matrix_create + ifeast_solve_resident. */
int ifeast_solve(ifeast_ctx *ctx, const ifeast_csr *A, const ifeast_csr *B, const ifeast_contour *C,
                 const ifeast_params *p, const double *X0, ifeast_result *res);

/* --------------------------------------------------------- serving loop */
/* Continuous batching: submit copies the request and returns at once; a
 * background scheduler admits requests by device footprint against the
 * context budget, keeps their state resident and interleaves their inner
 * iterations on the device.  REJECTED if one request alone exceeds the
 * budget.  wait blocks until the request finishes and fills `res`
 * (caller-allocated arrays as in ifeast_solve); latency_s is completion
 * minus submission time. */
int ifeast_submit(ifeast_ctx *ctx, const ifeast_csr *A, const ifeast_csr *B, const ifeast_contour *C,
                  const ifeast_params *p, const double *X0, uint64_t *ticket);
int ifeast_poll(ifeast_ctx *ctx, uint64_t ticket, int *done);
int ifeast_wait(ifeast_ctx *ctx, uint64_t ticket, ifeast_result *res, double *latency_s);

/* ------------------------------------------------------- kernel timing */
/* Classes of kernels whose launches are timed when timing is on. */
enum { IFEAST_KERNEL_SPMM = 0,   /* batched shifted SpMM (Algorithm 2, step 1) */
       IFEAST_KERNEL_GRAM = 1,   /* Gram products of the block orthogonalization (CGS, Cholesky QR) */
       IFEAST_KERNEL_UPDATE = 2, /* block updates W -= V H, W R^-1 and restart combinations */
       IFEAST_KERNEL_QACC = 3,   /* quadrature accumulation Q += Re sum_s wf_s V_s y_s */
       IFEAST_KERNEL_OUTER = 4 };/* FP64 products of the Rayleigh-Ritz step */
typedef struct {
  int64_t launches;
  double seconds;  /* sum of launch durations, from HIP events on the context's stream */
  double flops;    /* algorithmic floating-point operations of those launches (active shifts only) */
  double bytes;    /* algorithmic device-memory bytes: every operand read once, every result written once */
} ifeast_kernel_stat;
/* enable != 0: reset the totals and time every later compute call on this
 * context (two events per timed launch, flushed every 256 launches);
 * 0: stop timing.  Totals survive until the next ifeast_set_timing. */
int ifeast_set_timing(ifeast_ctx *ctx, int enable);
/* Totals of class `kind` (IFEAST_KERNEL_*) since timing was last enabled. */
int ifeast_kernel_stats(ifeast_ctx *ctx, int kind, ifeast_kernel_stat *out);

/* ------------------------------------------------- steps (device pointers) */
/* One launch of the batched shifted product for all systems
 * (Algorithm 2, step 1, the only access to A and B):
 *     W[:, s*m0:(s+1)*m0] = z_s B V[:, s*m0:(s+1)*m0] - A V[:, s*m0:(s+1)*m0],
 * s = 0..ns-1.  V and W are device n x (ns*m0) complex blocks, row-major;
 * precision MIXED means complex FP32 elements with the FP32 matrix copy,
 * FP64 means complex FP64.  z: host array of ns complex shifts.  B NULL =
 * identity.  Asynchronous: the product is queued on the context's stream
 * (ifeast_set_stream) and W is complete when that stream reaches it; the
 * first product of a new (matrix, width, precision) also times the SpMM
 * schedules and keeps the fastest for that matrix. */
int ifeast_spmm_shifted_dev(ifeast_ctx *ctx, const ifeast_matrix *A, const ifeast_matrix *B, int precision,
                            int ns, const double *z, int m0, const void *V, void *W);

/* One inexact filter application (Algorithm 2, steps 1-2) on device data:
 * given B-orthonormal Ritz vectors X (n x m0, FP64), Ritz values lam (m0)
 * and residuals R = A X - B X diag(lam) (n x m0), solve every shifted system
 * for the correction from the right-hand side R (z_k - lam)^{-1} with
 * restarted block GMRES and return
 *     Q = X rho_hat(Lambda) + sum_k w_k D_k   (2 Re of the sum for HALF contours).
 * rf is ||R_F|| (used by IFEAST_INNER_GLOBAL).  inner_iters (host, nc
 * entries, may be NULL) receives the block iterations per shift. */
int ifeast_filter_dev(ifeast_ctx *ctx, const ifeast_matrix *A, const ifeast_matrix *B, const ifeast_contour *C,
                      const ifeast_params *p, const double *X, const double *lam, const double *R, double rf,
                      double *Q, int32_t *inner_iters);

/* Rayleigh-Ritz and residuals on device data (Algorithm 2, steps 3-4):
 * B-orthonormalise span(Q) and solve the reduced problem, returning Ritz
 * values lam (ascending), vectors X = Q C (n x m0), residual block R and its
 * column norms resid, and eta (filter gains 1/||c_l||; pass Q = filter(X)
 * of a B-orthonormal X for them to be meaningful). */
int ifeast_rayleigh_ritz_dev(ifeast_ctx *ctx, const ifeast_matrix *A, const ifeast_matrix *B, int m0,
                             const double *Q, double *lam, double *X, double *R, double *resid, double *eta);

/* ifeast_rayleigh_ritz_dev for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid allocation): the same outputs from the
 * same kernels, with every scratch buffer taken from a per-device array of 64 MiB that the
 * library holds until the process ends (A Q is staged in X).  Nothing is allocated by the call.
 * The scratch needed grows with n and m0 (and by n m0 doubles when B is given); a problem that
 * needs more than the array returns IFEAST_ERR_INVALID_ARG before any work is queued.  All calls
 * on one device share the array: calls that overlap on one device race.  Q must not alias X. */
int ifeast_rayleigh_ritz_dev_noalloc(ifeast_ctx *ctx, const ifeast_matrix *A, const ifeast_matrix *B, int m0,
                                     const double *Q, double *lam, double *X, double *R, double *resid,
                                     double *eta);

/* Non-Hermitian Rayleigh-Ritz on device data (Algorithm 2, steps 3-4, right Galerkin condition,
 * B = I): orthonormalise span(Q) (n x m0, FP64, row-major), solve the reduced eigenproblem of
 * Q^T A Q and return the Ritz values lam + i lam_im (m0 each, ascending real part) and the
 * Ritz block X = Q C in pair format: a real Ritz value owns one column, its unit eigenvector;
 * a conjugate pair a -+ ib (b > 0) owns two adjacent columns j, j+1 holding Re x and Im x of
 * the eigenvector x of a + ib (||x|| = 1), with lam_im[j] = -b, lam_im[j+1] = +b.  R = A X - X
 * Lambda in the same format (a pair's columns: real and imaginary parts of A x - lambda x),
 * resid the residual norm of each complex eigenvector (shared by a pair's columns), and eta
 * the filter gains 1 / ||Xprev c_l|| (Xprev: the block filtered into Q, n x m0; NULL: gains
 * against the identity).  Xprev must not alias X.  ERR_NUMERICAL-style failures (the Schur
 * iteration not converging) leave NaN in lam[0]. */
int ifeast_rayleigh_ritz_general_dev(ifeast_ctx *ctx, const ifeast_matrix *A, int m0, const double *Q,
                                     const double *Xprev, double *lam, double *lam_im, double *X, double *R,
                                     double *resid, double *eta);

#ifdef __cplusplus
}
#endif

#endif /* IFEAST_H */
