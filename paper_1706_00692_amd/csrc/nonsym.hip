// Kernels of the non-Hermitian path (real A, B = I, a contour symmetric about the real axis).
//
// Ritz pairs of a real nonsymmetric matrix are real or come in conjugate pairs.  The engine
// keeps the Ritz block real ("pair format"): a real eigenvalue owns one column holding its
// eigenvector; a pair a -+ ib (b > 0) owns two adjacent columns j, j+1 holding Re x and Im x
// of the eigenvector x of a + ib, with lam_im[j] = -b, lam_im[j+1] = +b.  Then
//     A [x_j, x_{j+1}] = [x_j, x_{j+1}] J,   J = [[a, b], [-b, a]],
// so the block X spans the same complex subspace as the complex Ritz vectors, and every block
// operation of Algorithm 2 (the residual R = A X - X Lambda, the start block R (z - Lambda)^{-1},
// the filter value X rho_hat(Lambda)) acts on 2 x 2 real blocks instead of complex scalars.
//
//  * k_svqb_pass: one SVQB orthonormalisation pass of span(Q); the engine runs three (the
//    first floors the Gram's tiny eigenvalues, the next two make the result orthonormal to
//    rounding: with one pass the floored directions are not orthonormal, and for a nonnormal
//    A that alone held the Ritz residuals near sqrt(eps)).
//  * k_rr_general: the reduced problem of the Rayleigh-Ritz step (Algorithm 2, step 3, right
//    Galerkin condition) on the orthonormal basis: Hessenberg reduction, Francis double-shift
//    QR to the real Schur form, eigenvectors of the quasi-triangular factor by back
//    substitution, unit 2-norm, ascending order by real part, filter gains.
//  * pair-aware residual, residual norms, filter values, start blocks.
#include "internal.h"

#define RR_MARK(i) \
  do {             \
  } while (0)
#include "dense_dev.h"

namespace ifeast {

namespace {

constexpr double kEps = 2.220446049250313e-16;

// ---------------------------------------------------------------- Hessenberg
// H (LDS, m x m, stride ld) <- P^T H P upper Hessenberg, Z (global, row-major m x m) <- Z P,
// by Householder reflectors I - beta v v^T on rows / columns k+1.. (k = 0 .. m-3).
// vb, pb: LDS vectors of m doubles.
__device__ void hessenberg_reduce(double* H, int ld, int m, double* Z, double* red, double* vb, double* pb) {
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int k = 0; k + 2 < m; ++k) {
    const int n1 = k + 1;
    double x = 0.0;
    for (int r = n1 + tid; r < m; r += nth) x += H[r * ld + k] * H[r * ld + k];
    const double sigma = block_sum(x, red);
    const double x0 = H[n1 * ld + k];
    const double alpha = x0 >= 0.0 ? -sqrt(sigma) : sqrt(sigma);
    const double v0 = x0 - alpha;
    const double vn2 = sigma - x0 * x0 + v0 * v0;
    const double beta = (sigma > 0.0 && vn2 > 0.0) ? 2.0 / vn2 : 0.0;
    if (beta == 0.0) continue;  // uniform: every thread computed the same values
    for (int r = n1 + tid; r < m; r += nth) vb[r] = (r == n1) ? v0 : H[r * ld + k];
    __syncthreads();
    // rows n1..: p_c = beta sum_r v_r H[r][c] for c >= k (eight lanes per column)
    {
      const int c = k + (tid >> 3), part = tid & 7;
      double acc = 0.0;
      if (c < m)
        for (int r = n1 + part; r < m; r += 8) acc += vb[r] * H[r * ld + c];
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      acc += __shfl_xor(acc, 4);
      if (c < m && part == 0) pb[c] = beta * acc;
    }
    __syncthreads();
    for (int idx = tid; idx < (m - n1) * (m - k); idx += nth) {
      const int r = n1 + idx / (m - k), c = k + idx % (m - k);
      H[r * ld + c] -= vb[r] * pb[c];
    }
    __syncthreads();
    // columns n1..: q_r = beta sum_c H[r][c] v_c for every row, and the same for Z
    {
      const int r = tid >> 3, part = tid & 7;
      double acc = 0.0, accz = 0.0;
      if (r < m)
        for (int c = n1 + part; c < m; c += 8) {
          acc += H[r * ld + c] * vb[c];
          accz += Z[r * m + c] * vb[c];
        }
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      acc += __shfl_xor(acc, 4);
      accz += __shfl_xor(accz, 1);
      accz += __shfl_xor(accz, 2);
      accz += __shfl_xor(accz, 4);
      if (r < m && part == 0) {
        pb[r] = beta * acc;
        vb[m + r] = beta * accz;  // vb holds 2m doubles
      }
    }
    __syncthreads();
    for (int idx = tid; idx < m * (m - n1); idx += nth) {
      const int r = idx / (m - n1), c = n1 + idx % (m - n1);
      H[r * ld + c] -= pb[r] * vb[c];
      Z[r * m + c] -= vb[m + r] * vb[c];
    }
    __syncthreads();
    // column k below the subdiagonal is exactly zero now
    for (int r = n1 + tid; r < m; r += nth) H[r * ld + k] = (r == n1) ? alpha : 0.0;
    __syncthreads();
  }
}

// Householder reflector mapping (x0, x1, x2) to (alpha, 0, 0): P = I - tau v v^T with v[0] set
// here; tau = 0 means the identity (nothing to annihilate).
__device__ inline double reflector3(double x0, double x1, double x2, double* v) {
  if (x1 == 0.0 && x2 == 0.0) return 0.0;
  const double nrm = sqrt(x0 * x0 + x1 * x1 + x2 * x2);
  const double alpha = x0 >= 0.0 ? -nrm : nrm;
  v[0] = x0 - alpha;
  v[1] = x1;
  v[2] = x2;
  return 2.0 / (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
}

// P = I - tau v v^T (length nv = 2 or 3, on rows / columns k..k+nv-1) applied as H <- P H P and
// Z <- Z P: rows k.. over columns [c0, m), then columns k.. over rows [0, rmax], and Z's columns
// (thread r owns row r of Z).  Barriers inside; every thread calls it.
__device__ void apply_reflector(double* H, int ld, int m, double* Z, int k, int nv, const double* v, double tau,
                                int c0, int rmax, int zero_col) {
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int c = c0 + tid; c < m; c += nth) {
    double h[3] = {0.0, 0.0, 0.0};
    double t = 0.0;
    for (int i = 0; i < nv; ++i) {
      h[i] = H[(k + i) * ld + c];
      t += v[i] * h[i];
    }
    t *= tau;
    for (int i = 0; i < nv; ++i) H[(k + i) * ld + c] = h[i] - t * v[i];
    // the column the bulge came from keeps only its new subdiagonal entry
    if (c == zero_col)
      for (int i = 1; i < nv; ++i) H[(k + i) * ld + c] = 0.0;
  }
  __syncthreads();
  for (int r = tid; r <= rmax; r += nth) {
    double h[3] = {0.0, 0.0, 0.0};
    double t = 0.0;
    for (int i = 0; i < nv; ++i) {
      h[i] = H[r * ld + k + i];
      t += h[i] * v[i];
    }
    t *= tau;
    for (int i = 0; i < nv; ++i) H[r * ld + k + i] = h[i] - t * v[i];
  }
  for (int r = tid; r < m; r += nth) {
    double z[3] = {0.0, 0.0, 0.0};
    double t = 0.0;
    for (int i = 0; i < nv; ++i) {
      z[i] = Z[r * m + k + i];
      t += z[i] * v[i];
    }
    t *= tau;
    for (int i = 0; i < nv; ++i) Z[r * m + k + i] = z[i] - t * v[i];
  }
  __syncthreads();
}

// Plane rotation G = [[cs, -sn], [sn, cs]] on indices (p, p+1): H <- G^T H G (rows over columns
// [p, m), columns over rows [0, p+1]), Z <- Z G.
__device__ void apply_rotation(double* H, int ld, int m, double* Z, int p, double cs, double sn) {
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int c = p + tid; c < m; c += nth) {
    const double a = H[p * ld + c], b = H[(p + 1) * ld + c];
    H[p * ld + c] = cs * a + sn * b;
    H[(p + 1) * ld + c] = -sn * a + cs * b;
  }
  __syncthreads();
  for (int r = tid; r <= p + 1; r += nth) {
    const double a = H[r * ld + p], b = H[r * ld + p + 1];
    H[r * ld + p] = cs * a + sn * b;
    H[r * ld + p + 1] = -sn * a + cs * b;
  }
  for (int r = tid; r < m; r += nth) {
    const double a = Z[r * m + p], b = Z[r * m + p + 1];
    Z[r * m + p] = cs * a + sn * b;
    Z[r * m + p + 1] = -sn * a + cs * b;
  }
  __syncthreads();
}

// Real Schur form of the upper Hessenberg H (LDS) by the Francis double-shift QR iteration
// with deflation on negligible subdiagonal entries; the orthogonal factor accumulates into Z.
// A 2 x 2 diagonal block with real eigenvalues is split by a rotation, so on return every
// remaining 2 x 2 block holds a complex conjugate pair.  Returns 0, or 1 when an eigenvalue
// needed more than the iteration budget.  Every thread calls it; control flow is uniform
// (all threads read the same LDS values after a barrier).
__device__ int francis_schur(double* H, int ld, int m, double* Z, double* red) {
  const int tid = threadIdx.x;
  double hn = 0.0;
  for (int idx = tid; idx < m * m; idx += blockDim.x) hn = fmax(hn, fabs(H[(idx / m) * ld + idx % m]));
  hn = block_max(hn, red);
  int hi = m - 1, it = 0, total = 0;
  while (hi >= 0) {
    __syncthreads();
    int l = hi;
    while (l > 0) {
      double s = fabs(H[(l - 1) * ld + l - 1]) + fabs(H[l * ld + l]);
      if (s == 0.0) s = hn;
      if (fabs(H[l * ld + l - 1]) <= kEps * s) break;
      --l;
    }
    __syncthreads();
    if (l > 0 && tid == 0) H[l * ld + l - 1] = 0.0;
    __syncthreads();
    if (l == hi) {
      --hi;
      it = 0;
      continue;
    }
    if (l == hi - 1) {
      // 2 x 2 block [[a, b], [c, d]]: real eigenvalues are split off by the rotation whose
      // first column is the eigenvector (lam1 - d, c) of lam1 = d + p + sign(p) sqrt(disc)
      const double a = H[(hi - 1) * ld + hi - 1], b = H[(hi - 1) * ld + hi];
      const double c = H[hi * ld + hi - 1], d = H[hi * ld + hi];
      const double p = 0.5 * (a - d), disc = p * p + b * c;
      if (disc >= 0.0 && c != 0.0) {
        const double sq = sqrt(disc);
        const double lam1 = d + p + (p >= 0.0 ? sq : -sq);
        const double v0 = lam1 - d, v1 = c;
        const double nv = hypot(v0, v1);
        apply_rotation(H, ld, m, Z, hi - 1, v0 / nv, v1 / nv);
        if (tid == 0) H[hi * ld + hi - 1] = 0.0;
      }
      hi -= 2;
      it = 0;
      continue;
    }
    ++it;
    if (++total > 30 * m) return 1;
    double s, t;
    if (it % 10 == 0) {
      // exceptional shift after every ten sweeps without a deflation
      const double w = fabs(H[hi * ld + hi - 1]) + (hi - 2 >= l ? fabs(H[(hi - 1) * ld + hi - 2]) : 0.0);
      s = 1.5 * w;
      t = w * w;
    } else {
      const double a11 = H[(hi - 1) * ld + hi - 1], a12 = H[(hi - 1) * ld + hi];
      const double a21 = H[hi * ld + hi - 1], a22 = H[hi * ld + hi];
      s = a11 + a22;
      t = a11 * a22 - a12 * a21;
    }
    // first column of (H - s1 I)(H - s2 I) restricted to rows l, l+1, l+2
    const double h00 = H[l * ld + l], h01 = H[l * ld + l + 1], h10 = H[(l + 1) * ld + l];
    const double h11 = H[(l + 1) * ld + l + 1], h21 = H[(l + 2) * ld + l + 1];
    double x = h00 * h00 + h01 * h10 - s * h00 + t;
    double y = h10 * (h00 + h11 - s);
    double z = h10 * h21;
    for (int k = l; k <= hi - 2; ++k) {
      double v[3];
      const double tau = reflector3(x, y, z, v);
      if (tau != 0.0)
        apply_reflector(H, ld, m, Z, k, 3, v, tau, k > l ? k - 1 : l, min(k + 3, hi), k > l ? k - 1 : -1);
      x = H[(k + 1) * ld + k];
      y = H[(k + 2) * ld + k];
      z = k < hi - 2 ? H[(k + 3) * ld + k] : 0.0;
      __syncthreads();
    }
    {
      double v[3];
      const double tau = reflector3(x, y, 0.0, v);
      const int k = hi - 1;
      if (tau != 0.0) apply_reflector(H, ld, m, Z, k, 2, v, tau, k - 1, hi, k - 1);
    }
  }
  __syncthreads();
  return 0;
}

// Complex helpers on (re, im) pairs held in registers.
struct cx {
  double r, i;
};
__device__ inline cx cx_mul(cx a, cx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline cx cx_div(cx a, cx b) {
  // Smith's algorithm (no overflow in the squared modulus)
  if (fabs(b.r) >= fabs(b.i)) {
    const double q = b.i / b.r, d = b.r + b.i * q;
    return {(a.r + a.i * q) / d, (a.i - a.r * q) / d};
  }
  const double q = b.r / b.i, d = b.r * q + b.i;
  return {(a.r * q + a.i) / d, (a.i * q - a.r) / d};
}

// Eigenvectors of the quasi-triangular T (LDS) by back substitution, one wave per eigenvalue
// block: real lambda at k: y_k = 1 and (T - lambda I) y = 0 solved upwards; a pair at (k, k+1)
// (a -+ ib, b > 0): the block's eigenvector (T[k][k+1], lambda - T[k][k]) for lambda = a + ib,
// then the same recurrence in complex arithmetic.  2 x 2 blocks above are solved as 2 x 2
// systems; near-singular pivots are raised to smin.  Lane l keeps the right-hand sides of rows
// l and l + 64 in registers.  Y (global, m x m): column k (real) or columns k, k+1 (Re, Im).
__device__ void schur_eigvecs(const double* T, int ld, int m, const int* typ, const double* lre, const double* lim,
                              double tnorm, double* Y) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int k = wave; k < m; k += nw) {
    if (typ[k] == 2) continue;
    const bool pair = typ[k] == 1;
    const cx lam = pair ? cx{lre[k + 1], lim[k + 1]} : cx{lre[k], 0.0};
    const double smin = fmax(kEps * (sqrt(lam.r * lam.r + lam.i * lam.i) + tnorm), 1e-290);
    cx yk = {1.0, 0.0}, yk1 = {0.0, 0.0};
    if (pair) {
      yk = {T[k * ld + k + 1], 0.0};
      yk1 = {lam.r - T[k * ld + k], lam.i};
    }
    // right-hand sides of the rows above the block: -(T[r][k] y_k + T[r][k+1] y_{k+1})
    cx acc[2];
    for (int h = 0; h < 2; ++h) {
      const int r = lane + 64 * h;
      cx v = {0.0, 0.0};
      if (r < k) {
        v.r = -T[r * ld + k] * yk.r;
        v.i = -T[r * ld + k] * yk.i;
        if (pair) {
          v.r -= T[r * ld + k + 1] * yk1.r;
          v.i -= T[r * ld + k + 1] * yk1.i;
        }
      }
      acc[h] = v;
    }
    // the column(s) of Y from the block down (the rows above are written as they are solved)
    for (int r = k + lane; r < m; r += 64) {
      double re = 0.0, im = 0.0;
      if (r == k) {
        re = yk.r;
        im = yk.i;
      } else if (pair && r == k + 1) {
        re = yk1.r;
        im = yk1.i;
      }
      Y[r * m + k] = re;
      if (pair) Y[r * m + k + 1] = im;
    }
    auto get = [&](int r) -> cx {
      const int h = r >> 6;  // uniform
      const cx v = h == 0 ? acc[0] : acc[1];
      return {lane_bcast(v.r, r & 63), lane_bcast(v.i, r & 63)};
    };
    int i = k - 1;
    while (i >= 0) {
      if (typ[i] == 2) {
        // rows (i-1, i): [[t11 - lam, t12], [t21, t22 - lam]] y = rhs
        const cx r1 = get(i - 1), r2 = get(i);
        const cx a11 = {T[(i - 1) * ld + i - 1] - lam.r, -lam.i}, a22 = {T[i * ld + i] - lam.r, -lam.i};
        const double a12 = T[(i - 1) * ld + i], a21 = T[i * ld + i - 1];
        cx det = cx_mul(a11, a22);
        det.r -= a12 * a21;
        if (sqrt(det.r * det.r + det.i * det.i) < smin) det = {smin, 0.0};
        cx t1 = cx_mul(r1, a22);
        t1.r -= a12 * r2.r;
        t1.i -= a12 * r2.i;
        cx t2 = cx_mul(a11, r2);
        t2.r -= a21 * r1.r;
        t2.i -= a21 * r1.i;
        const cx y1 = cx_div(t1, det), y2 = cx_div(t2, det);
        for (int h = 0; h < 2; ++h) {
          const int r = lane + 64 * h;
          if (r < i - 1) {
            const double c1 = T[r * ld + i - 1], c2 = T[r * ld + i];
            acc[h].r -= c1 * y1.r + c2 * y2.r;
            acc[h].i -= c1 * y1.i + c2 * y2.i;
          }
        }
        if (lane == 0) {
          Y[(i - 1) * m + k] = y1.r;
          Y[i * m + k] = y2.r;
          if (pair) {
            Y[(i - 1) * m + k + 1] = y1.i;
            Y[i * m + k + 1] = y2.i;
          }
        }
        i -= 2;
      } else {
        const cx rhs = get(i);
        cx den = {T[i * ld + i] - lam.r, -lam.i};
        if (sqrt(den.r * den.r + den.i * den.i) < smin) den = {smin, 0.0};
        const cx yi = cx_div(rhs, den);
        for (int h = 0; h < 2; ++h) {
          const int r = lane + 64 * h;
          if (r < i) {
            const double c = T[r * ld + i];
            acc[h].r -= c * yi.r;
            acc[h].i -= c * yi.i;
          }
        }
        if (lane == 0) {
          Y[i * m + k] = yi.r;
          if (pair) Y[i * m + k + 1] = yi.i;
        }
        i -= 1;
      }
    }
  }
}

// Products of m x m matrices (global, row-major) with up to 16 outputs per thread of 1024.
__device__ void small_gemm(int m, const double* A, bool transA, const double* B, double* C, const int* bcol) {
  const int mm = m * m;
  for (int idx = threadIdx.x; idx < mm; idx += blockDim.x) {
    const int r = idx / m, c = idx % m;
    const int cb = bcol != nullptr ? bcol[c] : c;
    double s = 0.0;
    if (transA)
      for (int e = 0; e < m; ++e) s += A[e * m + r] * B[e * m + cb];
    else
      for (int e = 0; e < m; ++e) s += A[r * m + e] * B[e * m + cb];
    C[idx] = s;
  }
}

// One SVQB orthonormalisation pass on a block P (n x m0) from its Gram G = P^T P: G scaled to a
// unit diagonal, D G D = U Theta U^T, Theta floored at eps m0 max Theta, T = D U Theta^{-1/2}, so
// P T is orthonormal on the directions the Gram resolves.  Tacc (m0 x m0) <- Tacc T (first pass:
// Tacc = T).  work (global): 3 m0^2 doubles.  LDS: m0^2 doubles + the static arrays.
__global__ __launch_bounds__(1024) void k_svqb_pass(int m0, const double* __restrict__ G, double* __restrict__ T,
                                                   double* __restrict__ Tacc, int first, double* __restrict__ work) {
  extern __shared__ double sm[];
  __shared__ double red[32];
  __shared__ double dsc[128], th[128];
  const int tid = threadIdx.x, nth = blockDim.x, m = m0, mm = m0 * m0;
  double* U = work;
  double* save = work + mm;
  double* Hv = work + 2 * mm;
  for (int a = tid; a < m; a += nth) {
    const double d = G[a * m + a];
    dsc[a] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
  }
  __syncthreads();
  for (int idx = tid; idx < mm; idx += nth) {
    const int r = idx / m, c = idx % m;
    sm[idx] = 0.5 * (G[r * m + c] + G[c * m + r]) * dsc[r] * dsc[c];
  }
  __syncthreads();
  sym_eig_ql(sm, m, U, red, Hv, save);
  double tmax = 0.0;
  for (int a = tid; a < m; a += nth) tmax = fmax(tmax, sm[a * m + a]);
  tmax = block_max(tmax, red);
  for (int a = tid; a < m; a += nth) th[a] = 1.0 / sqrt(fmax(sm[a * m + a], kEps * m * tmax));
  __syncthreads();
  for (int idx = tid; idx < mm; idx += nth) {
    const int r = idx / m, c = idx % m;
    T[idx] = dsc[r] * U[idx] * th[c];
  }
  __syncthreads();
  if (first) {
    for (int idx = tid; idx < mm; idx += nth) Tacc[idx] = T[idx];
    return;
  }
  // Tacc T staged in LDS, then written over Tacc
  for (int idx = tid; idx < mm; idx += nth) {
    const int r = idx / m, c = idx % m;
    double s = 0.0;
    for (int e = 0; e < m; ++e) s += Tacc[r * m + e] * T[e * m + c];
    sm[idx] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < mm; idx += nth) Tacc[idx] = sm[idx];
}

// Reduced problem of the non-Hermitian Rayleigh-Ritz step on an orthonormal basis P = Q Tacc of
// span(Q): GA = P^T A P (m0 x m0, FP64), Tacc the transform from Q, GX = X^T X of the filtered
// block (null: identity).  Real Schur form GA = Z S Z^T, eigenvectors W = Z Y of unit 2-norm
// (pairs: ||W_j||^2 + ||W_{j+1}||^2 = 1), ascending by real part.  Outputs: lam, lam_im (pair
// format), W (X = P W), C = Tacc W (X = Q C), eta_l = 1 / ||X c_l|| (pairs: over both columns).
// A Schur iteration that does not converge leaves NaN in lam[0].
// work (global): 6 m0^2 doubles.  LDS: m0 (m0 + 1) doubles + the static arrays.
__global__ __launch_bounds__(1024) void k_rr_general(int m0, const double* __restrict__ GA,
                                                    const double* __restrict__ Tacc, const double* __restrict__ GX,
                                                    double* __restrict__ lam, double* __restrict__ lam_im,
                                                    double* __restrict__ Wout, double* __restrict__ C,
                                                    double* __restrict__ eta, double* __restrict__ work) {
  extern __shared__ double sm[];
  __shared__ double red[32];
  __shared__ double th[128], lre[128], lim[128], nrm[128], vb[256], pb[128];
  __shared__ int typ[128], slot[128];
  const int tid = threadIdx.x, nth = blockDim.x, m = m0, mm = m0 * m0, ld = m0 + 1;
  const double* Tm = Tacc;
  double* Wt = work;
  double* Z = work + mm;
  double* Y = work + 2 * mm;
  double* Wv = work + 3 * mm;
  double* Ws = Wout;
  // 1. GA into LDS (stride ld)
  for (int idx = tid; idx < mm; idx += nth) {
    const int r = idx / m, c = idx % m;
    sm[r * ld + c] = GA[idx];
    Z[idx] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  // 2. Hessenberg form and real Schur form
  hessenberg_reduce(sm, ld, m, Z, red, vb, pb);
  const int fail = francis_schur(sm, ld, m, Z, red);
  if (fail) {
    if (tid == 0) lam[0] = __longlong_as_double(0x7ff8000000000000LL);
    return;
  }
  // 3. eigenvalues from the diagonal blocks
  for (int i = tid; i < m; i += nth) {
    const bool first = i + 1 < m && sm[(i + 1) * ld + i] != 0.0;
    const bool second = i > 0 && sm[i * ld + i - 1] != 0.0;
    typ[i] = first ? 1 : (second ? 2 : 0);
    if (first || second) {
      const int k = first ? i : i - 1;
      const double a = sm[k * ld + k], b = sm[k * ld + k + 1], c = sm[(k + 1) * ld + k], d = sm[(k + 1) * ld + k + 1];
      const double p = 0.5 * (a - d), disc = p * p + b * c;
      const double bi = sqrt(fmax(-disc, 0.0));
      lre[i] = 0.5 * (a + d);
      lim[i] = first ? -bi : bi;
    } else {
      lre[i] = sm[i * ld + i];
      lim[i] = 0.0;
    }
  }
  double tn = 0.0;
  for (int idx = tid; idx < mm; idx += nth) tn = fmax(tn, fabs(sm[(idx / m) * ld + idx % m]));
  tn = block_max(tn, red);
  __syncthreads();
  // 4. eigenvectors of S, then W = Z Y, unit 2-norm per real vector / per pair
  schur_eigvecs(sm, ld, m, typ, lre, lim, tn * m, Y);
  __syncthreads();
  small_gemm(m, Z, false, Y, Wv, nullptr);
  __syncthreads();
  for (int c = tid; c < m; c += nth) {
    double ss = 0.0;
    for (int r = 0; r < m; ++r) ss += Wv[r * m + c] * Wv[r * m + c];
    nrm[c] = ss;
  }
  __syncthreads();
  for (int c = tid; c < m; c += nth) {
    const double tot = typ[c] == 0 ? nrm[c] : (typ[c] == 1 ? nrm[c] + nrm[c + 1] : nrm[c - 1] + nrm[c]);
    th[c] = tot > 0.0 ? 1.0 / sqrt(tot) : 0.0;
  }
  __syncthreads();
  // 5. ascending order of the blocks by real part (ties by position); a pair takes two slots
  for (int b = tid; b < m; b += nth) {
    if (typ[b] == 2) continue;
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      if (typ[j] == 2) continue;
      if (lre[j] < lre[b] || (lre[j] == lre[b] && j < b)) rank += typ[j] == 1 ? 2 : 1;
    }
    slot[rank] = b;
    if (typ[b] == 1) slot[rank + 1] = b + 1;
  }
  __syncthreads();
  for (int idx = tid; idx < mm; idx += nth) {
    const int r = idx / m, c = idx % m;
    const int src = slot[c];
    Ws[idx] = Wv[r * m + src] * th[src];
  }
  for (int c = tid; c < m; c += nth) {
    lam[c] = lre[slot[c]];
    lam_im[c] = lim[slot[c]];
  }
  __syncthreads();
  // 6. C = Tacc W, gains from the filtered block's Gram
  small_gemm(m, Tm, false, Ws, C, nullptr);
  __syncthreads();
  if (GX != nullptr) {
    small_gemm(m, GX, false, C, Wt, nullptr);  // Wt = GX C
    __syncthreads();
  }
  for (int c = tid; c < m; c += nth) {
    double q = 0.0;
    for (int r = 0; r < m; ++r) q += C[r * m + c] * (GX != nullptr ? Wt[r * m + c] : C[r * m + c]);
    nrm[c] = q;
  }
  __syncthreads();
  for (int c = tid; c < m; c += nth) {
    const double li = lam_im[c];
    const double q = li < 0.0 ? nrm[c] + nrm[c + 1] : (li > 0.0 ? nrm[c - 1] + nrm[c] : nrm[c]);
    eta[c] = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  }
}

// ------------------------------------------------------- pair-aware elementwise
// R = A X - X Lambda_b (Lambda_b block diagonal: 2 x 2 blocks J for the pairs).
__global__ void k_residual_pairs(int64_t n, int m, const double* __restrict__ AX, const double* __restrict__ X,
                                 const double* __restrict__ lam, const double* __restrict__ lam_im,
                                 double* __restrict__ R) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int j = (int)(idx % m);
  const double li = lam_im[j];
  double v = AX[idx] - lam[j] * X[idx];
  if (li < 0.0) v -= li * X[idx + 1];       // + b x_{j+1}
  else if (li > 0.0) v -= li * X[idx - 1];  // - b x_{j-1}
  R[idx] = v;
}

// Residual norms of the complex eigenvectors: a pair's columns share sqrt(r_j^2 + r_{j+1}^2).
__global__ void k_pair_norms(int m, const double* __restrict__ lam_im, double* __restrict__ resid) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m || !(lam_im[j] < 0.0) || j + 1 >= m) return;
  const double v = hypot(resid[j], resid[j + 1]);
  resid[j] = v;
  resid[j + 1] = v;
}

// rho_hat(lambda) = sum_k w_k / (z_k - lambda) over every node of the rule (no 2 Re fold), for
// the eigenvalue a + ib of each column (a pair's two columns take the value at a + i|b|).
__global__ void k_rho_pairs(int m0, int nc, const double* __restrict__ z, const double* __restrict__ w,
                            const double* __restrict__ lam, const double* __restrict__ lam_im,
                            double* __restrict__ rho, double* __restrict__ rho_im) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m0) return;
  const double l = lam[j], li = fabs(lam_im[j]);
  double rr = 0.0, ri = 0.0;
  for (int k = 0; k < nc; ++k) {
    const double zr = z[2 * k] - l, zi = z[2 * k + 1] - li;
    const double d = zr * zr + zi * zi;
    rr += (w[2 * k] * zr + w[2 * k + 1] * zi) / d;
    ri += (w[2 * k + 1] * zr - w[2 * k] * zi) / d;
  }
  rho[j] = rr;
  rho_im[j] = lam_im[j] == 0.0 ? 0.0 : ri;
}

// Y = X rho_hat(Lambda_b): a pair's block is [[p, q], [-q, p]] with rho_hat(a + ib) = p + iq.
__global__ void k_scale_pairs(int64_t n, int m, const double* __restrict__ X, const double* __restrict__ rho,
                              const double* __restrict__ rho_im, const double* __restrict__ lam_im,
                              double* __restrict__ Y) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int j = (int)(idx % m);
  const double li = lam_im[j], p = rho[j], q = rho_im[j];
  double v = p * X[idx];
  if (li < 0.0) v -= q * X[idx + 1];
  else if (li > 0.0) v += q * X[idx - 1];
  Y[idx] = v;
}

// S_s = S0 (z_s I - Lambda_b)^{-1} per shift (S0 m0 x m0 complex row-major with zero imaginary
// parts, S ns x m0 x m0): a pair's 2 x 2 block inverse is [[z - a, b], [-b, z - a]] / d,
// d = (z - a)^2 + b^2.
__global__ void k_start_rhs_pairs(int ns, int m0, const double2* __restrict__ S0, const double* __restrict__ lam,
                                  const double* __restrict__ lam_im, const double* __restrict__ z,
                                  double2* __restrict__ S) {
  const int s = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns || idx >= m0 * m0) return;
  const int r = idx / m0, j = idx % m0;
  const cx zs = {z[2 * s], z[2 * s + 1]};
  const double li = lam_im[j];
  cx out;
  if (li == 0.0) {
    out = cx_div({S0[idx].x, S0[idx].y}, {zs.r - lam[j], zs.i});
  } else {
    const double b = fabs(li);
    const cx zma = {zs.r - lam[j], zs.i};
    cx d = cx_mul(zma, zma);
    d.r += b * b;
    const int j0 = li < 0.0 ? j : j - 1;  // the pair's first (real-part) column
    const cx s0 = {S0[r * m0 + j0].x, S0[r * m0 + j0].y}, s1 = {S0[r * m0 + j0 + 1].x, S0[r * m0 + j0 + 1].y};
    cx num;
    if (li < 0.0) {  // column j0: s0 (z - a) - s1 b
      num = cx_mul(s0, zma);
      num.r -= s1.r * b;
      num.i -= s1.i * b;
    } else {  // column j0 + 1: s0 b + s1 (z - a)
      num = cx_mul(s1, zma);
      num.r += s0.r * b;
      num.i += s0.i * b;
    }
    out = cx_div(num, d);
  }
  S[(int64_t)s * m0 * m0 + idx] = make_double2(out.r, out.i);
}

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_svqb_pass(hipStream_t st, int m0, const double* G, double* T, double* Tacc, int first, double* work) {
  IF_REQUIRE(m0 >= 2 && m0 <= 128, "svqb: m0 must be in [2, 128]");
  const size_t lds = (size_t)m0 * m0 * sizeof(double);
  if (lds > 64 * 1024)
    IF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_svqb_pass), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
  hipLaunchKernelGGL(k_svqb_pass, dim3(1), dim3(1024), lds, st, m0, G, T, Tacc, first, work);
  IF_HIP(hipGetLastError());
}

void launch_rr_general(hipStream_t st, int m0, const double* GA, const double* Tacc, const double* GX, double* lam,
                       double* lam_im, double* W, double* C, double* eta, double* work) {
  IF_REQUIRE(m0 >= 2 && m0 <= 128, "rayleigh-ritz: m0 must be in [2, 128]");
  const size_t lds = (size_t)m0 * (m0 + 1) * sizeof(double);
  if (lds > 64 * 1024)
    IF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_rr_general), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
  hipLaunchKernelGGL(k_rr_general, dim3(1), dim3(1024), lds, st, m0, GA, Tacc, GX, lam, lam_im, W, C, eta, work);
  IF_HIP(hipGetLastError());
}

void launch_residual_pairs(hipStream_t st, int64_t n, int m, const double* AX, const double* X, const double* lam,
                           const double* lam_im, double* R) {
  const int64_t tot = n * m;
  hipLaunchKernelGGL(k_residual_pairs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, m, AX, X, lam, lam_im,
                     R);
  IF_HIP(hipGetLastError());
}

void launch_pair_norms(hipStream_t st, int m, const double* lam_im, double* resid) {
  hipLaunchKernelGGL(k_pair_norms, dim3((m + 127) / 128), dim3(128), 0, st, m, lam_im, resid);
  IF_HIP(hipGetLastError());
}

void launch_rho_pairs(hipStream_t st, int m0, int nc, const double* z, const double* w, const double* lam,
                      const double* lam_im, double* rho, double* rho_im) {
  hipLaunchKernelGGL(k_rho_pairs, dim3((m0 + 127) / 128), dim3(128), 0, st, m0, nc, z, w, lam, lam_im, rho, rho_im);
  IF_HIP(hipGetLastError());
}

void launch_scale_pairs(hipStream_t st, int64_t n, int m, const double* X, const double* rho, const double* rho_im,
                        const double* lam_im, double* Y) {
  const int64_t tot = n * m;
  hipLaunchKernelGGL(k_scale_pairs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, m, X, rho, rho_im,
                     lam_im, Y);
  IF_HIP(hipGetLastError());
}

void launch_start_rhs_pairs(hipStream_t st, int ns, int m0, const cd* S0, const double* lam, const double* lam_im,
                            const double* z, cd* S) {
  const int mm = m0 * m0;
  hipLaunchKernelGGL(k_start_rhs_pairs, dim3((mm + 255) / 256, ns), dim3(256), 0, st, ns, m0,
                     reinterpret_cast<const double2*>(S0), lam, lam_im, z, reinterpret_cast<double2*>(S));
  IF_HIP(hipGetLastError());
}

}  // namespace ifeast
