// Kernels of the shared-basis inner solve (standard problems, B = I).
//
// For B = I the block Krylov space of z_s I - A from the right-hand side
// R (z_s - Lambda)^{-1} is that of A from R for every shift z_s: a diagonal
// scaling of the block's columns and a shift of the operator leave the block
// Krylov space unchanged (Sec. 3.2 solves each shifted system from B X or its
// residual form; the spaces coincide).  One real block Arnoldi
//     M V_j = V_{j+1} Hm,   M = -A
// therefore serves all shifts: (z_s I - A) V_j = V_{j+1} (z_s I~ + Hm), and only
// the small least-squares problems, with right-hand sides [S0 D_s; 0], differ
// per shift.  The helpers below move data between the shared real block
// Hessenberg Hm and the per-shift complex ones the least-squares kernels use.
#include "internal.h"

namespace ifeast {

namespace {

typedef double2 c2;
__device__ inline c2 cmk(double r, double i) { return make_double2(r, i); }
__device__ inline c2 cmul(c2 a, c2 b) { return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline c2 cdiv(c2 a, c2 b) {
  const double d = b.x * b.x + b.y * b.y;
  return cmk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

inline unsigned nblk(int64_t total) { return (unsigned)((total + 255) / 256); }

template <class T>
__global__ void k_to_T(int64_t count, const double* __restrict__ X, T* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) Y[i] = (T)X[i];
}

// Estimated loss of orthogonality of the projected block W against the older basis blocks:
// max over columns b of ||G[:, b]|| / ||w_b|| with G = U^T W (nk x m0, row-major) the
// sketch product and ||w_b||^2 the diagonal of gw = W^T W; out[0] = that maximum (NaN
// when some column is not finite).  One workgroup of 128 threads.
__global__ __launch_bounds__(128) void k_sketch_check_real(int nk, int m0, const double* __restrict__ G,
                                                           const double* __restrict__ gw, double* __restrict__ out) {
  __shared__ double red[2];
  double r = 0.0;
  for (int b = threadIdx.x; b < m0; b += blockDim.x) {
    double ss = 0.0;
    for (int a = 0; a < nk; ++a) ss += G[a * m0 + b] * G[a * m0 + b];
    const double d = gw[b * m0 + b];
    const double v = d > 0.0 ? sqrt(ss / d) : (ss > 0.0 ? INFINITY : 0.0);
    r = (v > r || v != v) ? v : r;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double t = __shfl_xor(r, o);
    r = (t > r || t != t) ? t : r;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[1] > red[0] || red[1] != red[1]) ? red[1] : red[0];
}

// Gram of the block after a projection W2 = W1 - V C with orthonormal V: W2^T W2 =
// W1^T W1 - C^T C.  gw (m0 x m0) holds W1^T W1 on entry; C has `rows` rows of m0.
// One workgroup per 16 x 16 tile of gw; rows staged through LDS 160 at a time.
__global__ __launch_bounds__(256) void k_gram_downdate(int rows, int m0, const double* __restrict__ C,
                                                       double* __restrict__ gw, const int* __restrict__ active) {
  if (active != nullptr && active[0] == 0) return;
  // chunks of KR rows: the two-block case (2 x 80 rows) is one chunk, so its loads overlap
  constexpr int KR = 160;
  __shared__ double ca[KR][17], cb[KR][17];
  const int nt = (m0 + 15) / 16;
  const int ta = blockIdx.x / nt, tb = blockIdx.x % nt;
  const int a0 = ta * 16, b0 = tb * 16;
  const int tid = threadIdx.x, ia = tid >> 4, ib = tid & 15;
  double acc = 0.0;
  for (int r0 = 0; r0 < rows; r0 += KR) {
    for (int idx = tid; idx < KR * 16; idx += 256) {
      const int r = idx >> 4, c = idx & 15;
      const bool in = r0 + r < rows;
      ca[r][c] = (in && a0 + c < m0) ? C[(int64_t)(r0 + r) * m0 + a0 + c] : 0.0;
      cb[r][c] = (in && b0 + c < m0) ? C[(int64_t)(r0 + r) * m0 + b0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < KR; ++r) acc += ca[r][ia] * cb[r][ib];
    __syncthreads();
  }
  if (a0 + ia < m0 && b0 + ib < m0) gw[(a0 + ia) * m0 + b0 + ib] -= acc;
}

// Hm block (j+1, j) = R factor of the new block (real part of Racc, upper triangular).
__global__ void k_subdiag_real(int m0, int j, int ldh, const c2* __restrict__ Racc, double* __restrict__ Hm) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m0 * m0) return;
  const int a = idx / m0, b = idx % m0;
  Hm[(int64_t)(j * m0 + b) * ldh + (j + 1) * m0 + a] = Racc[idx].x;
}

// Block column j of every active shift's Hbar_s = z_s I~ + Hm (rows 0..(j+2) m0).
// grid (ns, m0); one workgroup per (shift, column).
// band > 0: rows above block row j - band are taken as zero (for symmetric A the
// orthogonalisation coefficients there vanish in exact arithmetic: block Lanczos).
__global__ void k_shift_column(int m0, int j, int ldh, int kcap, const double* __restrict__ z,
                               const int* __restrict__ active, const double* __restrict__ Hm, c2* __restrict__ H,
                               int band) {
  const int s = blockIdx.x, c = blockIdx.y;
  if (active[s] == 0) return;
  const int col = j * m0 + c;
  const double* src = Hm + (int64_t)col * ldh;
  c2* dst = H + (int64_t)s * ldh * kcap * m0 + (int64_t)col * ldh;
  const double zr = z[2 * s], zi = z[2 * s + 1];
  const int r0 = band > 0 ? max(0, j - band) * m0 : 0;
  for (int r = threadIdx.x; r < (j + 2) * m0; r += blockDim.x)
    dst[r] = r < r0 ? cmk(0.0, 0.0) : (r == col) ? cmk(src[r] + zr, zi) : cmk(src[r], 0.0);
}

// Right-hand side of shift s in the basis: S_s = S0 diag(1 / (z_s - lambda_c)), row-major.
__global__ void k_start_rhs(int ns, int m0, const c2* __restrict__ S0, const double* __restrict__ lam,
                            const double* __restrict__ z, c2* __restrict__ S) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)ns * m0 * m0) return;
  const int s = (int)(idx / ((int64_t)m0 * m0));
  const int rc = (int)(idx % ((int64_t)m0 * m0));
  const int c = rc % m0;
  S[idx] = cdiv(cmk(S0[rc].x, 0.0), cmk(z[2 * s] - lam[c], z[2 * s + 1]));
}

// Yr[b] (m0 x m0, type T, row k = basis column, column o) = Re sum_s wf_s y_s[b m0 + k][o]
// for b < jmax: Q += V_b Yr[b] is the quadrature sum's correction.
template <class T>
__global__ void k_sum_y(int ns, int m0, int kcap, int jmax, const c2* __restrict__ y, const double* __restrict__ wf,
                        T* __restrict__ Yr) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)jmax * m0 * m0) return;
  const int b = (int)(idx / ((int64_t)m0 * m0));
  const int k = (int)((idx / m0) % m0), o = (int)(idx % m0);
  const int64_t ldy = (int64_t)kcap * m0;
  double acc = 0.0;
  for (int s = 0; s < ns; ++s) {
    const c2 v = y[(int64_t)s * kcap * m0 * m0 + o * ldy + b * m0 + k];
    acc += wf[2 * s] * v.x - wf[2 * s + 1] * v.y;
  }
  Yr[idx] = (T)acc;
}

// Loss of orthogonality a first Gram-Schmidt pass left in W against the local blocks:
// max over columns b of ||G2[:, b]|| / ||w_b|| with G2 = [V_lo..]^T W (rows x m0) and
// ||w_b||^2 the diagonal of gw = W^T W.  act[0] = act[1] = (that loss > eta, or not finite): the
// second pass is needed; act[2] = 1 (W's own term).  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_local_loss(int rows, int m0, const double* __restrict__ G2,
                                                     const double* __restrict__ gw, double eta, int* __restrict__ act) {
  // column b's sum of squares in 1024 / m0 row slices (coalesced: consecutive threads, consecutive
  // columns), combined in LDS; the slice sums are added in a fixed order
  __shared__ double part[1024];
  __shared__ double colr[128];
  const int t = threadIdx.x, ns = 1024 / m0;
  const int b = t % m0, sl = t / m0;
  // (the loops are unrolled so that their loads are in flight together; each thread's sum keeps
  // its order)
  double g2 = 0.0;
  if (sl < ns) {
#pragma unroll 8
    for (int a = sl; a < rows; a += ns) g2 += G2[(int64_t)a * m0 + b] * G2[(int64_t)a * m0 + b];
  }
  part[t] = g2;
  __syncthreads();
  if (t < m0) {
    double sum = 0.0;
    for (int k = 0; k < ns; ++k) sum += part[k * m0 + t];
    const double w2 = gw[(int64_t)t * m0 + t];
    colr[t] = w2 > 0.0 ? sum / w2 : (sum > 0.0 ? INFINITY : 0.0);
  }
  __syncthreads();
  if (t == 0) {
    double mx = 0.0;
    for (int c = 0; c < m0; ++c) mx = (colr[c] > mx || colr[c] != colr[c]) ? colr[c] : mx;
    const int need = mx <= eta * eta ? 0 : 1;
    act[0] = need;
    act[1] = need;
    act[2] = 1;
  }
}

// The three device decisions of a shared-basis step in one launch (one workgroup of 1024 threads),
// all from the step's Grams with gw = W^T W:
//  * sketch (Gsk = U^T W, nk x m0, may be null): out[0] = max_b ||Gsk[:, b]|| / ||w_b|| (NaN when
//    some column is not finite), as k_sketch_check_real;
//  * Gershgorin certificate of gw: single[0] / two[0] / count[0], as k_gersh_flags;
//  * local loss (G2 = [V_lo..]^T W, rows x m0): act[0] = act[1] = (loss > eta), act[2] = 1, as
//    k_local_loss.
__global__ __launch_bounds__(1024) void k_step_checks(int nk, int m0, const double* __restrict__ Gsk,
                                                      const double* __restrict__ gw, double gersh, double dead_thr,
                                                      int* __restrict__ single, int* __restrict__ two,
                                                      int* __restrict__ count, int rows, const double* __restrict__ G2,
                                                      double eta, int* __restrict__ act, double* __restrict__ out) {
  __shared__ double dsc[128], colr[128], colk[128];
  __shared__ double part[1024];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  __syncthreads();
  // column norms of gw; the local loss's and the sketch's column sums of squares beside them
  const int ns = 1024 / m0;
  const int b = t % m0, sl = t / m0;
  // (the loops are unrolled so that their loads are in flight together; each thread's sum keeps
  // its order)
  double g2 = 0.0;
  if (sl < ns) {
#pragma unroll 8
    for (int a = sl; a < rows; a += ns) g2 += G2[(int64_t)a * m0 + b] * G2[(int64_t)a * m0 + b];
  }
  part[t] = g2;
  if (t < m0) {
    const double d = gw[t * m0 + t];
    if (!(d > dead_thr)) bad = 1;
    dsc[t] = sqrt(fmax(d, 1e-300));
    if (Gsk != nullptr) {
      double ss = 0.0;
#pragma unroll 16
      for (int a = 0; a < nk; ++a) ss += Gsk[a * m0 + t] * Gsk[a * m0 + t];
      colk[t] = d > 0.0 ? sqrt(ss / d) : (ss > 0.0 ? INFINITY : 0.0);
    }
  }
  __syncthreads();
  // Gershgorin: 8 lanes per row of the scaled Gram
  const int r = t >> 3, pp = t & 7;
  double off = 0.0;
  if (r < m0) {
#pragma unroll 8
    for (int c = pp; c < m0; c += 8)
      if (c != r) off += fabs(gw[r * m0 + c]) / (dsc[r] * dsc[c]);
  }
  off += __shfl_xor(off, 1);
  off += __shfl_xor(off, 2);
  off += __shfl_xor(off, 4);
  if (r < m0 && pp == 0 && !(off <= gersh)) bad = 1;
  if (t < m0) {
    double sum = 0.0;
    for (int k = 0; k < ns; ++k) sum += part[k * m0 + t];
    const double w2 = gw[(int64_t)t * m0 + t];
    colr[t] = w2 > 0.0 ? sum / w2 : (sum > 0.0 ? INFINITY : 0.0);
  }
  __syncthreads();
  if (t < 64) {
    // wave 0: the largest column loss and sketched estimate over the lanes, then across them (a
    // NaN wins, so that a check that went wrong asks for the extra pass)
    auto nanmax = [](double a, double b) { return (b > a || b != b) ? b : a; };
    double mx = 0.0, mk = 0.0;
    for (int c = t; c < m0; c += 64) {
      mx = nanmax(mx, colr[c]);
      if (Gsk != nullptr) mk = nanmax(mk, colk[c]);
    }
    for (int o = 32; o >= 1; o >>= 1) {
      mx = nanmax(mx, __shfl_xor(mx, o));
      mk = nanmax(mk, __shfl_xor(mk, o));
    }
    if (t == 0) {
      single[0] = bad ? 0 : 1;
      two[0] = bad ? 1 : 0;
      if (count != nullptr) count[0] += bad ? 0 : 1;
      const int need = mx <= eta * eta ? 0 : 1;
      act[0] = need;
      act[1] = need;
      act[2] = 1;
      if (Gsk != nullptr) out[0] = mk;
    }
  }
}

// The second Gram-Schmidt pass folded into the normalisation.  With G2 = [V_lo..V_{lo+nl-1}]^T W
// the second pass's coefficients and R^{-1} = Tinv the Cholesky-QR factor of
// (W - V G2)^T (W - V G2) = W^T W - G2^T G2, the next block is
//     V_{j+1} = (W - V G2) Tinv = V (-G2 Tinv) + W Tinv,
// one product over [V_lo.., W] with the stacked coefficients written here:
// Cf[b] = -G2_b Tinv (b < nl) and Cf[nl] = Tinv; also G2T = G2 in type T and Hm += G2 (block rows
// lo.. of block column j, as the second pass accumulates its coefficients).
// G2: nl blocks m0 x m0 row-major (FP64); Tinv: m0 x m0 row-major, upper triangular.
template <class T>
__global__ void k_fold_second_pass(int m0, int nl, const double* __restrict__ G2, const T* __restrict__ Tinv,
                                   T* __restrict__ Cf, T* __restrict__ G2T, double* __restrict__ Hm, int ldh, int j,
                                   int lo, const int* __restrict__ need) {
  const int64_t mm = (int64_t)m0 * m0;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (nl + 1) * mm) return;
  const int b = (int)(idx / mm), a = (int)((idx % mm) / m0), q = (int)(idx % m0);
  if (b == nl) {
    Cf[idx] = Tinv[a * m0 + q];
    return;
  }
  if (need != nullptr && need[0] == 0) return;  // no second pass: W itself is normalised
  const double* g = G2 + b * mm + (int64_t)a * m0;
  double acc = 0.0;
  for (int k = 0; k <= q; ++k) acc += g[k] * (double)Tinv[k * m0 + q];
  Cf[idx] = (T)(-acc);
  G2T[idx] = (T)g[q];
  Hm[(int64_t)(j * m0 + q) * ldh + (int64_t)(lo + b) * m0 + a] += g[q];
}

}  // namespace

template <class T>
void launch_to_T(hipStream_t st, int64_t count, const double* X, T* Y) {
  hipLaunchKernelGGL((k_to_T<T>), dim3(nblk(count)), dim3(256), 0, st, count, X, Y);
  IF_HIP(hipGetLastError());
}
void launch_sketch_check_real(hipStream_t st, int nk, int m0, const double* G, const double* gw, double* out) {
  hipLaunchKernelGGL(k_sketch_check_real, dim3(1), dim3(128), 0, st, nk, m0, G, gw, out);
  IF_HIP(hipGetLastError());
}
void launch_gram_downdate(hipStream_t st, int rows, int m0, const double* C, double* gw, const int* active) {
  const int nt = (m0 + 15) / 16;
  hipLaunchKernelGGL(k_gram_downdate, dim3(nt * nt), dim3(256), 0, st, rows, m0, C, gw, active);
  IF_HIP(hipGetLastError());
}
void launch_subdiag_real(hipStream_t st, int m0, int j, int ldh, const cd* Racc, double* Hm) {
  hipLaunchKernelGGL(k_subdiag_real, dim3(nblk((int64_t)m0 * m0)), dim3(256), 0, st, m0, j, ldh,
                     reinterpret_cast<const c2*>(Racc), Hm);
  IF_HIP(hipGetLastError());
}
void launch_shift_column(hipStream_t st, int ns, int m0, int j, int ldh, int kcap, const double* z, const int* active,
                         const double* Hm, cd* H, int band) {
  hipLaunchKernelGGL(k_shift_column, dim3(ns, m0), dim3(256), 0, st, m0, j, ldh, kcap, z, active, Hm,
                     reinterpret_cast<c2*>(H), band);
  IF_HIP(hipGetLastError());
}
void launch_start_rhs(hipStream_t st, int ns, int m0, const cd* S0, const double* lam, const double* z, cd* S) {
  hipLaunchKernelGGL(k_start_rhs, dim3(nblk((int64_t)ns * m0 * m0)), dim3(256), 0, st, ns, m0,
                     reinterpret_cast<const c2*>(S0), lam, z, reinterpret_cast<c2*>(S));
  IF_HIP(hipGetLastError());
}
template <class T>
void launch_sum_y(hipStream_t st, int ns, int m0, int kcap, int jmax, const cd* y, const double* wf, T* Yr) {
  hipLaunchKernelGGL((k_sum_y<T>), dim3(nblk((int64_t)jmax * m0 * m0)), dim3(256), 0, st, ns, m0, kcap, jmax,
                     reinterpret_cast<const c2*>(y), wf, Yr);
  IF_HIP(hipGetLastError());
}

template <class T>
void launch_fold_second_pass(hipStream_t st, int m0, int nl, const double* G2, const T* Tinv, T* Cf, T* G2T,
                             double* Hm, int ldh, int j, int lo, const int* need) {
  hipLaunchKernelGGL((k_fold_second_pass<T>), dim3(nblk((int64_t)(nl + 1) * m0 * m0)), dim3(256), 0, st, m0, nl, G2,
                     Tinv, Cf, G2T, Hm, ldh, j, lo, need);
  IF_HIP(hipGetLastError());
}
void launch_step_checks(hipStream_t st, int nk, int m0, const double* Gsk, const double* gw, double gersh,
                        double dead_thr, int* single, int* two, int* count, int rows, const double* G2, double eta,
                        int* act, double* out) {
  IF_REQUIRE(m0 <= 128, "step checks: m0 > 128");
  hipLaunchKernelGGL(k_step_checks, dim3(1), dim3(1024), 0, st, nk, m0, Gsk, gw, gersh, dead_thr, single, two, count,
                     rows, G2, eta, act, out);
  IF_HIP(hipGetLastError());
}
void launch_local_loss(hipStream_t st, int rows, int m0, const double* G2, const double* gw, double eta, int* act) {
  IF_REQUIRE(m0 <= 128, "local loss: m0 > 128");
  hipLaunchKernelGGL(k_local_loss, dim3(1), dim3(1024), 0, st, rows, m0, G2, gw, eta, act);
  IF_HIP(hipGetLastError());
}

template void launch_fold_second_pass<float>(hipStream_t, int, int, const double*, const float*, float*, float*,
                                             double*, int, int, int, const int*);
template void launch_fold_second_pass<double>(hipStream_t, int, int, const double*, const double*, double*, double*,
                                              double*, int, int, int, const int*);
template void launch_to_T<float>(hipStream_t, int64_t, const double*, float*);
template void launch_to_T<double>(hipStream_t, int64_t, const double*, double*);
template void launch_sum_y<float>(hipStream_t, int, int, int, int, const cd*, const double*, float*);
template void launch_sum_y<double>(hipStream_t, int, int, int, int, const cd*, const double*, double*);

}  // namespace ifeast
