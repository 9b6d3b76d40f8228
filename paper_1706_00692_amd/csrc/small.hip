// Small dense kernels of the inner solve and the Rayleigh-Ritz step, in FP64.
//
// They act on m0 x m0 (or (k+1)m0 x k m0) matrices, run one workgroup per
// shifted system, and are latency-bound; keeping them on the device keeps
// the whole inner loop free of host round trips except one status word.
//
//  * cholqr_factor: Cholesky of the column-scaled Gram of a block (block
//    Arnoldi normalisation, Sec. 3.1) and the inverse factor for the update.
//  * cgs_combine: complex Gram blocks from their real-view products, added to
//    the block Hessenberg matrix Hbar (Sec. 3.1).
//  * lsq_*: block GMRES least squares min ||E1 S - Hbar Y|| (Sec. 3.2) by an
//    incremental Householder QR of Hbar, one block column per Arnoldi step,
//    with the per-column residual norms the stopping rule needs (Algorithm 2,
//    step 1).
//  * rr_small: reduced eigenproblem of the Rayleigh-Ritz step (Algorithm 2,
//    step 3) by SVQB B-orthonormalisation and cyclic Jacobi.
//  * classify: membership, filter-gain test and ||R_F|| (Algorithm 2, step 4).
#include "internal.h"

// Phase timestamps of the Rayleigh-Ritz kernel, compiled in only for profiling builds.
#ifdef IFEAST_RR_PROFILE
__device__ unsigned long long ifeast_rr_prof[32];
extern "C" void ifeast_rr_prof_read(unsigned long long* out) {
  (void)hipMemcpyFromSymbol(out, HIP_SYMBOL(ifeast_rr_prof), 32 * sizeof(unsigned long long));
}
#define RR_MARK(i)                                                \
  do {                                                            \
    __syncthreads();                                              \
    if (threadIdx.x == 0) ::ifeast_rr_prof[i] = wall_clock64();   \
  } while (0)
#else
#define RR_MARK(i) \
  do {             \
  } while (0)
#endif

#include <cstdlib>

#include "dense_dev.h"

namespace ifeast {

namespace {

// Real 2x2 form of complex h acting on interleaved row vectors: [vr, vi] * M = v * h.
template <class T>
__device__ inline void store_realified(T* M, int ldm, int a, int b, c2 h) {
  M[(2 * a) * ldm + 2 * b] = (T)h.x;
  M[(2 * a) * ldm + 2 * b + 1] = (T)h.y;
  M[(2 * a + 1) * ldm + 2 * b] = (T)(-h.y);
  M[(2 * a + 1) * ldm + 2 * b + 1] = (T)h.x;
}

// complex entry (a, b) of V^H W from the real-view product G = V_r^T W_r (2m x 2m)
__device__ inline c2 gram_entry(const double* G, int ld, int a, int b) {
  const double rr = G[(2 * a) * ld + 2 * b], ii = G[(2 * a + 1) * ld + 2 * b + 1];
  const double ri = G[(2 * a) * ld + 2 * b + 1], ir = G[(2 * a + 1) * ld + 2 * b];
  return cmk(rr + ii, ri - ir);
}

// ------------------------------------------------------------ CholQR factor
// A column whose squared norm is at most dead_thr is treated as converged,
// and a column whose Cholesky pivot (of the unit-diagonal scaled Gram) falls
// to tau_dep or below is numerically in the span of the columns before it:
// both get a zero basis column and a zero row of R (for a dependent column
// its projection onto the earlier columns stays in R's column), so the
// block Krylov space deflates instead of amplifying rounding noise.  The
// least squares then gives such columns a zero coefficient.
template <class T>
__global__ __launch_bounds__(256) void k_cholqr_factor(int m0, const double* __restrict__ G, double shift_rel,
                                                       double dead_thr, double tau_dep, const int* __restrict__ active,
                                                       T* __restrict__ Tinv, c2* __restrict__ Racc, int accumulate,
                                                       c2* __restrict__ work) {
  const int s = blockIdx.x;
  if (active != nullptr && active[s] == 0) return;
  const int tid = threadIdx.x, m2 = 2 * m0;
  const double* Gs = G + (int64_t)s * m2 * m2;
  c2* L = work + (int64_t)s * 3 * m0 * m0;
  c2* Ri = L + m0 * m0;
  c2* Tm = Ri + m0 * m0;
  T* Tv = Tinv + (int64_t)s * m2 * m2;
  c2* Ra = Racc + (int64_t)s * m0 * m0;
  __shared__ double dsc[128];
  __shared__ int dead[128];
  __shared__ double piv;
  __shared__ int dep;

  for (int a = tid; a < m0; a += 256) {
    const double g = Gs[(2 * a) * m2 + 2 * a] + Gs[(2 * a + 1) * m2 + 2 * a + 1];
    const bool dd = !(g > dead_thr);
    dead[a] = dd ? 1 : 0;
    dsc[a] = dd ? 1.0 : sqrt(g);
  }
  __syncthreads();
  for (int idx = tid; idx < m0 * m0; idx += 256) {
    const int a = idx / m0, b = idx % m0;
    c2 g;
    if (dead[a] || dead[b]) {
      g = cmk(a == b ? 1.0 : 0.0, 0.0);
    } else {
      g = cscale(1.0 / (dsc[a] * dsc[b]), gram_entry(Gs, m2, a, b));
      if (a == b) g = cmk(g.x + shift_rel, 0.0);
    }
    L[idx] = g;
  }
  __syncthreads();
  // Cholesky G = L L^H (lower triangle of L) with deflation of small pivots
  for (int c = 0; c < m0; ++c) {
    if (tid == 0) {
      const double p = L[c * m0 + c].x;
      dep = (!dead[c] && !(p > tau_dep)) ? 1 : 0;
      if (dep) dead[c] = 1;
      piv = dead[c] ? 1.0 : sqrt(p);
      L[c * m0 + c] = cmk(piv, 0.0);
    }
    __syncthreads();
    if (dead[c]) {
      for (int r = c + 1 + tid; r < m0; r += 256) L[r * m0 + c] = cmk(0.0, 0.0);
      __syncthreads();
      continue;
    }
    const double inv = 1.0 / piv;
    for (int r = c + 1 + tid; r < m0; r += 256) L[r * m0 + c] = cscale(inv, L[r * m0 + c]);
    __syncthreads();
    const int nt = m0 - c - 1;
    for (int idx = tid; idx < nt * nt; idx += 256) {
      const int r = c + 1 + idx / nt, q = c + 1 + idx % nt;
      if (q <= r) L[r * m0 + q] = csub(L[r * m0 + q], cmul(L[r * m0 + c], cconj(L[q * m0 + c])));
    }
    __syncthreads();
  }
  // Ri = (L^H)^{-1}, upper triangular; R'[c][e] = conj(L[e][c])
  for (int d = tid; d < m0; d += 256) {
    for (int c = m0 - 1; c > d; --c) Ri[c * m0 + d] = cmk(0.0, 0.0);
    for (int c = d; c >= 0; --c) {
      c2 sum = cmk(c == d ? 1.0 : 0.0, 0.0);
      for (int e = c + 1; e <= d; ++e) sum = csub(sum, cmul(cconj(L[e * m0 + c]), Ri[e * m0 + d]));
      Ri[c * m0 + d] = cscale(1.0 / L[c * m0 + c].x, sum);
    }
  }
  __syncthreads();
  // W_new = W D^{-1} Ri  ->  real form of D^{-1} Ri; factor R = L^H D.  Dead columns:
  // zero basis column (column of Tinv) and zero row of R (R[a][a] included).
  for (int idx = tid; idx < m0 * m0; idx += 256) {
    const int a = idx / m0, b = idx % m0;
    store_realified(Tv, m2, a, b, (dead[b] || dead[a]) ? cmk(0.0, 0.0) : cscale(1.0 / dsc[a], Ri[idx]));
    Tm[idx] = (b >= a && !dead[a]) ? cscale(dsc[b], cconj(L[b * m0 + a])) : cmk(0.0, 0.0);
  }
  __syncthreads();
  if (accumulate) {
    // Racc <- R * Racc (both upper triangular); Ri is free now
    for (int idx = tid; idx < m0 * m0; idx += 256) {
      const int a = idx / m0, b = idx % m0;
      c2 sum = cmk(0.0, 0.0);
      for (int e = a; e <= b; ++e) sum = cadd(sum, cmul(Tm[a * m0 + e], Ra[e * m0 + b]));
      Ri[idx] = sum;
    }
    __syncthreads();
    for (int idx = tid; idx < m0 * m0; idx += 256) Ra[idx] = Ri[idx];
  } else {
    for (int idx = tid; idx < m0 * m0; idx += 256) Ra[idx] = Tm[idx];
  }
}

// Same factorisation with the lower triangle of L packed in LDS (row r at r(r+1)/2):
// Cholesky, the update Racc <- R Racc, then L is inverted in place (trailing block
// first: column j of L^{-1} below the diagonal is -(L22^{-1} l) / l_jj) and
// Tinv = D^{-1} (L^{-1})^H is written out.  One workgroup per shift.
__device__ inline int pk(int r, int c) { return r * (r + 1) / 2 + c; }

template <class T, bool REAL>
__global__ __launch_bounds__(512) void k_cholqr_lds(int m0, const double* __restrict__ G, double shift_rel,
                                                    double dead_thr, double tau_dep, const int* __restrict__ active,
                                                    T* __restrict__ Tinv, c2* __restrict__ Racc, int accumulate,
                                                    c2* __restrict__ work, int ra_in_lds) {
  const int s = blockIdx.x;
  if (active != nullptr && active[s] == 0) return;
  extern __shared__ c2 lds_c2[];
  c2* L = lds_c2;                       // m0 (m0 + 1) / 2
  c2* x = L + m0 * (m0 + 1) / 2;        // m0
  // REAL: G is the m0 x m0 Gram of a real block and Tinv the real m0 x m0 factor;
  // otherwise G and Tinv are real views (2m0 x 2m0) of complex ones
  const int tid = threadIdx.x, m2 = 2 * m0;
  const int gw = REAL ? m0 : m2;
  const double* Gs = G + (int64_t)s * gw * gw;
  T* Tv = Tinv + (int64_t)s * gw * gw;
  c2* Ra = Racc + (int64_t)s * m0 * m0;
  c2* tmp = work + (int64_t)s * 3 * m0 * m0;
  __shared__ double dsc[128];
  __shared__ int dead[128];

  for (int a = tid; a < m0; a += blockDim.x) {
    const double g = REAL ? Gs[a * m0 + a] : Gs[(2 * a) * m2 + 2 * a] + Gs[(2 * a + 1) * m2 + 2 * a + 1];
    const bool dd = !(g > dead_thr);
    dead[a] = dd ? 1 : 0;
    dsc[a] = dd ? 1.0 : sqrt(g);
  }
  __syncthreads();
  for (int idx = tid; idx < m0 * m0; idx += blockDim.x) {
    const int a = idx / m0, b = idx % m0;
    if (b > a) continue;
    c2 g;
    if (dead[a] || dead[b]) {
      g = cmk(a == b ? 1.0 : 0.0, 0.0);
    } else {
      g = cscale(1.0 / (dsc[a] * dsc[b]), REAL ? cmk(Gs[a * m0 + b], 0.0) : gram_entry(Gs, m2, a, b));
      if (a == b) g = cmk(g.x + shift_rel, 0.0);
    }
    L[pk(a, b)] = g;
  }
  __syncthreads();
  // right-looking Cholesky with deflation of small pivots
  __shared__ double piv;
  for (int c = 0; c < m0; ++c) {
    if (tid == 0) {
      const double p = L[pk(c, c)].x;
      if (!dead[c] && !(p > tau_dep)) dead[c] = 1;
      piv = dead[c] ? 1.0 : sqrt(p);
      L[pk(c, c)] = cmk(piv, 0.0);
    }
    __syncthreads();
    const bool dc = dead[c] != 0;
    const double inv = 1.0 / piv;
    for (int r = c + 1 + tid; r < m0; r += blockDim.x) L[pk(r, c)] = dc ? cmk(0.0, 0.0) : cscale(inv, L[pk(r, c)]);
    __syncthreads();
    if (dc) continue;
    const int nt = m0 - c - 1;
    for (int idx = tid; idx < nt * nt; idx += blockDim.x) {
      const int r = c + 1 + idx / nt, q = c + 1 + idx % nt;
      if (q <= r) L[pk(r, q)] = csub(L[pk(r, q)], cmul(L[pk(r, c)], cconj(L[pk(q, c)])));
    }
    __syncthreads();
  }
  // R = L^H D with zero rows for dead columns; Racc <- R Racc (upper triangular).  The
  // previous Racc is staged in LDS when it fits beside L, else read from global memory
  // eight entries at a time.
  if (accumulate) {
    c2* Rs = x + m0;
    const bool staged = ra_in_lds != 0;
    if (staged) {
      for (int idx = tid; idx < m0 * m0; idx += blockDim.x) Rs[idx] = Ra[idx];
      __syncthreads();
    }
    const c2* Rsrc = staged ? Rs : Ra;
    for (int idx = tid; idx < m0 * m0; idx += blockDim.x) {
      const int a = idx / m0, b = idx % m0;
      c2 v = cmk(0.0, 0.0);
      if (b >= a && !dead[a]) {
        for (int e0 = a; e0 <= b; e0 += 8) {
          c2 rv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) rv[u] = (e0 + u <= b) ? Rsrc[(e0 + u) * m0 + b] : cmk(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (e0 + u <= b) v = cadd(v, cmul(cscale(dsc[e0 + u], cconj(L[pk(e0 + u, a)])), rv[u]));
        }
      }
      tmp[idx] = v;
    }
  } else {
    for (int idx = tid; idx < m0 * m0; idx += blockDim.x) {
      const int a = idx / m0, b = idx % m0;
      tmp[idx] = (b >= a && !dead[a]) ? cscale(dsc[b], cconj(L[pk(b, a)])) : cmk(0.0, 0.0);
    }
  }
  __syncthreads();
  for (int idx = tid; idx < m0 * m0; idx += blockDim.x) Ra[idx] = tmp[idx];
  // L <- L^{-1} in place, trailing block first; each row's dot product is split over 8
  // consecutive lanes and summed with shuffles
  for (int j = m0 - 1; j >= 0; --j) {
    for (int i = j + 1 + tid; i < m0; i += blockDim.x) x[i] = L[pk(i, j)];
    const double ljj = 1.0 / L[pk(j, j)].x;
    __syncthreads();
    const int nrows = m0 - 1 - j;
    for (int base = 0; base < nrows; base += (int)blockDim.x / 8) {
      const int i = j + 1 + base + tid / 8, part = tid % 8;
      c2 v = cmk(0.0, 0.0);
      if (i < m0)
        for (int k = j + 1 + part; k <= i; k += 8) v = cadd(v, cmul(L[pk(i, k)], x[k]));
      for (int o = 1; o < 8; o <<= 1) {
        v.x += __shfl_xor(v.x, o);
        v.y += __shfl_xor(v.y, o);
      }
      if (i < m0 && part == 0) L[pk(i, j)] = cscale(-ljj, v);
    }
    __syncthreads();
    if (tid == 0) L[pk(j, j)] = cmk(ljj, 0.0);
  }
  __syncthreads();
  // Tinv = D^{-1} Ri with Ri = (L^{-1})^H; dead columns and rows are zero
  for (int idx = tid; idx < m0 * m0; idx += blockDim.x) {
    const int a = idx / m0, b = idx % m0;
    const c2 v = (b < a || dead[a] || dead[b]) ? cmk(0.0, 0.0) : cscale(1.0 / dsc[a], cconj(L[pk(b, a)]));
    if (REAL)
      Tv[a * m0 + b] = (T)v.x;
    else
      store_realified(Tv, m2, a, b, v);
  }
}

// Real-block factor (the shared basis), blocked by 16-column panels so that it needs a few
// dozen block barriers instead of several per column.  L (m0 x m0, row-major) in LDS:
//  1. unit-diagonal scaled Gram (+ shift), dead columns as identity;
//  2. Cholesky: per panel, wave 0 factors the 16 x 16 diagonal block (with the deflation
//     test), then the rows below solve against it, then the trailing matrix is updated;
//  3. Racc <- R Racc (or R), R = L^T D with zero rows for dead columns;
//  4. L^{-1}: one wave inverts each diagonal block, then block row i of the inverse is
//     -L_ii^{-1} sum_{k=j..i-1} L_ik X_kj, for all j < i at once;
//  5. Tinv = D^{-1} (L^{-1})^T with dead rows and columns zero.
// LDS: L, a 16 x m0 block row, and the previous R (m0 <= 96; for larger m0 the previous R goes
// to Rs_glob, an m0 x m0 global scratch, and the rest still fits: 145 KiB at m0 = 128).
template <class T>
__global__ __launch_bounds__(512) void k_cholqr_real(int m0, const double* __restrict__ G, double shift_rel,
                                                     double dead_thr, double tau_dep, T* __restrict__ Tinv,
                                                     c2* __restrict__ Racc, int accumulate,
                                                     const int* __restrict__ single, int role,
                                                     double* __restrict__ Hm, int ldh, int jstep,
                                                     T* __restrict__ Hr_next, double* __restrict__ Rs_glob) {
  // single[0] != 0 (the Gram is certified well conditioned): the first pass (role 0) runs
  // unshifted and the second (role 1) is not needed
  bool final_pass = role == 1;
  if (single != nullptr && single[0] != 0) {
    if (role == 1) return;
    shift_rel = 0.0;
    tau_dep = 0.25 * m0 * (sizeof(T) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16);
    final_pass = true;
  }
  // Hm != null: the final pass also writes the new subdiagonal block Hm(j+1, j) = R; with
  // Hr_next != null also its transpose into rows j m0.. of block column j+1 and into Hr_next
  // (the next step's first-pass coefficients against V_j, which the recurrence gives)
  const bool lanczos_out = Hm != nullptr && final_pass;
  constexpr int NB = 16;
  extern __shared__ double lds_d[];
  // rows of L padded to an odd number of doubles: column walks hit distinct LDS banks
  const int ldl = m0 + 1;
  double* L = lds_d;            // m0 x ldl
  double* tmp = L + m0 * ldl;   // 16 x m0
  double* Rs = Rs_glob != nullptr ? Rs_glob : tmp + NB * m0;  // m0 x m0
  __shared__ double dsc[128], dinv[128];
  __shared__ int dead[128];
  const int tid = threadIdx.x, nth = blockDim.x, wave = tid >> 6, lane = tid & 63;
  const int P = m0 / NB;
  RR_MARK(16);
  // ---- 1.  The Gram's entries are loaded (sixteen per thread in flight, the first round together
  // with the diagonal), then scaled by the reciprocals of the column norms.
  constexpr int kGU = 16;
  double gv[kGU];
  auto gload = [&](int i0) {
#pragma unroll
    for (int u = 0; u < kGU; ++u) {
      const int idx = i0 + u * nth;
      gv[u] = idx < m0 * m0 ? G[idx] : 0.0;
    }
  };
  gload(tid);
  for (int a = tid; a < m0; a += nth) {
    const double g = G[a * m0 + a];
    const bool dd = !(g > dead_thr);
    dead[a] = dd ? 1 : 0;
    dsc[a] = dd ? 1.0 : sqrt(g);
    dinv[a] = 1.0 / dsc[a];  // scaling reciprocals (reset to the Cholesky pivots' below)
  }
  __syncthreads();
  for (int i0 = tid; i0 < m0 * m0; i0 += kGU * nth) {
    if (i0 != tid) gload(i0);
#pragma unroll
    for (int u = 0; u < kGU; ++u) {
      const int idx = i0 + u * nth;
      if (idx >= m0 * m0) break;
      const int a = idx / m0, b = idx % m0;
      double g;
      if (dead[a] || dead[b]) g = a == b ? 1.0 : 0.0;
      else g = gv[u] * (dinv[a] * dinv[b]) + (a == b ? shift_rel : 0.0);
      L[a * ldl + b] = g;
      if (accumulate) Rs[idx] = Racc[idx].x;
    }
  }
  __syncthreads();
  // ---- 2. blocked Cholesky (lower triangle of L)
  RR_MARK(17);
  for (int p = 0; p < P; ++p) {
    const int c0 = p * NB;
    if (wave == 0) {
      // the diagonal block in registers: lane i < 16 holds row i; the column entries other
      // lanes need are broadcast from their lanes, so the 16 dependent column steps touch no LDS
      const int i = lane;
      double arow[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) arow[q] = i < NB ? L[(c0 + i) * ldl + c0 + q] : 0.0;
      int my_dead = 0;
      double my_dinv = 1.0;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double pv0 = lane_bcast(arow[c], c);
        const bool dc = dead[c0 + c] != 0 || !(pv0 > tau_dep);
        // 1/sqrt(p) from the hardware estimate and two Newton steps (each doubles the correct
        // bits), sqrt(p) = p / sqrt(p): a shorter dependent chain than a rounded square root
        // and division
        const double pp = dc ? 1.0 : pv0;
        double rpv = __builtin_amdgcn_rsq(pp);
        rpv = rpv * (1.5 - 0.5 * pp * rpv * rpv);
        rpv = rpv * (1.5 - 0.5 * pp * rpv * rpv);
        const double pv = pp * rpv;
        if (i > c) arow[c] = dc ? 0.0 : arow[c] * rpv;
        if (i == c) {
          arow[c] = pv;
          my_dead = dc ? 1 : 0;
          my_dinv = rpv;
        }
        if (!dc) {
#pragma unroll
          for (int q = c + 1; q < NB; ++q) {
            const double lqc = lane_bcast(arow[c], q);
            if (q <= i) arow[q] -= arow[c] * lqc;
          }
        }
      }
      if (i < NB) {
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q <= i) L[(c0 + i) * ldl + c0 + q] = arow[q];
        dead[c0 + i] = my_dead;
        dinv[c0 + i] = my_dinv;
      }
    }
    __syncthreads();
    // rows below the diagonal block: x L11^T = a, forward along the panel's columns (the
    // row's solved entries stay in registers)
    for (int r = c0 + NB + tid; r < m0; r += nth) {
      double xr[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        double v = L[r * ldl + c0 + c];
#pragma unroll
        for (int k = 0; k < c; ++k) v -= xr[k] * L[(c0 + c) * ldl + c0 + k];
        xr[c] = dead[c0 + c] ? 0.0 : v * dinv[c0 + c];
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) L[r * ldl + c0 + c] = xr[c];
    }
    __syncthreads();
    // trailing matrix, lower triangle: lane -> column q (its panel row in registers), wave ->
    // every (nth/64)-th row r, whose panel row all lanes read at one LDS address
    const int t0 = c0 + NB;
    for (int q = t0 + lane; q < m0; q += 64) {
      double lq[NB];
#pragma unroll
      for (int k = 0; k < NB; ++k) lq[k] = L[q * ldl + c0 + k];
      for (int r = t0 + wave; r < m0; r += nth / 64) {
        if (q > r) continue;
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < NB; ++k) v += L[r * ldl + c0 + k] * lq[k];
        L[r * ldl + q] -= v;
      }
    }
    __syncthreads();
  }
  // ---- 3. R factor (global writes; the previous R was staged in LDS)
  RR_MARK(18);
  auto rfac = [&](int a, int b) {
    double v = 0.0;
    if (b >= a && !dead[a]) {
      if (accumulate)
        for (int e = a; e <= b; ++e) v += dsc[e] * L[e * ldl + a] * Rs[e * m0 + b];
      else
        v = dsc[b] * L[b * ldl + a];
    }
    return v;
  };
  // R row-major into Racc and (transposed) block column jstep + 1 of Hm: consecutive threads,
  // consecutive b
  for (int idx = tid; idx < m0 * m0; idx += nth) {
    const int a = idx / m0, b = idx % m0;
    const double v = rfac(a, b);
    Racc[idx] = make_double2(v, 0.0);
    if (lanczos_out && Hr_next != nullptr) Hm[(int64_t)((jstep + 1) * m0 + a) * ldh + jstep * m0 + b] = v;
  }
  // R into block column jstep of Hm (column-major) and Hr_next: consecutive threads, consecutive a
  if (lanczos_out) {
    for (int idx = tid; idx < m0 * m0; idx += nth) {
      const int b = idx / m0, a = idx % m0;
      const double v = rfac(a, b);
      Hm[(int64_t)(jstep * m0 + b) * ldh + (jstep + 1) * m0 + a] = v;
      if (Hr_next != nullptr) Hr_next[b * m0 + a] = (T)v;
    }
  }
  // the inversion overwrites L's diagonal blocks, which the R entries above read; the R stores
  // themselves need not complete before it
  lds_barrier();
  // ---- 4a. invert the diagonal blocks, one wave each (in place)
  RR_MARK(19);
  for (int p = wave; p < P; p += nth / 64) {
    const int c0 = p * NB;
    const int i = lane;  // row of the block (lanes 16..63 idle), held in registers
    double xrow[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) xrow[q] = (i < NB && q <= i) ? L[(c0 + i) * ldl + c0 + q] : 0.0;
    // column j of the inverse from columns j+1.. (rows of the inverse in registers) and
    // column j of L (still unchanged in the registers of lanes k > j)
#pragma unroll
    for (int j = NB - 1; j >= 0; --j) {
      const double ljj = lane_bcast(xrow[j], j);
      double v = 0.0;
#pragma unroll
      for (int k = j + 1; k < NB; ++k) {
        const double lkj = lane_bcast(xrow[j], k);
        if (k <= i) v += xrow[k] * lkj;
      }
      if (i > j && i < NB) xrow[j] = -v / ljj;
      if (i == j) xrow[j] = 1.0 / ljj;
    }
    if (i < NB) {
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q <= i) L[(c0 + i) * ldl + c0 + q] = xrow[q];
    }
  }
  __syncthreads();
  // ---- 4b. block rows of the inverse below the diagonal
  RR_MARK(20);
  for (int bi = 1; bi < P; ++bi) {
    const int r0 = bi * NB, w = bi * NB;  // block row start; the blocks j < bi span columns [0, w)
    // S_j = sum_{k=j..bi-1} L_{bi,k} X_{k,j}  (X: the inverse so far), into tmp[16][w]
    for (int idx = tid; idx < NB * w; idx += nth) {
      const int r = idx / w, c = idx % w;
      // X is lower triangular (rows k >= c); L's storage above the diagonal is not part of it.
      // The same trip count on every lane (the rows above c masked), so the loads pipeline.
      double v = 0.0;
#pragma unroll 8
      for (int k = 0; k < r0; ++k) {
        const double p = L[(r0 + r) * ldl + k] * L[k * ldl + c];
        v += k >= c ? p : 0.0;
      }
      tmp[r * m0 + c] = v;
    }
    __syncthreads();
    // X_{bi,j} = -L_{bi,bi}^{-1} S_j (the diagonal block is already inverted)
    for (int idx = tid; idx < NB * w; idx += nth) {
      const int r = idx / w, c = idx % w;
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < NB; ++m) {
        const double p = L[(r0 + r) * ldl + r0 + m] * tmp[m * m0 + c];
        v += m <= r ? p : 0.0;
      }
      L[(r0 + r) * ldl + c] = -v;
    }
    __syncthreads();
  }
  // ---- 5.
  RR_MARK(21);
  for (int idx = tid; idx < m0 * m0; idx += nth) {
    const int a = idx / m0, b = idx % m0;
    const double v = (b < a || dead[a] || dead[b]) ? 0.0 : L[b * ldl + a] / dsc[a];
    Tinv[idx] = (T)v;
  }
  RR_MARK(22);
}

template <class T>
__global__ void k_cgs_combine(int ns, int ni, int m0, int j, int ldh, const double* __restrict__ G,
                              const int* __restrict__ active, c2* __restrict__ H, T* __restrict__ Hr, int accumulate) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)m0 * m0;
  if (idx >= (int64_t)ns * ni * per) return;
  const int item = (int)(idx / per);
  const int s = item / ni, i = item % ni;
  if (active != nullptr && active[s] == 0) return;
  const int a = (int)((idx % per) / m0), b = (int)(idx % m0);
  const int m2 = 2 * m0;
  const c2 c = gram_entry(G + (int64_t)item * m2 * m2, m2, a, b);
  c2* h = H + (int64_t)s * ldh * ((int64_t)(ldh / m0 - 1) * m0) + (int64_t)(j * m0 + b) * ldh + i * m0 + a;
  *h = accumulate ? cadd(*h, c) : c;
  store_realified(Hr + (int64_t)item * m2 * m2, m2, a, b, c);
}

// Per shift, from the Gram G = W1^H W1 (real view) of the block after one classical
// Gram-Schmidt pass and the coefficients H of that pass (column block j of Hbar):
//  * need[s]: a second Gram-Schmidt pass is needed, because some live column kept less
//    than the fraction eta of its norm (||W0 e_c||^2 = ||H e_c||^2 + ||W1 e_c||^2);
//  * single[s]: one unshifted Cholesky-QR pass suffices, because no second pass is needed,
//    no column is negligible and Gershgorin's theorem puts every eigenvalue of the
//    unit-diagonal scaled Gram in [1 - delta, 1 + delta] with delta <= gersh (so the
//    Q factor of one pass is orthonormal to about kappa^2 u, kappa <= (1 + gersh) / (1 - gersh));
//  * twopass[s] = active and not single.
__global__ void k_orth_check(int m0, int j, int ldh, double eta2, double gersh, double dead_thr,
                             const double* __restrict__ G, const int* __restrict__ active,
                             const c2* __restrict__ H, int* __restrict__ need, int* __restrict__ single,
                             int* __restrict__ twopass) {
  const int s = blockIdx.x;
  if (active != nullptr && active[s] == 0) {
    if (threadIdx.x == 0) need[s] = single[s] = twopass[s] = 0;
    return;
  }
  __shared__ int any_need, any_bad;
  __shared__ double dsc[128];
  if (threadIdx.x == 0) any_need = any_bad = 0;
  __syncthreads();
  const int m2 = 2 * m0, kk = ldh / m0 - 1;
  const double* Gs = G + (int64_t)s * m2 * m2;
  const c2* Hs = H + (int64_t)s * ldh * kk * m0 + (int64_t)j * m0 * ldh;
  for (int c = threadIdx.x; c < m0; c += blockDim.x) {
    const double w1 = Gs[(2 * c) * m2 + 2 * c] + Gs[(2 * c + 1) * m2 + 2 * c + 1];
    double h = 0.0;
    for (int r = 0; r < (j + 1) * m0; ++r) h += cabs2(Hs[r + (int64_t)c * ldh]);
    if (w1 > 1e-30 && w1 < eta2 * (w1 + h)) atomicOr(&any_need, 1);
    if (!(w1 > dead_thr)) atomicOr(&any_bad, 1);
    dsc[c] = sqrt(fmax(w1, 1e-300));
  }
  __syncthreads();
  for (int r = threadIdx.x; r < m0; r += blockDim.x) {
    double off = 0.0;
    for (int c = 0; c < m0; ++c)
      if (c != r) off += sqrt(cabs2(gram_entry(Gs, m2, r, c))) / (dsc[r] * dsc[c]);
    if (!(off <= gersh)) atomicOr(&any_bad, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    need[s] = any_need;
    single[s] = (any_need == 0 && any_bad == 0) ? 1 : 0;
    twopass[s] = single[s] ? 0 : 1;
  }
}

__global__ void k_store_subdiag(int ns, int m0, int j, int ldh, const int* __restrict__ active,
                                const c2* __restrict__ Racc, c2* __restrict__ H) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)m0 * m0;
  if (idx >= ns * per) return;
  const int s = (int)(idx / per);
  if (active != nullptr && active[s] == 0) return;
  const int a = (int)((idx % per) / m0), b = (int)(idx % m0);
  const int kk = ldh / m0 - 1;
  H[(int64_t)s * ldh * kk * m0 + (int64_t)(j * m0 + b) * ldh + (j + 1) * m0 + a] = Racc[s * per + a * m0 + b];
}

// -------------------------------------------------------------- least squares
struct LsqView {
  c2 *H, *Vh, *g, *y, *u;
  double *tau, *res;
  const double* tol;
};

__device__ inline LsqView lsq_view(const LsqArgs& a, int s) {
  const int m0 = a.m0, k = a.k, ldh = a.ldh;
  LsqView v;
  v.H = reinterpret_cast<c2*>(a.H) + (int64_t)s * ldh * k * m0;
  v.Vh = reinterpret_cast<c2*>(a.Vh) + (int64_t)s * k * 2 * m0 * m0;
  v.tau = a.tauh + (int64_t)s * k * m0;
  v.g = reinterpret_cast<c2*>(a.g) + (int64_t)s * ldh * m0;
  v.y = reinterpret_cast<c2*>(a.y) + (int64_t)s * k * m0 * m0;
  v.u = reinterpret_cast<c2*>(a.u) + (int64_t)s * ldh * m0;
  v.res = a.res + (int64_t)s * m0;
  v.tol = a.tol + (int64_t)s * m0;
  return v;
}

// ---- wave-level helpers: one 64-lane wavefront owns one column
__device__ inline c2 wave_csum(c2 v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  return v;
}
__device__ inline double wave_dsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// x[r] -= tau v[r] (v^H x) over the support rows [r0, r1); x is a wave-owned column
// (LDS or global), v a reflector vector in global memory.
__device__ inline void wave_reflect(const c2* __restrict__ v, double tau, int r0, int r1, c2* x, int lane) {
  c2 d = cmk(0.0, 0.0);
  for (int r = r0 + lane; r < r1; r += 64) d = cadd(d, cjmul(v[r], x[r]));
  d = wave_csum(d);
  const c2 f = cscale(tau, d);
  for (int r = r0 + lane; r < r1; r += 64) x[r] = csub(x[r], cmul(f, v[r]));
  // row ownership moves between lanes from one reflector to the next
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Apply reflectors c = c_begin..c_end-1 (in order, or reversed) of one step to a wave-owned
// column x (LDS); reflector c lives in v + c*ld with support rows [c, m0 + c].  The next
// reflector's vector is loaded into registers while the current one is applied.
__device__ inline void wave_reflect_run(const c2* __restrict__ V, const double* __restrict__ tau, int m0, int ld,
                                        c2* x, int lane, bool reverse) {
  constexpr int R = 3;  // support m0 + 1 <= 129 rows -> at most 3 rows per lane
  c2 cur[R], nxt[R];
  auto load = [&](int c, c2* dst) {
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int r = c + lane + 64 * t;
      dst[t] = (r <= m0 + c) ? V[(int64_t)c * ld + r] : cmk(0.0, 0.0);
    }
  };
  int c = reverse ? m0 - 1 : 0;
  const int step = reverse ? -1 : 1;
  load(c, cur);
  for (int it = 0; it < m0; ++it, c += step) {
    const int cn = c + step;
    if (it + 1 < m0) load(cn, nxt);
    const double tv = tau[c];
    if (tv != 0.0) {
      c2 d = cmk(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int r = c + lane + 64 * t;
        if (r <= m0 + c) d = cadd(d, cjmul(cur[t], x[r]));
      }
      d = wave_csum(d);
      const c2 f = cscale(tv, d);
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int r = c + lane + 64 * t;
        if (r <= m0 + c) x[r] = csub(x[r], cmul(f, cur[t]));
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
#pragma unroll
    for (int t = 0; t < R; ++t) cur[t] = nxt[t];
  }
}

__global__ __launch_bounds__(256) void k_lsq_init(LsqArgs a, const c2* __restrict__ S) {
  const int s = blockIdx.x;
  if (a.active[s] == 0) return;
  const LsqView v = lsq_view(a, s);
  const int m0 = a.m0, ldh = a.ldh, tid = threadIdx.x;
  for (int64_t idx = tid; idx < (int64_t)ldh * m0; idx += 256) v.g[idx] = cmk(0.0, 0.0);
  __syncthreads();
  const c2* Ss = S + (int64_t)s * m0 * m0;
  for (int idx = tid; idx < m0 * m0; idx += 256) {
    const int r = idx / m0, c = idx % m0;
    v.g[r + (int64_t)c * ldh] = Ss[idx];
  }
  __syncthreads();
  for (int c = tid; c < m0; c += 256) {
    double ss = 0.0;
    for (int r = 0; r < m0; ++r) ss += cabs2(v.g[r + (int64_t)c * ldh]);
    v.res[c] = sqrt(ss);
  }
  if (tid == 0) {
    a.iters[s] = 0;
    a.cycle_done[s] = 0;
  }
}

// Step j for m0 > 96, after the earlier reflectors (k_lsq_reflect): Householder QR of the slab
// rows [j m0, (j+2) m0) of block column j (its lower half is upper triangular) in global memory,
// the same reflectors on the right-hand side, per-column residual norms and the stopping rule.
// One workgroup per shift, one wave per column.
__global__ __launch_bounds__(256) void k_lsq_qr(LsqArgs a, int j) {
  const int s = blockIdx.x;
  if (a.active[s] == 0) return;
  const LsqView v = lsq_view(a, s);
  const int m0 = a.m0, ldh = a.ldh, m2 = 2 * m0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int base = j * m0;
  c2* h = v.H + (int64_t)j * m0 * ldh + base;  // slab (row r, col c) at h[r + c * ldh]
  c2* Vj = v.Vh + (int64_t)j * m2 * m0;
  double* tj = v.tau + j * m0;
  __shared__ double sh_tau;
  __shared__ int sh_ok;
  for (int c = 0; c < m0; ++c) {
    c2* vc = Vj + (int64_t)c * m2;
    const int r0 = c, r1 = m0 + c + 1;
    if (wave == 0) {
      c2* xc = h + (int64_t)c * ldh;
      double ss = 0.0;
      for (int r = r0 + lane; r < r1; r += 64) ss += cabs2(xc[r]);
      ss = wave_dsum(ss);
      const double nrm = sqrt(ss);
      const c2 x0 = xc[r0];
      double tau = 0.0;
      c2 beta = x0, v0 = cmk(0.0, 0.0);
      if (nrm > 0.0) {
        const double ax = sqrt(cabs2(x0));
        const c2 ph = ax > 0.0 ? cscale(1.0 / ax, x0) : cmk(1.0, 0.0);
        beta = cscale(-nrm, ph);
        v0 = csub(x0, beta);
        const double vn2 = ss - cabs2(x0) + cabs2(v0);
        tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
      }
      for (int r = lane; r < m2; r += 64) {
        c2 val = cmk(0.0, 0.0);
        if (tau != 0.0) val = (r == r0) ? v0 : ((r > r0 && r < r1) ? xc[r] : cmk(0.0, 0.0));
        vc[r] = val;
      }
      if (lane == 0) {
        tj[c] = tau;
        sh_tau = tau;
      }
      // the column becomes (beta, 0, ..., 0) on its support
      if (tau != 0.0)
        for (int r = r0 + lane; r < r1; r += 64) xc[r] = (r == r0) ? beta : cmk(0.0, 0.0);
    }
    __syncthreads();
    const double tau = sh_tau;
    if (tau != 0.0)
      for (int col = c + 1 + wave; col < m0; col += 4) wave_reflect(vc, tau, r0, r1, h + (int64_t)col * ldh, lane);
    __syncthreads();
  }
  // the same reflectors on the right-hand side columns
  for (int col = wave; col < m0; col += 4) {
    c2* gc = v.g + base + (int64_t)col * ldh;
    for (int c = 0; c < m0; ++c) {
      const double tau = tj[c];
      if (tau != 0.0) wave_reflect(Vj + (int64_t)c * m2, tau, c, m0 + c + 1, gc, lane);
    }
  }
  if (tid == 0) sh_ok = 1;
  __syncthreads();
  // residual norms: the last m0 rows of the transformed right-hand side
  for (int col = wave; col < m0; col += 4) {
    const c2* gc = v.g + (int64_t)(j + 1) * m0 + (int64_t)col * ldh;
    double ss = 0.0;
    for (int r = lane; r < m0; r += 64) ss += cabs2(gc[r]);
    ss = wave_dsum(ss);
    if (lane == 0) {
      const double rn = sqrt(ss);
      v.res[col] = rn;
      if (!(rn <= v.tol[col])) atomicAnd(&sh_ok, 0);
    }
  }
  __syncthreads();
  if (tid == 0) {
    a.iters[s] = j + 1;
    if (sh_ok) {
      a.cycle_done[s] = 1;
      a.active[s] = 0;
    }
  }
}

// Step j, part 4: the stopping rule of the shift (every column's residual at or below
// its threshold ends the cycle).  One wave per shift.
__global__ void k_lsq_stop(LsqArgs a, int j) {
  const int s = blockIdx.x;
  if (a.active[s] == 0) return;
  const LsqView v = lsq_view(a, s);
  const int lane = threadIdx.x;
  int bad = 0;
  for (int c = lane; c < a.m0; c += 64) bad |= !(v.res[c] <= v.tol[c]);
  for (int o = 32; o > 0; o >>= 1) bad |= __shfl_xor(bad, o);
  if (lane == 0) {
    a.iters[s] = j + 1;
    if (!bad) {
      a.cycle_done[s] = 1;
      a.active[s] = 0;
    }
  }
}

// ---- step j with one 16-lane group per column (DPP row reductions instead of wave-wide lane
// permutes, so a reflector's dot product costs four dependent stages): k_lsq_reflect for the
// earlier reflectors, k_lsq_qr_regs for the new slab (m0 <= 96), k_lsq_reflect for the
// right-hand side and its residual norms, k_lsq_stop.
//
// Reflectors of earlier steps on a block of columns.  grid (ns, ceil(m0/16)), 256 threads:
// group g owns column 16 y + g.  RHS == false: the reflectors of steps i0..j-1 on block column
// j of Hbar (i0 = 0, or j - band - 1 for a banded Hbar); RHS == true: those of step j on the
// right-hand side slab rows [j m0, (j+2) m0), then the column's residual norm (the slab's last
// m0 rows).  M0 > 0: m0 fixed at compile time (the lane masks fold away); 0: a.m0.
// Reflector block i acts on rows [i m0, (i+2) m0) only and leaves rows [i m0, (i+1) m0) final, so the group keeps that window in registers: rows i m0 + 16 q + l
// (top) and (i+1) m0 + 16 q + l (bottom) in lane l's slot q < SH = ceil(m0/16), the next
// block's rows loading while the current block applies.  The reflectors pass through LDS in
// chunks of rc columns (rc * 2 m0 <= kChunk), the next chunk's loads in flight meanwhile.
// s_waitcnt operand (gfx9 encoding): vector memory count 0, the other counters unconstrained
constexpr int kVmcntZero = 0x0F70;
constexpr int kChunk = 2560;  // complex entries of one reflector chunk (40 KiB)
constexpr int kChunkPer = kChunk / 256;

template <int SH, bool RHS, int M0>
__global__ __launch_bounds__(256) void k_lsq_reflect(LsqArgs a, int j, int rc) {
  extern __shared__ c2 vch[];  // rc x 2 m0 reflector entries, then rc taus
  const int s = blockIdx.x;
  if (a.active[s] == 0 || (!RHS && j == 0)) return;
  const LsqView v = lsq_view(a, s);
  const int m0 = M0 > 0 ? M0 : a.m0, ldh = a.ldh, m2 = 2 * m0;
  const int tid = threadIdx.x, l = tid & 15;
  const int col = blockIdx.y * 16 + (tid >> 4);
  const bool has = col < m0;  // the same for the 16 lanes of a group
  double* tch = reinterpret_cast<double*>(vch + rc * m2);
  const int i0 = RHS ? j : (a.band > 0 ? max(0, j - a.band - 1) : 0);
  const int i1 = RHS ? j + 1 : j;  // reflector blocks [i0, i1)
  c2* h = (RHS ? v.g : v.H + (int64_t)j * m0 * ldh) + (int64_t)(has ? col : 0) * ldh;  // row 0 of the column
  auto load_rows = [&](int r0, c2* dst) {
#pragma unroll
    for (int q = 0; q < SH; ++q) {
      const int rr = 16 * q + l;
      dst[q] = (has && rr < m0) ? h[r0 + rr] : cmk(0.0, 0.0);
    }
  };
  auto store_rows = [&](int r0, const c2* src) {
#pragma unroll
    for (int q = 0; q < SH; ++q) {
      const int rr = 16 * q + l;
      if (has && rr < m0) h[r0 + rr] = src[q];
    }
  };
  c2 top[SH], bot[SH], nxt[SH];
  load_rows(i0 * m0, top);
  load_rows((i0 + 1) * m0, bot);
  // the window is complete before the loop: otherwise the reflector loop, unable to tell these
  // loads from the chunk prefetches, waits on every prefetch at its first reflector
  __builtin_amdgcn_s_waitcnt(kVmcntZero);
  if (i0 + 1 < i1) load_rows((i0 + 2) * m0, nxt);
  const int nch = (m0 + rc - 1) / rc, total = (i1 - i0) * nch;
  c2 pre[kChunkPer];
  double pre_tau = 0.0;
  auto fetch = [&](int t) {
    const int i = i0 + t / nch, c0 = (t % nch) * rc, cnt = min(rc, m0 - c0);
    const c2* src = v.Vh + ((int64_t)i * m0 + c0) * m2;  // reflector c0 of step i
#pragma unroll
    for (int q = 0; q < kChunkPer; ++q) {
      const int e = tid + 256 * q;
      pre[q] = e < cnt * m2 ? src[e] : cmk(0.0, 0.0);
    }
    pre_tau = tid < cnt ? v.tau[i * m0 + c0 + tid] : 0.0;
  };
  fetch(0);
  for (int t = 0; t < total; ++t) {
    const int i = i0 + t / nch, c0 = (t % nch) * rc, cnt = min(rc, m0 - c0);
    __syncthreads();  // the previous chunk is no longer read
#pragma unroll
    for (int q = 0; q < kChunkPer; ++q) {
      const int e = tid + 256 * q;
      if (e < cnt * m2) vch[e] = pre[q];
    }
    if (tid < cnt) tch[tid] = pre_tau;
    __syncthreads();
    if (t + 1 < total) fetch(t + 1);
    if (has) {
      for (int cc = 0; cc < cnt; ++cc) {
        const double tv = tch[cc];
        if (tv == 0.0) continue;
        // the reflector's entries for this lane's rows, all loads first; it is zero off its
        // support rows c .. m0 + c (padding lanes take zeros)
        const c2* vc = vch + cc * m2;
        c2 vt[SH], vu[SH];
#pragma unroll
        for (int q = 0; q < SH; ++q) {
          const int rr = min(16 * q + l, m0 - 1);
          vt[q] = vc[rr];
          vu[q] = vc[m0 + rr];
        }
        c2 d = cmk(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < SH; ++q) {
          if (16 * q + l >= m0) {
            vt[q] = cmk(0.0, 0.0);
            vu[q] = cmk(0.0, 0.0);
          }
          d = cadd(d, cjmul(vt[q], top[q]));
          d = cadd(d, cjmul(vu[q], bot[q]));
        }
        const c2 f = cscale(tv, row16_csum(d));
#pragma unroll
        for (int q = 0; q < SH; ++q) {
          top[q] = csub(top[q], cmul(f, vt[q]));
          bot[q] = csub(bot[q], cmul(f, vu[q]));
        }
      }
    }
    if ((t + 1) % nch == 0) {
      // block i done: rows [i m0, (i+1) m0) are final; the window moves down one block
      store_rows(i * m0, top);
      if (i + 1 < i1) {
#pragma unroll
        for (int q = 0; q < SH; ++q) {
          top[q] = bot[q];
          bot[q] = nxt[q];
        }
        if (i + 2 < i1) load_rows((i + 3) * m0, nxt);
      } else {
        store_rows((i + 1) * m0, bot);
      }
    }
  }
  if (RHS) {
    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < SH; ++q) ss += cabs2(bot[q]);
    ss = row16_sum(ss);
    if (has && l == 0) v.res[col] = sqrt(ss);
  }
}

// Householder QR of the slab rows [j m0, (j+2) m0) of block column j (its lower half upper
// triangular), reflectors and taus to Vh / tauh, R in place, with the columns in registers:
// one workgroup per shift, 512 threads in 32 groups of 16 lanes,
// group g owning columns g, g + 32, ..  (MAXC at most).  Reflector c acts on rows c..m0+c, and the
// owner of column c + 1 forms reflector c + 1 from rows c+1..m0+c+1, so every column a group
// still updates keeps rows [b, b + 16 NW) in registers, b = 16 floor(c / 16) (NW slots of 16
// rows, NW = floor((m0 + 32) / 16)): every 16 steps the top slot (final rows of R) goes to global
// memory and the next 16 rows of the slab enter from it (loaded one window shift ahead).  A
// finished column writes its window back.  Only the reflectors pass through LDS (two buffers
// indexed by slab row, zero off the support), so the factorisation moves no column data
// through LDS and needs little of it.  M0 > 0: m0 fixed at compile time; 0: a.m0.
template <int NW, int MAXC, int M0>
__global__ __launch_bounds__(512) void k_lsq_qr_regs(LsqArgs a, int j) {
  constexpr int NG = 32;
  __shared__ c2 vb[2][256 + 32];
  __shared__ double tb[2];
  const int s = blockIdx.x;
  if (a.active[s] == 0) return;
  const LsqView v = lsq_view(a, s);
  const int m0 = M0 > 0 ? M0 : a.m0, ldh = a.ldh, m2 = 2 * m0;
  const int tid = threadIdx.x, g = tid >> 4, l = tid & 15, gl0 = tid & 48;  // gl0: the group's first lane in its wave
  c2* h = v.H + (int64_t)j * m0 * ldh + j * m0;  // slab (row r, col c) at h[r + c * ldh]
  c2* Vj = v.Vh + (int64_t)j * m2 * m0;
  double* tj = v.tau + j * m0;
  // column i of the group: g + 32 i; rows 0..m0+col of it are stored
  auto colof = [&](int i) { return g + NG * i; };
  auto ld = [&](int col, int r) { return (col < m0 && r <= m0 + col) ? h[(int64_t)col * ldh + r] : cmk(0.0, 0.0); };
  c2 x[MAXC][NW], pf[MAXC];
#pragma unroll
  for (int i = 0; i < MAXC; ++i) {
#pragma unroll
    for (int q = 0; q < NW; ++q) x[i][q] = ld(colof(i), 16 * q + l);
    pf[i] = ld(colof(i), 16 * NW + l);
  }
  for (int r = tid; r < 2 * (256 + 32); r += 512) (&vb[0][0])[r] = cmk(0.0, 0.0);
  __syncthreads();
  int base = 0;
  // reflector c from the window xv of column c (run by the owning group), rows c..m0+c
  auto form = [&](int c, const c2* xv) {
    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const int r = base + 16 * q + l;
      if (r >= c && r <= m0 + c) ss += cabs2(xv[q]);
    }
    ss = row16_sum(ss);
    const int q0 = (c - base) >> 4, l0 = (c - base) & 15;
    c2 x0 = cmk(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < NW; ++q)
      if (q == q0) x0 = cmk(lane_bcast(xv[q].x, gl0 + l0), lane_bcast(xv[q].y, gl0 + l0));
    const double nrm = sqrt(ss);
    double tau = 0.0;
    c2 beta = x0, v0 = cmk(0.0, 0.0);
    if (nrm > 0.0) {
      const double ax = sqrt(cabs2(x0));
      const c2 ph = ax > 0.0 ? cscale(1.0 / ax, x0) : cmk(1.0, 0.0);
      beta = cscale(-nrm, ph);
      v0 = csub(x0, beta);
      const double vn2 = ss - cabs2(x0) + cabs2(v0);
      tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
    }
    const int col = c;
    c2* vbc = vb[c & 1];
    c2* vg = Vj + (int64_t)c * m2;
    c2* hc = h + (int64_t)col * ldh;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
      const int r = base + 16 * q + l;
      const bool sup = tau != 0.0 && r >= c && r <= m0 + c;
      const c2 val = sup ? (r == c ? v0 : xv[q]) : cmk(0.0, 0.0);
      vbc[r] = val;
      if (r < m2) vg[r] = val;
      // the finished column: beta on row c, zeros below it on the support
      if (r <= m0 + col) hc[r] = (tau != 0.0 && r >= c) ? (r == c ? beta : cmk(0.0, 0.0)) : xv[q];
    }
    vbc[base + 16 * NW + l] = cmk(0.0, 0.0);  // the readers' window may reach one slot further
    for (int r = l; r < base; r += 16) vg[r] = cmk(0.0, 0.0);
    for (int r = base + 16 * NW + l; r < m2; r += 16) vg[r] = cmk(0.0, 0.0);
    if (l == 0) {
      tj[c] = tau;
      tb[c & 1] = tau;
    }
  };
  if (g == 0) form(0, x[0]);
  __syncthreads();
  // 16 steps per window position: the entering rows (loaded a window shift ahead) are consumed
  // only at a shift, so the steps in between never wait on global memory (a wait on the loads
  // would also wait on the reflectors' stores)
  for (int cw = 0; cw < m0; cw += 16) {
    if (cw > 0) {
      // the window moves down 16 rows: the top slot is final (rows below cw) in the columns still
      // updated (columns 0..cw are finished and written)
#pragma unroll
      for (int i = 0; i < MAXC; ++i) {
        const int col = colof(i);
        if (col > cw && col < m0) {
          h[(int64_t)col * ldh + base + l] = x[i][0];
#pragma unroll
          for (int q = 0; q + 1 < NW; ++q) x[i][q] = x[i][q + 1];
          x[i][NW - 1] = pf[i];
          pf[i] = ld(col, base + 16 + 16 * NW + l);
        }
      }
      base += 16;
    }
    const int cend = min(cw + 16, m0);
    for (int c = cw; c < cend; ++c) {
      const double tv = tb[c & 1];
      const bool live = tv != 0.0;
      // reflector c at this group's rows of the window (zero off its support)
      c2 vv[NW];
      const c2* vbc = vb[c & 1];
#pragma unroll
      for (int q = 0; q < NW; ++q) vv[q] = vbc[base + 16 * q + l];
#pragma unroll
      for (int i = 0; i < MAXC; ++i) {
        const int col = colof(i);
        if (live && col > c && col < m0) {
          c2 d = cmk(0.0, 0.0);
#pragma unroll
          for (int q = 0; q < NW; ++q) d = cadd(d, cjmul(vv[q], x[i][q]));
          const c2 f = cscale(tv, row16_csum(d));
#pragma unroll
          for (int q = 0; q < NW; ++q) x[i][q] = csub(x[i][q], cmul(f, vv[q]));
        }
      }
      if (c + 1 < m0 && g == (c + 1) % NG) {
        // the owner of column c + 1 (its slot (c + 1) / 32) forms reflector c + 1
        const int io = (c + 1) / NG;
        c2 xv[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) xv[q] = x[0][q];
#pragma unroll
        for (int i = 1; i < MAXC; ++i)
          if (i == io)
#pragma unroll
            for (int q = 0; q < NW; ++q) xv[q] = x[i][q];
        form(c + 1, xv);
      }
      __syncthreads();
    }
  }
}

// y = R^{-1} g_top (column-oriented back substitution, one wave per right-hand side)
// and u = Q_H [0; g_tail] (reflectors in reverse order).  grid (ns, ceil(m0/4)).
template <bool GLOBAL>
__global__ __launch_bounds__(256) void k_lsq_finish(LsqArgs a) {
  extern __shared__ c2 colbuf[];  // 4 x ldh
  const int s = blockIdx.x;
  const int J = a.iters[s];
  if (J == 0) return;
  const LsqView v = lsq_view(a, s);
  const int m0 = a.m0, ldh = a.ldh, m2 = 2 * m0, ldy = a.k * m0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = blockIdx.y * 4 + wave;
  if (col >= m0) return;
  const int n = J * m0;
  // GLOBAL: solve in place in the column of y (and form u in place in u)
  c2* x = GLOBAL ? v.y + (int64_t)col * ldy : colbuf + wave * ldh;
  const c2* gc = v.g + (int64_t)col * ldh;
  for (int r = lane; r < n; r += 64) x[r] = gc[r];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int c = n - 1; c >= 0; --c) {
    const c2* Rc = v.H + (int64_t)c * ldh;  // column c of R
    const c2 d = Rc[c];
    const c2 yc = cabs2(d) > 1e-300 ? cdiv(x[c], d) : cmk(0.0, 0.0);
    const int rlo = a.band > 0 ? max(0, (c / m0 - a.band - 1) * m0) : 0;
    for (int r = rlo + lane; r < c; r += 64) x[r] = csub(x[r], cmul(Rc[r], yc));
    if (lane == 0) x[c] = yc;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  }
  c2* yc = v.y + (int64_t)col * ldy;
  for (int r = lane; r < ldy; r += 64)
    if (!GLOBAL || r >= n) yc[r] = r < n ? x[r] : cmk(0.0, 0.0);
  if (!a.need_u) return;
  // u = Q_H [0; g_tail]
  if (GLOBAL) x = v.u + (int64_t)col * ldh;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int r = lane; r < ldh; r += 64) x[r] = (r >= n && r < n + m0) ? gc[r] : cmk(0.0, 0.0);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  for (int i = J - 1; i >= 0; --i)
    wave_reflect_run(v.Vh + (int64_t)i * m2 * m0, v.tau + i * m0, m0, m2, x + i * m0, lane, true);
  if (!GLOBAL) {
    c2* uc = v.u + (int64_t)col * ldh;
    for (int r = lane; r < ldh; r += 64) uc[r] = x[r];
  }
}

// y = R^{-1} g_top for a block-banded R (no u): block back substitution from the last block
// row up.  Per block b: the diagonal block R_bb (packed upper triangle, its diagonal as
// reciprocals) is staged in LDS once for the workgroup's four right-hand sides (one wave
// each) and solved column by column, then the rows of blocks b - band - 1 .. b - 1 take
// the products with R's block column b.  Each wave keeps its right-hand side's rows of the band + 2 blocks that the
// current block row touches in an LDS window (row r in slot r mod (band + 2) m0); solved
// blocks go to y, the next block above comes in from g.  grid (ns, ceil(m0/4)); LDS:
// m0 (m0 + 1) / 2 + 4 (band + 2) m0 complex.
__global__ __launch_bounds__(256) void k_lsq_finish_band(LsqArgs a) {
  extern __shared__ c2 fb_lds[];
  const int s = blockIdx.x;
  const int J = a.iters[s];
  if (J == 0) return;
  const LsqView v = lsq_view(a, s);
  const int m0 = a.m0, ldh = a.ldh, ldy = a.k * m0;
  const int WB = a.band + 2, W = WB * m0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int col = blockIdx.y * 4 + wave;
  const bool live = col < m0;  // dead waves still join the workgroup barriers
  c2* Rd = fb_lds;                                  // packed R_bb, column cl at cl (cl + 1) / 2
  c2* x = fb_lds + m0 * (m0 + 1) / 2 + wave * W;    // this wave's window
  const int n = J * m0;
  const c2* gc = v.g + (int64_t)(live ? col : 0) * ldh;
  c2* yc = v.y + (int64_t)(live ? col : 0) * ldy;
  if (live) {
    for (int r = n + lane; r < ldy; r += 64) yc[r] = cmk(0.0, 0.0);
    for (int r = max(0, n - W) + lane; r < n; r += 64) x[r % W] = gc[r];
  }
  for (int b = J - 1; b >= 0; --b) {
    const int b0 = b * m0;
    c2* xb = x + (b % WB) * m0;  // window slots of block b
    __syncthreads();
    for (int idx = tid; idx < m0 * (m0 + 1) / 2; idx += blockDim.x) {
      int cl = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
      while (cl * (cl + 1) / 2 > idx) --cl;
      while ((cl + 1) * (cl + 2) / 2 <= idx) ++cl;
      const int r = idx - cl * (cl + 1) / 2;
      const c2 h = v.H[(int64_t)(b0 + cl) * ldh + b0 + r];
      // the diagonal is kept as its reciprocal (0 for a deflated column)
      Rd[idx] = r == cl ? (cabs2(h) > 1e-300 ? cdiv(cmk(1.0, 0.0), h) : cmk(0.0, 0.0)) : h;
    }
    __syncthreads();
    if (live) {
      // triangular solve with R_bb on the rows of block b
      for (int cl = m0 - 1; cl >= 0; --cl) {
        const c2* Rc = Rd + cl * (cl + 1) / 2;
        const c2 yv = cmul(xb[cl], Rc[cl]);
        for (int r = lane; r < cl; r += 64) xb[r] = csub(xb[r], cmul(Rc[r], yv));
        if (lane == 0) xb[cl] = yv;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
      // rows of the blocks above within the band: x -= R(rows, block b) y_b
      const int rlo = max(0, (b - a.band - 1) * m0);
      for (int r0 = rlo; r0 < b0; r0 += 64) {
        const int r = r0 + lane;
        if (r < b0) {
          c2 acc = cmk(0.0, 0.0);
          const c2* Hr = v.H + (int64_t)b0 * ldh + r;
          // 16 independent loads in flight per chunk (m0 is a multiple of 16)
          for (int c0 = 0; c0 < m0; c0 += 16) {
            c2 hv[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) hv[u] = Hr[(int64_t)(c0 + u) * ldh];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc = cadd(acc, cmul(hv[u], xb[c0 + u]));
          }
          c2& t = x[((r / m0) % WB) * m0 + r % m0];
          t = csub(t, acc);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      // block b is solved: out to y; its slots take the block that block row b - 1 reaches
      const int nb = b - WB;
      for (int r = lane; r < m0; r += 64) {
        yc[b0 + r] = xb[r];
        if (nb >= 0) xb[r] = gc[nb * m0 + r];
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }
}

// y = R^{-1} g_top for a full upper triangular R (the non-Hermitian Hessenberg keeps every block
// above the diagonal), blocked and spread over the device, from the last block row up.  Per block
// row b two launches: SOLVE takes y_{b+1} out of block row b (x_b -= R(b, b+1) y_{b+1}) and solves
// R_bb y_b = x_b; the other takes y_{b+1} out of every block row rb < b.  Each workgroup handles one
// block row, one shift and 16 right-hand sides (q): wave w holds right-hand sides 16 q + 4 w .. + 3,
// lane l the rows l and l + 64 of the block in registers.  The products run on LDS chunks of 16
// columns of R and 16 rows of y_{b+1}; the solve on R_bb's packed upper triangle in LDS.  The
// working x lives in y itself (k_lsq_bsub_init copies g_top there).  grid (1 or b, ns, m0 / 16).
constexpr int kBsubRows = 2;  // row slots per lane: m0 <= 128 rows per block

__global__ void k_lsq_bsub_init(LsqArgs a) {
  const int s = blockIdx.x, col = blockIdx.y;
  const int J = a.iters[s];
  const LsqView v = lsq_view(a, s);
  const int n = J * a.m0, ldy = a.k * a.m0;
  const c2* gc = v.g + (int64_t)col * a.ldh;
  c2* yc = v.y + (int64_t)col * ldy;
  for (int r = threadIdx.x; r < ldy; r += blockDim.x) yc[r] = r < n ? gc[r] : cmk(0.0, 0.0);
}

template <bool SOLVE>
__global__ __launch_bounds__(256) void k_lsq_bsub(LsqArgs a, int b) {
  extern __shared__ c2 bs_lds[];
  const int rb = SOLVE ? b : blockIdx.x, s = blockIdx.y, q = blockIdx.z;
  const int J = a.iters[s];
  if (b >= J || (!SOLVE && b + 1 >= J)) return;  // this shift's solve starts lower down
  const LsqView v = lsq_view(a, s);
  const int m0 = a.m0, ldh = a.ldh, ldy = a.k * m0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  c2* Rc = bs_lds;            // 16 x m0: R(rows of block rb, 16 columns of block b + 1)
  c2* Yc = Rc + 16 * m0;      // 16 x 16: the matching rows of y_{b+1}, this group's right-hand sides
  c2* Rp = Yc + 16 * 16;      // packed upper triangle of R_bb, column c at c (c + 1) / 2
  const int r0 = rb * m0;
  const int rhs0 = 16 * q + 4 * wave;
  c2 x[kBsubRows][4];
#pragma unroll
  for (int t = 0; t < kBsubRows; ++t) {
    const int r = lane + 64 * t;
#pragma unroll
    for (int u = 0; u < 4; ++u) x[t][u] = r < m0 ? v.y[(int64_t)(rhs0 + u) * ldy + r0 + r] : cmk(0.0, 0.0);
  }
  if (b + 1 < J) {
    // x -= R(rb, b+1) y_{b+1}, 16 columns at a time
    const int c0 = (b + 1) * m0;
    c2 acc[kBsubRows][4];
#pragma unroll
    for (int t = 0; t < kBsubRows; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[t][u] = cmk(0.0, 0.0);
    for (int kc = 0; kc < m0; kc += 16) {
      __syncthreads();
      for (int idx = tid; idx < 16 * m0; idx += 256) {
        const int kk = idx / m0, r = idx % m0;
        Rc[idx] = v.H[(int64_t)(c0 + kc + kk) * ldh + r0 + r];
      }
      {
        const int kk = tid & 15, c = tid >> 4;
        Yc[kk * 16 + c] = v.y[(int64_t)(16 * q + c) * ldy + c0 + kc + kk];
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < 16; ++kk) {
        c2 yv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) yv[u] = Yc[kk * 16 + 4 * wave + u];
#pragma unroll
        for (int t = 0; t < kBsubRows; ++t) {
          const int r = lane + 64 * t;
          const c2 rv = r < m0 ? Rc[kk * m0 + r] : cmk(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[t][u] = cadd(acc[t][u], cmul(rv, yv[u]));
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kBsubRows; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) x[t][u] = csub(x[t][u], acc[t][u]);
  }
  if (!SOLVE) {
#pragma unroll
    for (int t = 0; t < kBsubRows; ++t) {
      const int r = lane + 64 * t;
      if (r < m0)
#pragma unroll
        for (int u = 0; u < 4; ++u) v.y[(int64_t)(rhs0 + u) * ldy + r0 + r] = x[t][u];
    }
    return;
  }
  // block row b: R_bb y_b = x_b.  R_bb's upper triangle to LDS; each lane keeps the reciprocal of
  // its rows' diagonal (0 for a deflated column)
  for (int idx = tid; idx < m0 * (m0 + 1) / 2; idx += 256) {
    int c = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while (c * (c + 1) / 2 > idx) --c;
    while ((c + 1) * (c + 2) / 2 <= idx) ++c;
    const int r = idx - c * (c + 1) / 2;
    Rp[idx] = v.H[(int64_t)(r0 + c) * ldh + r0 + r];
  }
  c2 rinv[kBsubRows];
#pragma unroll
  for (int t = 0; t < kBsubRows; ++t) {
    const int r = lane + 64 * t;
    const c2 d = r < m0 ? v.H[(int64_t)(r0 + r) * ldh + r0 + r] : cmk(0.0, 0.0);
    rinv[t] = cabs2(d) > 1e-300 ? cdiv(cmk(1.0, 0.0), d) : cmk(0.0, 0.0);
  }
  __syncthreads();
  // column-oriented back substitution on registers: row c's solution comes from its lane, the
  // rows above take R(r, c) y_c
  for (int c = m0 - 1; c >= 0; --c) {
    const int slot = c >> 6, owner = c & 63;
    const c2* col = Rp + c * (c + 1) / 2;
    c2 rv[kBsubRows];
#pragma unroll
    for (int t = 0; t < kBsubRows; ++t) {
      const int r = lane + 64 * t;
      rv[t] = r < c ? col[r] : cmk(0.0, 0.0);
    }
    c2 yc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c2 mine = cmk(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < kBsubRows; ++t)
        if (t == slot) mine = cmul(x[t][u], rinv[t]);
      yc[u] = cmk(lane_bcast(mine.x, owner), lane_bcast(mine.y, owner));
    }
#pragma unroll
    for (int t = 0; t < kBsubRows; ++t) {
      const int r = lane + 64 * t;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (r < c) x[t][u] = csub(x[t][u], cmul(rv[t], yc[u]));
        if (r == c) x[t][u] = yc[u];
      }
    }
  }
#pragma unroll
  for (int t = 0; t < kBsubRows; ++t) {
    const int r = lane + 64 * t;
    if (r < m0)
#pragma unroll
      for (int u = 0; u < 4; ++u) v.y[(int64_t)(rhs0 + u) * ldy + r0 + r] = x[t][u];
  }
}

// Yq[s][b]: (2m0 x m0) real form for Q += Re(V_b (wf y_b)); Uc[s][b]: (2m0 x 2m0) real form of u_b.
template <class T>
__global__ void k_make_coefs(LsqArgs a, const double* __restrict__ wfac, int jmax, T* __restrict__ Yq,
                             T* __restrict__ Uc, int complex_out) {
  const int s = blockIdx.x, b = blockIdx.y;  // b in [0, jmax]
  const int J = a.iters[s];
  const LsqView v = lsq_view(a, s);
  const int m0 = a.m0, m2 = 2 * m0, ldh = a.ldh, ldy = a.k * m0;
  const c2 wf = cmk(wfac[2 * s], wfac[2 * s + 1]);
  if (b < jmax) {
    const int ow = complex_out ? m2 : m0;
    T* Y = Yq + ((int64_t)s * jmax + b) * m2 * ow;
    for (int idx = threadIdx.x; idx < m0 * m0; idx += blockDim.x) {
      const int c = idx / m0, d = idx % m0;
      const c2 yv = (b < J) ? cmul(wf, v.y[b * m0 + c + (int64_t)d * ldy]) : cmk(0.0, 0.0);
      if (complex_out) {
        store_realified(Y, m2, c, d, yv);
      } else {
        Y[(2 * c) * ow + d] = (T)yv.x;
        Y[(2 * c + 1) * ow + d] = (T)(-yv.y);
      }
    }
  }
  T* U = Uc + ((int64_t)s * (jmax + 1) + b) * m2 * m2;
  for (int idx = threadIdx.x; idx < m0 * m0; idx += blockDim.x) {
    const int c = idx / m0, d = idx % m0;
    const c2 uv = (b <= J) ? v.u[b * m0 + c + (int64_t)d * ldh] : cmk(0.0, 0.0);
    store_realified(U, m2, c, d, uv);
  }
}

// ------------------------------------------------------------ Rayleigh-Ritz
// Outputs of an m0 x m0 product per thread of the 1024-thread Rayleigh-Ritz kernel (m0 <= 128).
constexpr int kRrPer = 16;

__global__ __launch_bounds__(1024) void k_rr_small(int m0, const double* __restrict__ GA, const double* __restrict__ GB,
                                                  double* __restrict__ lam, double* __restrict__ C,
                                                  double* __restrict__ eta, double* __restrict__ work,
                                                  int v_in_lds) {
  extern __shared__ double sm[];  // m0 * m0, then (v_in_lds) the m0 * m0 rotation accumulator
  __shared__ double red[16];
  __shared__ double dsc[128], th[128];
  __shared__ int order[128];
  const int tid = threadIdx.x, mm = m0 * m0;
  double* U = work;
  double* Tm = work + mm;
  double* W = work + 2 * mm;
  double* Ar = work + 3 * mm;
  RR_MARK(0);
  // 1. scaled, symmetrised B-Gram
  for (int a = tid; a < m0; a += blockDim.x) {
    const double d = GB[a * m0 + a];
    dsc[a] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
  }
  __syncthreads();
  for (int idx = tid; idx < mm; idx += blockDim.x) {
    const int r = idx / m0, c = idx % m0;
    sm[idx] = 0.5 * (GB[r * m0 + c] + GB[c * m0 + r]) * dsc[r] * dsc[c];
  }
  __syncthreads();
  if (v_in_lds)
    sym_eig_ql(sm, m0, U, red, sm + mm, W);
  else
    jacobi_eig(sm, m0, U, red, nullptr);
  RR_MARK(1);
  // 2. floor tiny eigenvalues (SVQB), T = D U Theta^{-1/2}
  double tmax = 0.0;
  for (int a = tid; a < m0; a += blockDim.x) tmax = fmax(tmax, sm[a * m0 + a]);
  tmax = block_max(tmax, red);
  for (int a = tid; a < m0; a += blockDim.x) th[a] = 1.0 / sqrt(fmax(sm[a * m0 + a], 2.220446049250313e-16 * m0 * tmax));
  __syncthreads();
  for (int idx = tid; idx < mm; idx += blockDim.x) {
    const int r = idx / m0, c = idx % m0;
    Tm[idx] = dsc[r] * U[idx] * th[c];
  }
  __syncthreads();
  // 3. Ar = T^T GA T (symmetrised), via W = GA T
  RR_MARK(2);
  if (v_in_lds) {
    // products from LDS: sa = sym(GA), sb = T; then sa = W, sb = Ar
    double* sa = sm;
    double* sb = sm + mm;
    for (int idx = tid; idx < mm; idx += blockDim.x) {
      const int r = idx / m0, c = idx % m0;
      sa[idx] = 0.5 * (GA[r * m0 + c] + GA[c * m0 + r]);
      sb[idx] = Tm[idx];
    }
    __syncthreads();
    double acc[kRrPer];
#pragma unroll
    for (int t = 0; t < kRrPer; ++t) {
      const int idx = tid + t * (int)blockDim.x;
      double sum = 0.0;
      if (idx < mm) {
        const int r = idx / m0, c = idx % m0;
        for (int e = 0; e < m0; ++e) sum += sa[r * m0 + e] * sb[e * m0 + c];
      }
      acc[t] = sum;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kRrPer; ++t) {
      const int idx = tid + t * (int)blockDim.x;
      if (idx < mm) sa[idx] = acc[t];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kRrPer; ++t) {
      const int idx = tid + t * (int)blockDim.x;
      double sum = 0.0;
      if (idx < mm) {
        const int r = idx / m0, c = idx % m0;
        for (int e = 0; e < m0; ++e) sum += sb[e * m0 + r] * sa[e * m0 + c];
      }
      acc[t] = sum;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kRrPer; ++t) {
      const int idx = tid + t * (int)blockDim.x;
      if (idx < mm) sb[idx] = acc[t];
    }
    __syncthreads();
    for (int idx = tid; idx < mm; idx += blockDim.x) {
      const int r = idx / m0, c = idx % m0;
      sa[idx] = 0.5 * (sb[r * m0 + c] + sb[c * m0 + r]);
    }
    __syncthreads();
    RR_MARK(3);
    sym_eig_ql(sm, m0, W, red, sm + mm, U);
  } else {
    for (int idx = tid; idx < mm; idx += blockDim.x) {
      const int r = idx / m0, c = idx % m0;
      double sum = 0.0;
      for (int e = 0; e < m0; ++e) sum += 0.5 * (GA[r * m0 + e] + GA[e * m0 + r]) * Tm[e * m0 + c];
      W[idx] = sum;
    }
    __syncthreads();
    for (int idx = tid; idx < mm; idx += blockDim.x) {
      const int r = idx / m0, c = idx % m0;
      double sum = 0.0;
      for (int e = 0; e < m0; ++e) sum += Tm[e * m0 + r] * W[e * m0 + c];
      Ar[idx] = sum;
    }
    __syncthreads();
    for (int idx = tid; idx < mm; idx += blockDim.x) {
      const int r = idx / m0, c = idx % m0;
      sm[idx] = 0.5 * (Ar[r * m0 + c] + Ar[c * m0 + r]);
    }
    __syncthreads();
    jacobi_eig(sm, m0, W, red, nullptr);
  }
  // 4. ascending order, C = T W(:, order), eta = 1/||c_l||
  RR_MARK(4);
  __shared__ double evs[128];
  // ascending ranks of the diagonal (ties by index), one thread per entry
  for (int c = tid; c < m0; c += blockDim.x) {
    const double key = sm[c * m0 + c];
    int rank = 0;
    for (int j = 0; j < m0; ++j) {
      const double v = sm[j * m0 + j];
      rank += (v < key || (v == key && j < c)) ? 1 : 0;
    }
    order[rank] = c;
    evs[rank] = key;
  }
  __syncthreads();
  if (v_in_lds) {
    double* sa = sm;
    double* sb = sm + mm;
    for (int idx = tid; idx < mm; idx += blockDim.x) {
      sa[idx] = Tm[idx];
      sb[idx] = W[idx];
    }
    __syncthreads();
    double acc[kRrPer];
#pragma unroll
    for (int t = 0; t < kRrPer; ++t) {
      const int idx = tid + t * (int)blockDim.x;
      double sum = 0.0;
      if (idx < mm) {
        const int r = idx / m0, oc = order[idx % m0];
        for (int e = 0; e < m0; ++e) sum += sa[r * m0 + e] * sb[e * m0 + oc];
        C[idx] = sum;
      }
      acc[t] = sum;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kRrPer; ++t) {
      const int idx = tid + t * (int)blockDim.x;
      if (idx < mm) sa[idx] = acc[t];
    }
    __syncthreads();
    for (int c = tid; c < m0; c += blockDim.x) {
      lam[c] = evs[c];
      double ss = 0.0;
      for (int r = 0; r < m0; ++r) ss += sa[r * m0 + c] * sa[r * m0 + c];
      eta[c] = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
    }
    RR_MARK(5);
    return;
  }
  for (int idx = tid; idx < mm; idx += blockDim.x) {
    const int r = idx / m0, c = idx % m0;
    const int oc = order[c];
    double sum = 0.0;
    for (int e = 0; e < m0; ++e) sum += Tm[r * m0 + e] * W[e * m0 + oc];
    C[idx] = sum;
  }
  __syncthreads();
  for (int c = tid; c < m0; c += blockDim.x) {
    lam[c] = evs[c];
    double ss = 0.0;
    for (int r = 0; r < m0; ++r) ss += C[r * m0 + c] * C[r * m0 + c];
    eta[c] = ss > 0.0 ? 1.0 / sqrt(ss) : 0.0;
  }
}

__global__ void k_classify(ClassifyArgs a, const double* __restrict__ lam, const double* __restrict__ lam_im,
                           const double* __restrict__ resid, const double* __restrict__ eta, int* __restrict__ flags,
                           double* __restrict__ out) {
  __shared__ double red[8];
  const int tid = threadIdx.x;
  double rf_in = 0.0, rf_geo = 0.0, rf_all = 0.0, cnt = 0.0, cgeo = 0.0;
  for (int j = tid; j < a.m0; j += 256) {
    const double l = lam[j], li = lam_im != nullptr ? lam_im[j] : 0.0;
    bool geo;
    if (a.kind == IFEAST_CONTOUR_CIRCLE) {
      geo = hypot(l - a.c_re, li - a.c_im) < a.r;
    } else {
      geo = (l > a.emin) && (l < a.emax);
    }
    // rho_hat(lambda) = sum_k w_k / (z_k - lambda)  (2 Re for half contours, real lambda)
    double rr = 0.0, ri = 0.0;
    for (int k = 0; k < a.nc; ++k) {
      const double zr = a.z[2 * k] - l, zi = a.z[2 * k + 1] - li;
      const double d = zr * zr + zi * zi;
      const double wr = a.w[2 * k], wi = a.w[2 * k + 1];
      rr += (wr * zr + wi * zi) / d;
      ri += (wi * zr - wr * zi) / d;
    }
    const double rho = a.half ? 2.0 * fabs(rr) : hypot(rr, ri);
    const bool ok = eta[j] >= a.tau * rho;
    int f = 0;
    if (geo && ok) f |= IFEAST_FLAG_INSIDE;
    if (geo && !ok) f |= IFEAST_FLAG_SPURIOUS;
    flags[j] = f;
    const double rj = resid[j];
    rf_all = fmax(rf_all, rj);
    if (geo) {
      rf_geo = fmax(rf_geo, rj);
      cgeo += 1.0;
    }
    if (geo && ok) {
      rf_in = fmax(rf_in, rj);
      cnt += 1.0;
    }
  }
  rf_in = block_max(rf_in, red);
  rf_geo = block_max(rf_geo, red);
  rf_all = block_max(rf_all, red);
  cnt = block_sum(cnt, red);
  cgeo = block_sum(cgeo, red);
  if (tid == 0) {
    out[0] = cnt > 0.0 ? rf_in : (cgeo > 0.0 ? rf_geo : rf_all);
    out[1] = cnt;
    out[2] = cgeo;  // Ritz values inside the contour, counted or not
  }
}

// ----------------------------------------------------------- elementwise
__global__ void k_col_sumsq(int64_t n, int m, const double* __restrict__ X, double* __restrict__ partial,
                            int64_t rows_per_block) {
  __shared__ double acc[256];
  const int tid = threadIdx.x;
  const int lanes = 256 / m;  // rows processed in parallel
  const int c = tid % m, lr = tid / m;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block, r1 = min(n, r0 + rows_per_block);
  double s = 0.0;
  if (lr < lanes)
    for (int64_t r = r0 + lr; r < r1; r += lanes) {
      const double x = X[r * m + c];
      s += x * x;
    }
  acc[tid] = (lr < lanes) ? s : 0.0;
  __syncthreads();
  if (tid < m) {
    double t = 0.0;
    for (int l = 0; l < lanes; ++l) t += acc[l * m + tid];
    partial[(int64_t)blockIdx.x * m + tid] = t;
  }
}

__global__ void k_col_sumsq_finish(int nb, int m, const double* __restrict__ partial, double* __restrict__ out,
                                   int do_sqrt) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += partial[(int64_t)b * m + c];
  out[c] = do_sqrt ? sqrt(t) : t;
}

__global__ void k_scale_cols(int64_t n, int m, const double* __restrict__ X, const double* __restrict__ f,
                             double* __restrict__ Y) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  Y[idx] = X[idx] * f[idx % m];
}

__global__ void k_residual(int64_t n, int m, const double* __restrict__ AX, const double* __restrict__ BX,
                           const double* __restrict__ lam, double* __restrict__ R) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  R[idx] = AX[idx] - BX[idx] * lam[idx % m];
}

template <class T>
__global__ void k_rhs_build(int64_t n, int m0, int ns, const double* __restrict__ R, const double* __restrict__ lam,
                            const double* __restrict__ z, T* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ldc = ns * m0;
  if (idx >= n * ldc) return;
  const int64_t row = idx / ldc;
  const int col = (int)(idx % ldc);
  const int s = col / m0, j = col % m0;
  // R_ij / (z_s - lambda_j)
  const double ar = z[2 * s] - lam[j], ai = z[2 * s + 1];
  const double d = ar * ar + ai * ai;
  const double r = R[row * m0 + j];
  out[2 * idx] = (T)(r * ar / d);
  out[2 * idx + 1] = (T)(-r * ai / d);
}

__global__ void k_fill_zero(uint32_t* p, int64_t words) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < words) p[idx] = 0u;
}

inline unsigned nblocks(int64_t total, int bs = 256) { return (unsigned)((total + bs - 1) / bs); }

}  // namespace

// ------------------------------------------------------------------ launchers
template <class T>
void launch_cholqr_factor(hipStream_t st, int ns, int m0, const double* G, double shift_rel, const int* active,
                          T* Tinv, cd* Racc, int accumulate, cd* work, bool real) {
  IF_REQUIRE(m0 <= 128, "cholqr: m0 > 128");
  // squared norms below this are not resolved by products in T
  const double dead_thr = sizeof(T) == 4 ? 1e-30 : 1e-280;
  // pivots of a shifted pass stay above the shift; an unshifted pass follows a shifted
  // one whose output Gram has pivots of order that shift unless columns are dependent
  const double eps = sizeof(T) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16;
  const double tau_dep = shift_rel > 0.0 ? 0.5 * shift_rel : 0.25 * m0 * eps;
  static int max_lds = -1;
  if (max_lds < 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) max_lds = 0;
  }
  size_t lds = ((size_t)m0 * (m0 + 1) / 2 + m0) * sizeof(c2);
  static const bool force_global = getenv("IFEAST_CHOLQR_GLOBAL") != nullptr;
  static const bool force_unblocked = getenv("IFEAST_CHOLQR_UNBLOCKED") != nullptr;
  if ((int64_t)lds + 2048 <= (int64_t)max_lds && !force_global) {
    // the previous R factor beside L when there is room
    const size_t with_ra = lds + (size_t)m0 * m0 * sizeof(c2);
    const int ra_in_lds = (accumulate && (int64_t)with_ra + 2048 <= (int64_t)max_lds) ? 1 : 0;
    if (ra_in_lds) lds = with_ra;
    const size_t lds_real = ((size_t)m0 * (m0 + 1) + (size_t)m0 * m0 + 16 * (size_t)m0) * sizeof(double);
    if (real && m0 <= 80 && ns == 1 && active == nullptr && (int64_t)lds_real + 2048 <= (int64_t)max_lds &&
        !force_unblocked) {
      if (lds_real > 64 * 1024)
        IF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cholqr_real<T>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_real));
      hipLaunchKernelGGL((k_cholqr_real<T>), dim3(1), dim3(512), lds_real, st, m0, G, shift_rel, dead_thr, tau_dep,
                         Tinv, reinterpret_cast<c2*>(Racc), accumulate, nullptr, 0, nullptr, 0, 0, nullptr,
                         nullptr);
    } else if (real) {
      if (lds > 64 * 1024)
        IF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cholqr_lds<T, true>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      hipLaunchKernelGGL((k_cholqr_lds<T, true>), dim3(ns), dim3(512), lds, st, m0, G, shift_rel, dead_thr, tau_dep,
                         active, Tinv, reinterpret_cast<c2*>(Racc), accumulate, reinterpret_cast<c2*>(work), ra_in_lds);
    } else {
      if (lds > 64 * 1024)
        IF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cholqr_lds<T, false>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      hipLaunchKernelGGL((k_cholqr_lds<T, false>), dim3(ns), dim3(512), lds, st, m0, G, shift_rel, dead_thr, tau_dep,
                         active, Tinv, reinterpret_cast<c2*>(Racc), accumulate, reinterpret_cast<c2*>(work),
                         ra_in_lds);
    }
  } else {
    IF_REQUIRE(!real, "cholqr: the real-block factor needs the LDS kernel");
    hipLaunchKernelGGL((k_cholqr_factor<T>), dim3(ns), dim3(256), 0, st, m0, G, shift_rel, dead_thr, tau_dep,
                       active, Tinv, reinterpret_cast<c2*>(Racc), accumulate, reinterpret_cast<c2*>(work));
  }
  IF_HIP(hipGetLastError());
}
// Certification of one Cholesky-QR pass for a real block: with the Gram scaled to a unit
// diagonal, every row's off-diagonal absolute sum <= gersh bounds the condition number by
// (1 + gersh) / (1 - gersh) (Gershgorin), and no column is below dead_thr.  single[0] /
// two[0] = certified / not; count[0] += certified.  One workgroup of 128 threads.
// 1024 threads: eight consecutive lanes share a row (m0 <= 128), each summing every eighth
// column, so the row sums take ten loads per lane instead of m0 dependent ones.
__global__ __launch_bounds__(1024) void k_gersh_flags(int m0, const double* __restrict__ G, double gersh,
                                                      double dead_thr, int* __restrict__ single,
                                                      int* __restrict__ two, int* __restrict__ count) {
  __shared__ double dsc[128];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < m0; c += blockDim.x) {
    const double d = G[c * m0 + c];
    if (!(d > dead_thr)) bad = 1;
    dsc[c] = sqrt(fmax(d, 1e-300));
  }
  __syncthreads();
  const int r = threadIdx.x >> 3, part = threadIdx.x & 7;
  double off = 0.0;
  if (r < m0) {
#pragma unroll 4
    for (int c = part; c < m0; c += 8)
      if (c != r) off += fabs(G[r * m0 + c]) / (dsc[r] * dsc[c]);
  }
  off += __shfl_xor(off, 1);
  off += __shfl_xor(off, 2);
  off += __shfl_xor(off, 4);
  if (r < m0 && part == 0 && !(off <= gersh)) bad = 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    single[0] = bad ? 0 : 1;
    two[0] = bad ? 1 : 0;
    if (count != nullptr) count[0] += bad ? 0 : 1;
  }
}

template <class T>
__global__ void k_copy_if(const int* __restrict__ flag, int64_t count, const T* __restrict__ src,
                          T* __restrict__ dst) {
  if (flag[0] == 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <class T>
void launch_cholqr_real_ctl(hipStream_t st, int m0, const double* G, double shift_rel, T* Tinv, cd* Racc,
                            int accumulate, const int* single, int role, double* Hm, int ldh, int jstep,
                            T* Hr_next, double* scratch) {
  IF_REQUIRE(m0 <= 128 && m0 % 16 == 0, "cholqr: the blocked real factor needs m0 a multiple of 16, <= 128");
  static int max_lds = -1;
  if (max_lds < 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) max_lds = 0;
  }
  const double dead_thr = sizeof(T) == 4 ? 1e-30 : 1e-280;
  const double eps = sizeof(T) == 4 ? 1.1920928955078125e-07 : 2.220446049250313e-16;
  const double tau_dep = shift_rel > 0.0 ? 0.5 * shift_rel : 0.25 * m0 * eps;
  const size_t base = ((size_t)m0 * (m0 + 1) + 16 * (size_t)m0) * sizeof(double);
  const size_t with_rs = base + (size_t)m0 * m0 * sizeof(double);
  // the previous R factor in LDS when it fits beside L (plus the kernel's static arrays)
  const bool rs_lds = (int64_t)with_rs + 4096 <= (int64_t)max_lds;
  IF_REQUIRE(rs_lds || scratch != nullptr || !accumulate, "cholqr: m0 x m0 scratch needed for this m0");
  IF_REQUIRE((int64_t)base + 4096 <= (int64_t)max_lds, "cholqr: not enough LDS for the blocked real factor");
  const size_t lds_real = rs_lds ? with_rs : base;
  if (lds_real > 64 * 1024)
    IF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_cholqr_real<T>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_real));
  hipLaunchKernelGGL((k_cholqr_real<T>), dim3(1), dim3(512), lds_real, st, m0, G, shift_rel, dead_thr, tau_dep, Tinv,
                     reinterpret_cast<c2*>(Racc), accumulate, single, role, Hm, ldh, jstep, Hr_next,
                     rs_lds ? nullptr : scratch);
  IF_HIP(hipGetLastError());
}
template void launch_cholqr_real_ctl<float>(hipStream_t, int, const double*, double, float*, cd*, int, const int*,
                                            int, double*, int, int, float*, double*);
template void launch_cholqr_real_ctl<double>(hipStream_t, int, const double*, double, double*, cd*, int,
                                             const int*, int, double*, int, int, double*, double*);

void launch_gersh_flags(hipStream_t st, int m0, const double* G, double gersh, double dead_thr, int* single, int* two,
                        int* count) {
  IF_REQUIRE(m0 <= 128, "gershgorin check: m0 > 128");
  hipLaunchKernelGGL(k_gersh_flags, dim3(1), dim3(1024), 0, st, m0, G, gersh, dead_thr, single, two, count);
  IF_HIP(hipGetLastError());
}

template <class T>
void launch_copy_if(hipStream_t st, const int* flag, int64_t count, const T* src, T* dst) {
  hipLaunchKernelGGL((k_copy_if<T>), dim3(2048), dim3(256), 0, st, flag, count, src, dst);
  IF_HIP(hipGetLastError());
}
template void launch_copy_if<float>(hipStream_t, const int*, int64_t, const float*, float*);
template void launch_copy_if<double>(hipStream_t, const int*, int64_t, const double*, double*);

template void launch_cholqr_factor<float>(hipStream_t, int, int, const double*, double, const int*, float*, cd*, int,
                                          cd*, bool);
template void launch_cholqr_factor<double>(hipStream_t, int, int, const double*, double, const int*, double*, cd*,
                                           int, cd*, bool);

template <class T>
void launch_cgs_combine(hipStream_t st, int ns, int ni, int m0, int j, int ldh, const double* G, const int* active,
                        cd* H, T* Hr, int accumulate) {
  const int64_t total = (int64_t)ns * ni * m0 * m0;
  hipLaunchKernelGGL((k_cgs_combine<T>), dim3(nblocks(total)), dim3(256), 0, st, ns, ni, m0, j, ldh, G, active,
                     reinterpret_cast<c2*>(H), Hr, accumulate);
  IF_HIP(hipGetLastError());
}
template void launch_cgs_combine<float>(hipStream_t, int, int, int, int, int, const double*, const int*, cd*,
                                        float*, int);
template void launch_cgs_combine<double>(hipStream_t, int, int, int, int, int, const double*, const int*, cd*,
                                         double*, int);

void launch_orth_check(hipStream_t st, int ns, int m0, int j, int ldh, double eta, double gersh, double dead_thr,
                       const double* G, const int* active, const cd* H, int* need, int* single, int* twopass) {
  IF_REQUIRE(m0 <= 128, "orth check: m0 > 128");
  hipLaunchKernelGGL(k_orth_check, dim3(ns), dim3(128), 0, st, m0, j, ldh, eta * eta, gersh, dead_thr, G, active,
                     reinterpret_cast<const c2*>(H), need, single, twopass);
  IF_HIP(hipGetLastError());
}

void launch_store_subdiag(hipStream_t st, int ns, int m0, int j, int ldh, const int* active, const cd* Racc,
                          cd* H) {
  const int64_t total = (int64_t)ns * m0 * m0;
  hipLaunchKernelGGL(k_store_subdiag, dim3(nblocks(total)), dim3(256), 0, st, ns, m0, j, ldh, active,
                     reinterpret_cast<const c2*>(Racc), reinterpret_cast<c2*>(H));
  IF_HIP(hipGetLastError());
}

void launch_lsq_init(hipStream_t st, const LsqArgs& a, const cd* S) {
  hipLaunchKernelGGL(k_lsq_init, dim3(a.ns), dim3(256), 0, st, a, reinterpret_cast<const c2*>(S));
  IF_HIP(hipGetLastError());
}
namespace {
template <int SH, bool RHS, int M0>
void launch_reflect_inst(hipStream_t st, const LsqArgs& a, int j, int rc, size_t lds) {
  hipLaunchKernelGGL((k_lsq_reflect<SH, RHS, M0>), dim3(a.ns, (a.m0 + 15) / 16), dim3(256), lds, st, a, j, rc);
}
// k_lsq_reflect for this m0: grid (ns, ceil(m0/16)), chunks of rc reflectors; the common block
// sizes get kernels compiled for them
template <bool RHS>
void launch_lsq_reflect(hipStream_t st, const LsqArgs& a, int j) {
  const int m2 = 2 * a.m0;
  const int rc = std::max(1, std::min(16, kChunk / m2));
  const size_t lds = (size_t)rc * m2 * sizeof(c2) + (size_t)rc * sizeof(double);
  switch (a.m0) {
    case 16: launch_reflect_inst<1, RHS, 16>(st, a, j, rc, lds); break;
    case 32: launch_reflect_inst<2, RHS, 32>(st, a, j, rc, lds); break;
    case 64: launch_reflect_inst<4, RHS, 64>(st, a, j, rc, lds); break;
    case 80: launch_reflect_inst<5, RHS, 80>(st, a, j, rc, lds); break;
    case 128: launch_reflect_inst<8, RHS, 128>(st, a, j, rc, lds); break;
    default:
      switch ((a.m0 + 15) / 16) {
#define IF_LSQ_SH(SH) \
  case SH: launch_reflect_inst<SH, RHS, 0>(st, a, j, rc, lds); break;
        IF_LSQ_SH(1) IF_LSQ_SH(2) IF_LSQ_SH(3) IF_LSQ_SH(4) IF_LSQ_SH(5) IF_LSQ_SH(6) IF_LSQ_SH(7) IF_LSQ_SH(8)
#undef IF_LSQ_SH
        default: IF_REQUIRE(false, "least squares: m0 > 128");
      }
  }
  IF_HIP(hipGetLastError());
}
template <int NW, int MAXC, int M0>
void launch_lsq_qr_regs_inst(hipStream_t st, const LsqArgs& a, int j) {
  hipLaunchKernelGGL((k_lsq_qr_regs<NW, MAXC, M0>), dim3(a.ns), dim3(512), 0, st, a, j);
  IF_HIP(hipGetLastError());
}
// k_lsq_qr_regs for this m0 (m0 <= 96); false if it does not apply
bool launch_lsq_qr_regs(hipStream_t st, const LsqArgs& a, int j) {
  switch (a.m0) {
    case 16: launch_lsq_qr_regs_inst<3, 1, 16>(st, a, j); return true;
    case 32: launch_lsq_qr_regs_inst<4, 1, 32>(st, a, j); return true;
    case 64: launch_lsq_qr_regs_inst<6, 2, 64>(st, a, j); return true;
    case 80: launch_lsq_qr_regs_inst<7, 3, 80>(st, a, j); return true;
    default:
      if (a.m0 > 96) return false;
      launch_lsq_qr_regs_inst<8, 3, 0>(st, a, j);
      return true;
  }
}
}  // namespace

void launch_lsq_step(hipStream_t st, const LsqArgs& a, int j) {
  IF_REQUIRE(a.m0 <= 128, "least squares: m0 > 128");
  if (j > 0) launch_lsq_reflect<false>(st, a, j);
  if (launch_lsq_qr_regs(st, a, j)) {
    launch_lsq_reflect<true>(st, a, j);
    hipLaunchKernelGGL(k_lsq_stop, dim3(a.ns), dim3(64), 0, st, a, j);
  } else {
    // m0 > 96: the slab in global memory, one wave per column
    hipLaunchKernelGGL(k_lsq_qr, dim3(a.ns), dim3(256), 0, st, a, j);
  }
  IF_HIP(hipGetLastError());
}
void launch_lsq_finish(hipStream_t st, const LsqArgs& a, int jmax) {
  static int max_lds = -1;
  if (max_lds < 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) max_lds = 0;
  }
  if (a.band == 0 && !a.need_u && jmax > 0 && a.m0 % 16 == 0 && a.m0 <= 64 * kBsubRows) {
    // full R: the blocked back substitution, one pair of launches per block row
    const size_t lds_upd = ((size_t)16 * a.m0 + 256) * sizeof(c2);
    const size_t lds_solve = lds_upd + (size_t)a.m0 * (a.m0 + 1) / 2 * sizeof(c2);
    if ((int64_t)lds_solve + 1024 <= (int64_t)max_lds) {
      if (lds_solve > 64 * 1024)
        IF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lsq_bsub<true>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_solve));
      hipLaunchKernelGGL(k_lsq_bsub_init, dim3(a.ns, a.m0), dim3(256), 0, st, a);
      for (int b = jmax - 1; b >= 0; --b) {
        hipLaunchKernelGGL(k_lsq_bsub<true>, dim3(1, a.ns, a.m0 / 16), dim3(256), lds_solve, st, a, b);
        if (b > 0) hipLaunchKernelGGL(k_lsq_bsub<false>, dim3(b, a.ns, a.m0 / 16), dim3(256), lds_upd, st, a, b);
      }
      IF_HIP(hipGetLastError());
      return;
    }
  }
  if (a.band > 0 && !a.need_u && a.m0 <= 128) {
    const size_t lds = ((size_t)a.m0 * (a.m0 + 1) / 2 + (size_t)4 * (a.band + 2) * a.m0) * sizeof(c2);
    if ((int64_t)lds + 1024 <= (int64_t)max_lds) {
      if (lds > 64 * 1024)
        IF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lsq_finish_band),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      hipLaunchKernelGGL(k_lsq_finish_band, dim3(a.ns, (a.m0 + 3) / 4), dim3(256), lds, st, a);
      IF_HIP(hipGetLastError());
      return;
    }
  }
  const size_t lds = (size_t)4 * a.ldh * sizeof(c2);
  if ((int64_t)lds + 1024 <= (int64_t)max_lds) {
    if (lds > 64 * 1024)
      IF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_lsq_finish<false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_lsq_finish<false>, dim3(a.ns, (a.m0 + 3) / 4), dim3(256), lds, st, a);
  } else {
    hipLaunchKernelGGL(k_lsq_finish<true>, dim3(a.ns, (a.m0 + 3) / 4), dim3(256), 0, st, a);
  }
  IF_HIP(hipGetLastError());
}

template <class T>
void launch_make_coefs(hipStream_t st, const LsqArgs& a, const double* wfac, int jmax, T* Yq, T* Uc,
                       int complex_out) {
  hipLaunchKernelGGL((k_make_coefs<T>), dim3(a.ns, jmax + 1), dim3(256), 0, st, a, wfac, jmax, Yq, Uc, complex_out);
  IF_HIP(hipGetLastError());
}
template void launch_make_coefs<float>(hipStream_t, const LsqArgs&, const double*, int, float*, float*, int);
template void launch_make_coefs<double>(hipStream_t, const LsqArgs&, const double*, int, double*, double*, int);

void launch_rr_small(hipStream_t st, int m0, const double* GA, const double* GB, double* lam, double* C, double* eta,
                     double* work) {
  IF_REQUIRE(m0 <= 128 && m0 % 2 == 0, "rayleigh-ritz: m0 must be even and <= 128");
  static int max_lds = -1;
  if (max_lds < 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) max_lds = 0;
  }
  size_t lds = (size_t)m0 * m0 * sizeof(double);
  // the Jacobi rotations accumulate in LDS too when both matrices fit
  const int v_in_lds = (int64_t)(2 * lds) + 16384 <= (int64_t)max_lds ? 1 : 0;
  if (v_in_lds) lds *= 2;
  if (lds > 64 * 1024)
    IF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_rr_small), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
  hipLaunchKernelGGL(k_rr_small, dim3(1), dim3(1024), lds, st, m0, GA, GB, lam, C, eta, work, v_in_lds);
  IF_HIP(hipGetLastError());
}

void launch_classify(hipStream_t st, const ClassifyArgs& a, const double* lam, const double* lam_im,
                     const double* resid, const double* eta, int* flags, double* out) {
  hipLaunchKernelGGL(k_classify, dim3(1), dim3(256), 0, st, a, lam, lam_im, resid, eta, flags, out);
  IF_HIP(hipGetLastError());
}

int col_sumsq_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 255) / 256)); }

void launch_col_sumsq(hipStream_t st, int64_t n, int m, const double* X, double* out, double* partial) {
  IF_REQUIRE(m <= 256, "col_sumsq: m > 256");
  const int nb = col_sumsq_blocks(n);
  const int64_t rpb = (n + nb - 1) / nb;
  hipLaunchKernelGGL(k_col_sumsq, dim3(nb), dim3(256), 0, st, n, m, X, partial, rpb);
  IF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_col_sumsq_finish, dim3(nblocks(m)), dim3(256), 0, st, nb, m, partial, out, 1);
  IF_HIP(hipGetLastError());
}

void launch_col_sumsq_finish(hipStream_t st, int nb, int m, const double* partial, double* out, int do_sqrt) {
  hipLaunchKernelGGL(k_col_sumsq_finish, dim3(nblocks(m)), dim3(256), 0, st, nb, m, partial, out, do_sqrt);
  IF_HIP(hipGetLastError());
}

void launch_scale_cols(hipStream_t st, int64_t n, int m, const double* X, const double* f, double* Y) {
  hipLaunchKernelGGL(k_scale_cols, dim3(nblocks(n * m)), dim3(256), 0, st, n, m, X, f, Y);
  IF_HIP(hipGetLastError());
}

void launch_residual(hipStream_t st, int64_t n, int m, const double* AX, const double* BX, const double* lam,
                     double* R) {
  hipLaunchKernelGGL(k_residual, dim3(nblocks(n * m)), dim3(256), 0, st, n, m, AX, BX, lam, R);
  IF_HIP(hipGetLastError());
}

template <class T>
void launch_rhs_build(hipStream_t st, int64_t n, int m0, int ns, const double* R, const double* lam, const double* z,
                      T* out) {
  hipLaunchKernelGGL((k_rhs_build<T>), dim3(nblocks(n * ns * m0)), dim3(256), 0, st, n, m0, ns, R, lam, z, out);
  IF_HIP(hipGetLastError());
}
template void launch_rhs_build<float>(hipStream_t, int64_t, int, int, const double*, const double*, const double*,
                                      float*);
template void launch_rhs_build<double>(hipStream_t, int64_t, int, int, const double*, const double*, const double*,
                                       double*);

void launch_fill_zero(hipStream_t st, void* p, size_t bytes) {
  IF_REQUIRE(bytes % 4 == 0, "fill_zero: size must be a multiple of 4");
  const int64_t words = (int64_t)(bytes / 4);
  if (words == 0) return;
  hipLaunchKernelGGL(k_fill_zero, dim3(nblocks(words)), dim3(256), 0, st, static_cast<uint32_t*>(p), words);
  IF_HIP(hipGetLastError());
}

}  // namespace ifeast
