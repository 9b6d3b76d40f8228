// Device helpers shared by the small dense kernels (one workgroup per problem, FP64):
// complex arithmetic on double2, workgroup reductions, lane broadcasts, and the symmetric
// eigensolvers of the Rayleigh-Ritz step.  Included by the translation units that use them;
// RR_MARK (phase timestamps of profiling builds) must be defined before inclusion.
#pragma once

#include <hip/hip_runtime.h>

namespace ifeast {
namespace {

typedef double2 c2;
__device__ inline c2 cmk(double r, double i) { return make_double2(r, i); }
__device__ inline c2 cadd(c2 a, c2 b) { return cmk(a.x + b.x, a.y + b.y); }
__device__ inline c2 csub(c2 a, c2 b) { return cmk(a.x - b.x, a.y - b.y); }
__device__ inline c2 cmul(c2 a, c2 b) { return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline c2 cconj(c2 a) { return cmk(a.x, -a.y); }
// conj(a) * b
__device__ inline c2 cjmul(c2 a, c2 b) { return cmk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
__device__ inline c2 cscale(double s, c2 a) { return cmk(s * a.x, s * a.y); }
__device__ inline double cabs2(c2 a) { return a.x * a.x + a.y * a.y; }
__device__ inline c2 cdiv(c2 a, c2 b) {
  const double d = cabs2(b);
  return cmk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// Block-wide reductions over 256 threads.
__device__ inline double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  __syncthreads();
  return t;
}
__device__ inline double block_max(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = sh[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) t = fmax(t, sh[i]);
  __syncthreads();
  return t;
}

// ---- 16-lane groups: lanes 16 q .. 16 q + 15 of a wave form one DPP row.
// v of another lane of the same row (CTRL: a DPP row permutation), one 32-bit half at a time.
template <int CTRL>
__device__ inline double row_perm(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// Sum over the 16 lanes of the row, in every lane of it: two quad butterflies (lane ^ 1,
// lane ^ 2), then the half-row and row mirrors, each adding the other half's partial sum.
// Every stage adds two operands that are swapped in the partner lane, so all 16 lanes end with
// the same bits.  All 16 lanes of the row must be active.
__device__ inline double row16_sum(double v) {
  v += row_perm<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += row_perm<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += row_perm<0x141>(v);  // row_half_mirror
  v += row_perm<0x140>(v);  // row_mirror
  return v;
}
__device__ inline c2 row16_csum(c2 v) { return cmk(row16_sum(v.x), row16_sum(v.y)); }

// Lane l's value of v in every lane (l wave-uniform; the whole wave active): two scalar reads
// of the register halves instead of a lane permute through the LDS unit.
// Workgroup barrier that orders LDS accesses only: global stores issued before it need not have
// completed (__syncthreads would wait for them).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ inline double lane_bcast(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Cyclic Jacobi with the round-robin pair order on a symmetric m x m matrix
// held in LDS (row-major, stride m); eigenvectors accumulate in global Vg.
// Vs: rotations accumulate in LDS (copied to Vg at the end) when given, else in Vg directly.
__device__ void jacobi_eig(double* a, int m, double* Vg, double* red, double* Vs) {
  __shared__ double cs[64], sn[64];
  __shared__ int pp[64], qq[64];
  const int tid = threadIdx.x, half = m / 2, nth = blockDim.x;
  double* V = Vs != nullptr ? Vs : Vg;
  for (int idx = tid; idx < m * m; idx += nth) V[idx] = (idx / m == idx % m) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int idx = tid; idx < m * m; idx += nth) {
      const int r = idx / m, c = idx % m;
      if (r != c) off += a[idx] * a[idx];
      else dia += a[idx] * a[idx];
    }
    off = block_sum(off, red);
    dia = block_sum(dia, red);
    // off-diagonal mass at rounding level of the diagonal: (m * eps)^2 relative
    if (off <= (double)m * m * 4.9e-32 * dia || off == 0.0) break;
    for (int round = 0; round < m - 1; ++round) {
      if (tid < half) {
        auto pos = [&](int t) { return t == 0 ? 0 : 1 + (t - 1 + round) % (m - 1); };
        const int p = pos(tid), q = pos(m - 1 - tid);
        const double apq = a[p * m + q], app = a[p * m + p], aqq = a[q * m + q];
        double c = 1.0, sv = 0.0;
        if (apq != 0.0) {
          const double th = (aqq - app) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          sv = t * c;
        }
        cs[tid] = c;
        sn[tid] = sv;
        pp[tid] = p;
        qq[tid] = q;
      }
      __syncthreads();
      // A <- J^T A J: the rotations of a round act on disjoint index pairs, so each 2 x 2
      // block (rows of pair i1, columns of pair i2) changes with rotations i1 and i2 only
      // and is updated in place by one thread
      for (int idx = tid; idx < half * half; idx += nth) {
        const int i1 = idx / half, i2 = idx % half;
        const int p1 = pp[i1], q1 = qq[i1], p2 = pp[i2], q2 = qq[i2];
        const double c1 = cs[i1], s1 = sn[i1], c2 = cs[i2], s2 = sn[i2];
        const double b00 = a[p1 * m + p2], b01 = a[p1 * m + q2];
        const double b10 = a[q1 * m + p2], b11 = a[q1 * m + q2];
        const double x00 = c2 * b00 - s2 * b01, x01 = s2 * b00 + c2 * b01;
        const double x10 = c2 * b10 - s2 * b11, x11 = s2 * b10 + c2 * b11;
        a[p1 * m + p2] = c1 * x00 - s1 * x10;
        a[q1 * m + q2] = s1 * x01 + c1 * x11;
        // the pair's own entry is annihilated by its rotation
        a[p1 * m + q2] = i1 == i2 ? 0.0 : c1 * x01 - s1 * x11;
        a[q1 * m + p2] = i1 == i2 ? 0.0 : s1 * x00 + c1 * x10;
      }
      // V <- V J (columns p, q of each pair)
      for (int idx = tid; idx < half * m; idx += nth) {
        const int i = idx / m, r = idx % m;
        const int p = pp[i], q = qq[i];
        const double c = cs[i], sv = sn[i];
        const double vp = V[r * m + p], vq = V[r * m + q];
        V[r * m + p] = c * vp - sv * vq;
        V[r * m + q] = sv * vp + c * vq;
      }
      __syncthreads();
    }
  }
  if (Vs != nullptr) {
    for (int idx = tid; idx < m * m; idx += nth) Vg[idx] = Vs[idx];
    __syncthreads();
  }
}

// Symmetric eigen-decomposition by Householder tridiagonalisation and the implicit QL
// iteration with Wilkinson-type shifts (Bowdler, Martin, Reinsch & Wilkinson, 1968), in one
// workgroup.  a (LDS, m x m, symmetric, m <= 128) is overwritten: on return its diagonal holds
// the eigenvalues and the rest is zero; Vg (global, m x m row-major) holds the eigenvectors as
// columns.  Hv: LDS scratch m x m.  save: global scratch m x m (a copy of the input, for the
// cyclic Jacobi fallback when an eigenvalue needs more than 60 QL sweeps).
// One thread runs each QL sweep's scalar recurrence and stores its rotations; every thread
// then applies them, in order, to its rows of the eigenvector matrix (rotation buffers alternate
// between sweeps, so one barrier per sweep).
__device__ void sym_eig_ql(double* a, int m, double* Vg, double* red, double* Hv, double* save) {
  __shared__ double dd[128], ee[128], bet[128], pv[128];
  __shared__ double cr[2][128], sr[2][128];
  __shared__ int sw_lo[2], sw_hi[2], sw_n[2];
  __shared__ int ql_fail;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int idx = tid; idx < m * m; idx += nth) save[idx] = a[idx];
  RR_MARK(6);
#ifdef IFEAST_RR_PROFILE
  if (tid == 0) ::ifeast_rr_prof[10] = ::ifeast_rr_prof[11] = 0;
#endif
  // ---- 1. tridiagonalisation, H_k = I - bet_k v v^T with v in row k of Hv (entries k+1 ..)
  for (int k = 0; k + 2 < m; ++k) {
    const int n1 = k + 1;
    double x = 0.0;
    for (int r = n1 + tid; r < m; r += nth) x += a[r * m + k] * a[r * m + k];
    const double sigma = block_sum(x, red);
    const double x0 = a[n1 * m + k];
    const double alpha = x0 >= 0.0 ? -sqrt(sigma) : sqrt(sigma);
    const double v0 = x0 - alpha;
    const double vn2 = sigma - x0 * x0 + v0 * v0;
    const double b = (sigma > 0.0 && vn2 > 0.0) ? 2.0 / vn2 : 0.0;
    for (int r = n1 + tid; r < m; r += nth) Hv[k * m + r] = (r == n1) ? v0 : a[r * m + k];
    if (tid == 0) {
      bet[k] = b;
      dd[k] = a[k * m + k];
      ee[k] = b != 0.0 ? alpha : x0;
    }
    __syncthreads();
    if (b != 0.0) {
      // pv = b A v on rows n1.., eight lanes per row
      {
        const int r = n1 + (tid >> 3), part = tid & 7;
        double acc = 0.0;
        if (r < m)
          for (int c = n1 + part; c < m; c += 8) acc += a[r * m + c] * Hv[k * m + c];
        acc += __shfl_xor(acc, 1);
        acc += __shfl_xor(acc, 2);
        acc += __shfl_xor(acc, 4);
        if (r < m && part == 0) pv[r] = b * acc;
      }
      __syncthreads();
      double t = 0.0;
      for (int r = n1 + tid; r < m; r += nth) t += Hv[k * m + r] * pv[r];
      const double K = 0.5 * b * block_sum(t, red);
      // A <- A - v w^T - w v^T with w = pv - K v, on rows and columns n1..
      const int nk = m - n1;
      for (int idx = tid; idx < nk * nk; idx += nth) {
        const int r = n1 + idx / nk, c = n1 + idx % nk;
        const double vr = Hv[k * m + r], vc = Hv[k * m + c];
        const double wr = pv[r] - K * vr, wc = pv[c] - K * vc;
        a[r * m + c] -= vr * wc + wr * vc;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (m >= 2) {
      dd[m - 2] = a[(m - 2) * m + m - 2];
      ee[m - 2] = a[(m - 1) * m + m - 2];
      bet[m - 2] = 0.0;
    }
    dd[m - 1] = a[(m - 1) * m + m - 1];
    ee[m - 1] = 0.0;
    bet[m - 1] = 0.0;
  }
  __syncthreads();
  // ---- 2. Q = H_0 H_1 ... (backward accumulation into a)
  RR_MARK(7);
  for (int idx = tid; idx < m * m; idx += nth) a[idx] = (idx / m == idx % m) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = m - 3; k >= 0; --k) {
    const double b = bet[k];
    if (b == 0.0) continue;
    const int n1 = k + 1, nk = m - n1;
    {
      const int c = n1 + (tid >> 3), part = tid & 7;
      double acc = 0.0;
      if (c < m)
        for (int r = n1 + part; r < m; r += 8) acc += Hv[k * m + r] * a[r * m + c];
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      acc += __shfl_xor(acc, 4);
      if (c < m && part == 0) pv[c] = b * acc;
    }
    __syncthreads();
    for (int idx = tid; idx < nk * nk; idx += nth) {
      const int r = n1 + idx / nk, c = n1 + idx % nk;
      a[r * m + c] -= Hv[k * m + r] * pv[c];
    }
    __syncthreads();
  }
  // ---- 3. implicit QL on (dd, ee): wave 0 runs each sweep's recurrence (the same values in
  // all its lanes; lane 0 stores), the other waves apply the sweep's rotations to their rows
  // of a while wave 0 computes the next sweep
  RR_MARK(8);
#ifdef IFEAST_RR_PROFILE
  if (tid == 0) ::ifeast_rr_prof[10] = ::ifeast_rr_prof[11] = 0;
#endif
  if (tid == 0) ql_fail = 0;
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63;
  if (wave == 0) {
    int l = 0, iter = 0, buf = 0;
    while (true) {
      int nrot = 0, hi = 0, lo = 0;
      while (l < m) {
        // first mx >= l whose subdiagonal entry is negligible (mx = m - 1 if none)
        int mx = m - 1;
        for (int base = 0; base < m - 1; base += 64) {
          const int idx = base + lane;
          bool neg = false;
          if (idx >= l && idx < m - 1) {
            const double ds = fabs(dd[idx]) + fabs(dd[idx + 1]);
            neg = fabs(ee[idx]) <= 2.220446049250313e-16 * ds;
          }
          const unsigned long long bal = __ballot(neg);
          if (bal != 0ull) {
            mx = base + __ffsll((long long)bal) - 1;
            break;
          }
        }
        if (mx == l) {
          ++l;
          iter = 0;
          continue;
        }
        if (++iter > 60) {
          if (lane == 0) ql_fail = 1;
          l = m;
          break;
        }
        double g = (dd[l + 1] - dd[l]) / (2.0 * ee[l]);
        double r = hypot(g, 1.0);
        g = dd[mx] - dd[l] + ee[l] / (g + (g >= 0.0 ? r : -r));
        double sv = 1.0, c = 1.0, p = 0.0;
        int i = mx - 1;
        bool cut = false;
        // the sweep reads only entries it has not written yet: load them one step ahead.
        // r and 1/r from the hardware reciprocal square root with two Newton steps
        double e_i = ee[i], d_i = dd[i], d_i1 = dd[i + 1];
        for (; i >= l; --i) {
          const double e_n = i > l ? ee[i - 1] : 0.0, d_n = i > l ? dd[i - 1] : 0.0;
          const double f = sv * e_i, bb = c * e_i;
          const double r2 = f * f + g * g;
          if (r2 == 0.0) {
            if (lane == 0) {
              ee[i + 1] = 0.0;
              dd[i + 1] = d_i1 - p;
              ee[mx] = 0.0;
            }
            cut = true;
            break;
          }
          double rs = __builtin_amdgcn_rsq(r2);
          rs = rs * (1.5 - 0.5 * r2 * rs * rs);
          rs = rs * (1.5 - 0.5 * r2 * rs * rs);
          sv = f * rs;
          c = g * rs;
          g = d_i1 - p;
          const double t = (d_i - g) * sv + 2.0 * c * bb;
          p = sv * t;
          if (lane == 0) {
            ee[i + 1] = r2 * rs;
            dd[i + 1] = g + p;
            cr[buf][i] = c;
            sr[buf][i] = sv;
          }
          g = c * t - bb;
          d_i1 = d_i;
          e_i = e_n;
          d_i = d_n;
        }
        if (!cut && lane == 0) {
          dd[l] -= p;
          ee[l] = g;
          ee[mx] = 0.0;
        }
        hi = mx - 1;
        lo = cut ? i + 1 : l;
        nrot = hi - lo + 1;
        if (nrot > 0) break;  // a sweep cut at its first rotation changed no vector: go on
      }
      if (l >= m) nrot = 0;
#ifdef IFEAST_RR_PROFILE
      if (lane == 0) {
        ::ifeast_rr_prof[10] += 1;
        ::ifeast_rr_prof[11] += nrot;
      }
#endif
      if (lane == 0) {
        sw_hi[buf] = hi;
        sw_lo[buf] = lo;
        sw_n[buf] = nrot;
      }
      __syncthreads();
      if (nrot <= 0) break;
      buf ^= 1;
    }
  } else {
    for (int buf = 0;; buf ^= 1) {
      __syncthreads();
      const int nrot = sw_n[buf];
      if (nrot <= 0) break;
      const int hi = sw_hi[buf], lo = sw_lo[buf];
      for (int r = tid - 64; r < m; r += nth - 64) {
        // rotation i changes z[i] and z[i + 1]; z[i] then feeds rotation i - 1: carried in a register
        double* z = a + r * m;
        double up = z[hi + 1];
        for (int i = hi; i >= lo; --i) {
          const double c = cr[buf][i], sv = sr[buf][i];
          const double zi = z[i];
          z[i + 1] = sv * zi + c * up;
          up = c * zi - sv * up;
        }
        z[lo] = up;
      }
    }
  }
  RR_MARK(9);
  __syncthreads();
  if (ql_fail) {
    for (int idx = tid; idx < m * m; idx += nth) a[idx] = save[idx];
    __syncthreads();
    jacobi_eig(a, m, Vg, red, Hv);
    return;
  }
  for (int idx = tid; idx < m * m; idx += nth) Vg[idx] = a[idx];
  __syncthreads();
  for (int idx = tid; idx < m * m; idx += nth) a[idx] = (idx / m == idx % m) ? dd[idx / m] : 0.0;
  __syncthreads();
}

}  // namespace
}  // namespace ifeast
