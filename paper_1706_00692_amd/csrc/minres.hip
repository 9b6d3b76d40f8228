// Batched shifted MINRES for the inner solves (standard symmetric problems, B = I).
//
// The paper's own experiments solve the shifted systems with MINRES (Sec. 2; Sec. 3 notes that
// with a short recurrence Q = V G_v is formed without storing the basis V).  For B = I the
// right-hand side of shift s and column c is r_c / (z_s - lambda_c), so every shift of column c
// works in the Krylov space of A from r_c: one real Lanczos recurrence per column serves all
// shifts,
//     A v_k = beta_k v_{k-1} + alpha_k v_k + beta_{k+1} v_{k+1},
// and for shift s the minimal-residual iterate over that space comes from the QR factorisation
// of the complex tridiagonal z_s I~ - T_k by Givens rotations (three nonzero entries per column
// of R), so the iterate is updated with direction vectors that obey a three-term recurrence:
//     d_k = (v_k - delta_k d_{k-1} - eps_k d_{k-2}) / gamma_k,   x += tau_k d_k.
// The m0 columns run side by side in one real n x m0 block (one SpMM per step), the nc shifts
// share it, and each iterate goes straight into the quadrature sum Q += Re(wf_s tau_k d_k): the
// only n-sized state per (column, shift) is d_{k-1}, d_{k-2}.
//
// Kernels: column dot products (alpha), the three-term update with its column norms (beta),
// the per-(column, shift) rotations, and the fused direction / quadrature / normalisation sweep.
#include "internal.h"

namespace ifeast {

namespace {

inline unsigned nblk(int64_t total) { return (unsigned)((total + 255) / 256); }

// Row blocks of the column reductions (at most 1024 partial sums per column).
inline int red_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 511) / 512)); }

// partial[b][c] = sum over the rows of block b of X[r][c] * Y[r][c] (FP64 sums).
template <class T>
__global__ __launch_bounds__(256) void k_mr_dot(int64_t n, int m0, const T* __restrict__ X, const T* __restrict__ Y,
                                                double* __restrict__ partial, int64_t rows_per_block) {
  __shared__ double acc[256];
  const int tid = threadIdx.x;
  const int lanes = 256 / m0;  // rows in parallel
  const int c = tid % m0, lr = tid / m0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block, r1 = min(n, r0 + rows_per_block);
  double s = 0.0;
  if (lr < lanes)
    for (int64_t r = r0 + lr; r < r1; r += lanes) s += (double)X[r * m0 + c] * (double)Y[r * m0 + c];
  acc[tid] = lr < lanes ? s : 0.0;
  __syncthreads();
  if (tid < m0) {
    double t = 0.0;
    for (int l = 0; l < lanes; ++l) t += acc[l * m0 + tid];
    partial[(int64_t)blockIdx.x * m0 + tid] = t;
  }
}

// U = A v_k - alpha v_k - beta_k v_{k-1} with MW = -A v_k (the SpMM's output), and partial sums
// of U^2 per column.  U may alias Vp (each element is read before it is written, by one thread).
template <class T>
__global__ __launch_bounds__(256) void k_mr_three(int64_t n, int m0, const T* __restrict__ MW, const T* __restrict__ V,
                                                  const T* Vp, const double* __restrict__ alpha,
                                                  const double* __restrict__ beta, T* U, double* __restrict__ partial,
                                                  int64_t rows_per_block) {
  __shared__ double acc[256];
  const int tid = threadIdx.x;
  const int lanes = 256 / m0;
  const int c = tid % m0, lr = tid / m0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block, r1 = min(n, r0 + rows_per_block);
  const T a = (T)alpha[c], b = (T)beta[c];
  double s = 0.0;
  if (lr < lanes)
    for (int64_t r = r0 + lr; r < r1; r += lanes) {
      const int64_t i = r * m0 + c;
      const T u = -MW[i] - a * V[i] - b * Vp[i];
      U[i] = u;
      s += (double)u * (double)u;
    }
  acc[tid] = lr < lanes ? s : 0.0;
  __syncthreads();
  if (tid < m0) {
    double t = 0.0;
    for (int l = 0; l < lanes; ++l) t += acc[l * m0 + tid];
    partial[(int64_t)blockIdx.x * m0 + tid] = t;
  }
}

// Column c's sum of the partials, by the 64 lanes of one wave.
__device__ inline double wave_colsum(const double* __restrict__ partial, int nb, int m0, int c) {
  double t = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) t += partial[(int64_t)b * m0 + c];
  for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
  return t;
}

struct MrState {
  int* siters;   // per shift: steps in which any of its columns iterated
  // per (column, shift), index c * ns + s
  double* c1;    // G_{k-1}: cosine
  double2* s1;   //          sine
  double* c2;    // G_{k-2}
  double2* s2;
  double2* g;    // transformed right-hand side entry k
  int* act;      // still iterating
  double4* co1;  // output of step k: (eps, delta) complex
  double4* co2;  //                   (1/gamma, wf tau) complex
  int* upd;      // the pair is updated at step k
  // per column
  double* alpha;   // alpha_k
  double* beta;    // beta_k (the coefficient of v_{k-1})
  double* bnext;   // beta_{k+1}
  double* ibnext;  // 1 / beta_{k+1} (0 on a breakdown)
  int* nact;       // pairs of the column still iterating after step k
};

__device__ inline double2 cm(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// alpha_k = v_k^T A v_k from the partial sums of v_k^T (-A v_k).  One wave per column.
__global__ __launch_bounds__(64) void k_mr_alpha(int m0, int nb, const double* __restrict__ pa,
                                                 double* __restrict__ alpha) {
  const int c = blockIdx.x;
  const double a = -wave_colsum(pa, nb, m0, c);
  if (threadIdx.x == 0) alpha[c] = a;
}

// Step k's Givens rotations for every (column, shift), one wave per column (lane s < ns a shift):
// the column of z_s I~ - T_k is (-beta_k, z_s - alpha_k, -beta_{k+1}) on rows k-1, k, k+1.
__global__ __launch_bounds__(64) void k_mr_rot(int m0, int ns, int nb, const double* __restrict__ pa,
                                               const double* __restrict__ pb, const double* __restrict__ z,
                                               const double* __restrict__ wf, const double* __restrict__ tol,
                                               MrState st, int k) {
  const int c = blockIdx.x, s = threadIdx.x;
  const bool first = k == 0;
  const double alpha = st.alpha[c];
  const double b2 = wave_colsum(pb, nb, m0, c);
  const double bn = sqrt(fmax(b2, 0.0));
  const double bk = first ? 0.0 : st.beta[c];
  int live = 0;
  if (s < ns) {
    const int p = c * ns + s;
    const bool on = st.act[p] != 0;
    st.upd[p] = on ? 1 : 0;
    if (on) {
      atomicMax(&st.siters[s], k + 1);
      const double2 zs = make_double2(z[2 * s], z[2 * s + 1]);
      // rows k-2, k-1 by G_{k-2}: (0, -beta_k) -> (eps, delta')
      const double2 s2 = st.s2[p];
      const double c2 = st.c2[p];
      const double2 eps = make_double2(-bk * s2.x, -bk * s2.y);
      const double dp = -bk * c2;  // real: c2 is real
      // rows k-1, k by G_{k-1}: (delta', z - alpha) -> (delta, gamma')
      const double2 s1 = st.s1[p];
      const double c1 = st.c1[p];
      const double2 za = make_double2(zs.x - alpha, zs.y);
      const double2 s1za = cm(s1, za);
      const double2 delta = make_double2(c1 * dp + s1za.x, s1za.y);
      const double2 gp = make_double2(-s1.x * dp + c1 * za.x, s1.y * dp + c1 * za.y);  // -conj(s1) delta' + c1 (z - a)
      // G_k annihilates -beta_{k+1} below gamma'
      const double ag = hypot(gp.x, gp.y);
      const double rho = hypot(ag, bn);
      double ck;
      double2 sk, gamma;
      if (ag > 0.0) {
        const double2 ph = make_double2(gp.x / ag, gp.y / ag);
        ck = ag / rho;
        sk = make_double2(-ph.x * bn / rho, -ph.y * bn / rho);
        gamma = make_double2(ph.x * rho, ph.y * rho);
      } else {
        ck = 0.0;
        sk = make_double2(-1.0, 0.0);
        gamma = make_double2(bn, 0.0);
      }
      const double2 g = st.g[p];
      const double2 tau = make_double2(ck * g.x, ck * g.y);
      // g <- -conj(s_k) g
      const double2 gn = cm(make_double2(-sk.x, sk.y), g);
      st.g[p] = gn;
      st.c2[p] = c1;
      st.s2[p] = s1;
      st.c1[p] = ck;
      st.s1[p] = sk;
      const double gg = gamma.x * gamma.x + gamma.y * gamma.y;
      const double2 ig = gg > 0.0 ? make_double2(gamma.x / gg, -gamma.y / gg) : make_double2(0.0, 0.0);
      const double2 wt = cm(make_double2(wf[2 * s], wf[2 * s + 1]), tau);
      st.co1[p] = make_double4(eps.x, eps.y, delta.x, delta.y);
      st.co2[p] = make_double4(ig.x, ig.y, wt.x, wt.y);
      // the minimal residual is |g_{k+1}|; a breakdown (beta_{k+1} = 0) ends the column exactly
      const bool done = !(hypot(gn.x, gn.y) > tol[s * m0 + c]) || bn == 0.0;
      st.act[p] = done ? 0 : 1;
      live = done ? 0 : 1;
    }
  }
  for (int o = 32; o > 0; o >>= 1) live += __shfl_xor(live, o);
  if (s == 0) {
    st.beta[c] = bn;
    st.bnext[c] = bn;
    st.ibnext[c] = bn > 0.0 ? 1.0 / bn : 0.0;
    st.nact[c] = live;
  }
}

// d_k = (v_k - delta d_{k-1} - eps d_{k-2}) / gamma into D2 (over d_{k-2}), Q += Re(sum_s wf tau d_k),
// and v_{k+1} = U / beta_{k+1} in place.  One thread per element (row, column).
template <class T>
__global__ __launch_bounds__(256) void k_mr_update(int64_t n, int m0, int ns, const T* __restrict__ V, T* U,
                                                   const double* __restrict__ ibn, const T* __restrict__ D1, T* D2,
                                                   MrState st, double* __restrict__ Q) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m0) return;
  const int c = (int)(idx % m0);
  const double v = (double)V[idx];
  const int64_t plane = n * m0;  // complex elements per shift
  double acc = 0.0;
  for (int s = 0; s < ns; ++s) {
    const int p = c * ns + s;
    if (!st.upd[p]) continue;
    const double4 a = st.co1[p], b = st.co2[p];
    const int64_t e = 2 * ((int64_t)s * plane + idx);
    const double d1r = (double)D1[e], d1i = (double)D1[e + 1];
    const double d2r = (double)D2[e], d2i = (double)D2[e + 1];
    // v - delta d1 - eps d2
    const double tr = v - (a.z * d1r - a.w * d1i) - (a.x * d2r - a.y * d2i);
    const double ti = -(a.z * d1i + a.w * d1r) - (a.x * d2i + a.y * d2r);
    const double dr = tr * b.x - ti * b.y, di = tr * b.y + ti * b.x;
    D2[e] = (T)dr;
    D2[e + 1] = (T)di;
    acc += b.z * dr - b.w * di;  // Re(wf tau d)
  }
  Q[idx] += acc;
  U[idx] = (T)((double)U[idx] * ibn[c]);
}

// Start: v_1 = r / ||r|| per column (beta_1 from the FP64 column norms), v_0 = 0, d = 0, and
// per (column, shift) the right-hand side entry g_1 = beta_1 / (z_s - lambda_c).
template <class T>
__global__ void k_mr_start_vec(int64_t n, int m0, const double* __restrict__ R, const double* __restrict__ rn,
                               T* __restrict__ V, T* __restrict__ Vp) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m0) return;
  const double b = rn[idx % m0];
  V[idx] = (T)(b > 0.0 ? R[idx] / b : 0.0);
  Vp[idx] = (T)0;
}

__global__ void k_mr_start_pairs(int m0, int ns, const double* __restrict__ rn, const double* __restrict__ lam,
                                 const double* __restrict__ z, MrState st) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m0 * ns) return;
  const int c = p / ns, s = p % ns;
  const double b = rn[c];
  const double ar = z[2 * s] - lam[c], ai = z[2 * s + 1];
  const double d = ar * ar + ai * ai;
  st.g[p] = make_double2(b * ar / d, -b * ai / d);
  st.c1[p] = st.c2[p] = 1.0;
  st.s1[p] = st.s2[p] = make_double2(0.0, 0.0);
  st.act[p] = b > 0.0 ? 1 : 0;
  st.upd[p] = 0;
  if (s == 0) st.beta[c] = 0.0;
  if (c == 0) st.siters[s] = 0;
}

}  // namespace

size_t minres_state_bytes(int m0, int ns) {
  const size_t pairs = (size_t)m0 * ns;
  return pairs * (8 + 16 + 8 + 16 + 16 + 4 + 32 + 32 + 4) + (size_t)m0 * (5 * 8 + 4) + (size_t)ns * 4 + 16 * 256;
}

size_t minres_partial_bytes(int64_t n, int m0) { return (size_t)red_blocks(n) * m0 * sizeof(double); }

namespace {
MrState carve_state(void* base, int m0, int ns) {
  const size_t pairs = (size_t)m0 * ns;
  char* p = static_cast<char*>(base);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) / 256 * 256;
    return q;
  };
  MrState st;
  st.siters = reinterpret_cast<int*>(take((size_t)ns * 4));
  st.c1 = reinterpret_cast<double*>(take(pairs * 8));
  st.s1 = reinterpret_cast<double2*>(take(pairs * 16));
  st.c2 = reinterpret_cast<double*>(take(pairs * 8));
  st.s2 = reinterpret_cast<double2*>(take(pairs * 16));
  st.g = reinterpret_cast<double2*>(take(pairs * 16));
  st.act = reinterpret_cast<int*>(take(pairs * 4));
  st.co1 = reinterpret_cast<double4*>(take(pairs * 32));
  st.co2 = reinterpret_cast<double4*>(take(pairs * 32));
  st.upd = reinterpret_cast<int*>(take(pairs * 4));
  st.alpha = reinterpret_cast<double*>(take((size_t)m0 * 8));
  st.beta = reinterpret_cast<double*>(take((size_t)m0 * 8));
  st.bnext = reinterpret_cast<double*>(take((size_t)m0 * 8));
  st.ibnext = reinterpret_cast<double*>(take((size_t)m0 * 8));
  st.nact = reinterpret_cast<int*>(take((size_t)m0 * 4));
  return st;
}
}  // namespace

template <class T>
int MinresRun<T>::start(hipStream_t st, const double* R, const double* rnorm, const double* lam, const double* z) {
  const int64_t tot = n * m0;
  hipLaunchKernelGGL((k_mr_start_vec<T>), dim3(nblk(tot)), dim3(256), 0, st, n, m0, R, rnorm, V, Vp);
  IF_HIP(hipGetLastError());
  launch_fill_zero(st, D1, (size_t)2 * ns * tot * sizeof(T));
  launch_fill_zero(st, D2, (size_t)2 * ns * tot * sizeof(T));
  const MrState ms = carve_state(state, m0, ns);
  hipLaunchKernelGGL(k_mr_start_pairs, dim3(nblk((int64_t)m0 * ns)), dim3(256), 0, st, m0, ns, rnorm, lam, z, ms);
  IF_HIP(hipGetLastError());
  k = 0;
  return 0;
}

template <class T>
void MinresRun<T>::step(hipStream_t st, const ifeast_matrix* A, const T* zeroshift, const double* z,
                        const double* wf, const double* tol, double* Q) {
  const int64_t tot = n * m0;
  const int nb = red_blocks(n);
  const int64_t rpb = (n + nb - 1) / nb;
  const MrState ms = carve_state(state, m0, ns);
  // W = -A v_k (the real block as n x m0/2 complex numbers, one zero shift)
  launch_spmm_shifted<T>(st, A, nullptr, 1, m0 / 2, zeroshift, nullptr, V, W);
  hipLaunchKernelGGL((k_mr_dot<T>), dim3(nb), dim3(256), 0, st, n, m0, V, W, pa, rpb);
  IF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mr_alpha, dim3(m0), dim3(64), 0, st, m0, nb, pa, ms.alpha);
  IF_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_mr_three<T>), dim3(nb), dim3(256), 0, st, n, m0, W, V, Vp, ms.alpha, ms.beta, Vp, pb, rpb);
  IF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_mr_rot, dim3(m0), dim3(64), 0, st, m0, ns, nb, pa, pb, z, wf, tol, ms, k);
  IF_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_mr_update<T>), dim3(nblk(tot)), dim3(256), 0, st, n, m0, ns, V, Vp, ms.ibnext, D1, D2, ms, Q);
  IF_HIP(hipGetLastError());
  // roles: v_{k+1} (now in Vp) becomes v_k; d_k (in D2) becomes d_{k-1}
  std::swap(V, Vp);
  std::swap(D1, D2);
  ++k;
}

template <class T>
const int* MinresRun<T>::column_active() const {
  return carve_state(state, m0, ns).nact;
}
template <class T>
const int* MinresRun<T>::shift_steps() const {
  return carve_state(state, m0, ns).siters;
}

template struct MinresRun<float>;
template struct MinresRun<double>;

}  // namespace ifeast
