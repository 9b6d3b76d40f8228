// Sparse matrix x tall block products.
//
// The shifted product is the only access IFEAST makes to A and B
// (Algorithm 2, step 1): every GMRES step of every shifted system needs
// W_s = z_s B V_s - A V_s.  All nc systems are handled in one launch on the
// concatenated block V = [V_0 .. V_{nc-1}] (n x nc*m0 complex, row-major), so
// each CSR row of A (and B) is read once per step for all shifts, and each
// row of V is one contiguous run of nc*m0 complex numbers: a wavefront
// streams it with 16-byte loads.
//
// One wavefront owns one matrix row; the 4 wavefronts of a workgroup own
// 4 consecutive rows.  Workgroups are renumbered so that each XCD (hardware
// places workgroup b on XCD b % 8) gets one contiguous range of rows: the
// stencil neighbours i +- 1 and i +- N of a row are then read by the same
// XCD and hit its L2.
#include "internal.h"

namespace ifeast {

namespace {

constexpr int kXcds = 8;

// Bijective XCD-aware renumbering of `nblk_pad` = 8 * per workgroups.
__device__ inline int xcd_block(int bid, int per) { return (bid % kXcds) * per + bid / kXcds; }

inline int xcd_per(int64_t nblk) { return (int)((nblk + kXcds - 1) / kXcds); }

template <class T> struct Vec16;
template <> struct Vec16<float> {
  using type = float4;  // two complex FP32 numbers
  static constexpr int C = 2;
};
template <> struct Vec16<double> {
  using type = double2;  // one complex FP64 number
  static constexpr int C = 1;
};

__device__ inline void axpy(float a, const float4& v, float4& acc) {
  acc.x += a * v.x; acc.y += a * v.y; acc.z += a * v.z; acc.w += a * v.w;
}
__device__ inline void axpy(double a, const double2& v, double2& acc) {
  acc.x += a * v.x; acc.y += a * v.y;
}
// out = z * s - acc for each complex number in the 16-byte vector
__device__ inline float4 zs_minus(float zr, float zi, const float4& s, const float4& acc) {
  return make_float4(zr * s.x - zi * s.y - acc.x, zr * s.y + zi * s.x - acc.y,
                     zr * s.z - zi * s.w - acc.z, zr * s.w + zi * s.z - acc.w);
}
__device__ inline double2 zs_minus(double zr, double zi, const double2& s, const double2& acc) {
  return make_double2(zr * s.x - zi * s.y - acc.x, zr * s.y + zi * s.x - acc.y);
}
template <class V> __device__ inline V vzero();
template <> __device__ inline float4 vzero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <> __device__ inline double2 vzero<double2>() { return make_double2(0.0, 0.0); }

template <class T, bool HAS_B>
__global__ __launch_bounds__(256) void k_spmm_shifted(int n, int per, const int* __restrict__ rp,
                                                      const int* __restrict__ ci, const T* __restrict__ va,
                                                      const int* __restrict__ brp, const int* __restrict__ bci,
                                                      const T* __restrict__ bva, int ns, int m0,
                                                      const T* __restrict__ zs, const int* __restrict__ active,
                                                      const T* __restrict__ V, T* __restrict__ W) {
  using V16 = typename Vec16<T>::type;
  constexpr int C = Vec16<T>::C;
  const int lb = xcd_block(blockIdx.x, per);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int row = lb * 4 + wave;
  if (row >= n) return;
  row = __builtin_amdgcn_readfirstlane(row);
  const int ldc = ns * m0;  // complex numbers per row
  const int nvec = ldc / C;  // 16-byte vectors per row
  const V16* __restrict__ Vv = reinterpret_cast<const V16*>(V);
  V16* __restrict__ Wv = reinterpret_cast<V16*>(W);
  const int e0 = rp[row], e1 = rp[row + 1];
  for (int vc = lane; vc < nvec; vc += 64) {
    const int s = (vc * C) / m0;
    if (active != nullptr && active[s] == 0) continue;
    V16 acc = vzero<V16>();
    for (int e = e0; e < e1; ++e) axpy(va[e], Vv[(int64_t)ci[e] * nvec + vc], acc);
    V16 self;
    if (HAS_B) {
      self = vzero<V16>();
      const int f0 = brp[row], f1 = brp[row + 1];
      for (int e = f0; e < f1; ++e) axpy(bva[e], Vv[(int64_t)bci[e] * nvec + vc], self);
    } else {
      self = Vv[(int64_t)row * nvec + vc];
    }
    Wv[(int64_t)row * nvec + vc] = zs_minus(zs[2 * s], zs[2 * s + 1], self, acc);
  }
}

__global__ __launch_bounds__(256) void k_spmm_real(int n, int per, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const double* __restrict__ va, int m,
                                                   const double* __restrict__ X, double* __restrict__ Y) {
  const int lb = xcd_block(blockIdx.x, per);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int row = lb * 4 + wave;
  if (row >= n) return;
  row = __builtin_amdgcn_readfirstlane(row);
  const int nvec = m / 2;  // m is even
  const double2* __restrict__ Xv = reinterpret_cast<const double2*>(X);
  double2* __restrict__ Yv = reinterpret_cast<double2*>(Y);
  const int e0 = rp[row], e1 = rp[row + 1];
  for (int vc = lane; vc < nvec; vc += 64) {
    double2 acc = make_double2(0.0, 0.0);
    for (int e = e0; e < e1; ++e) axpy(va[e], Xv[(int64_t)ci[e] * nvec + vc], acc);
    Yv[(int64_t)row * nvec + vc] = acc;
  }
}

}  // namespace

template <class T>
void launch_spmm_shifted(hipStream_t st, const ifeast_matrix* A, const ifeast_matrix* B, int ns, int m0,
                         const T* zs, const int* active, const T* V, T* W) {
  const int64_t n = A->n;
  const int64_t nblk = (n + 3) / 4;
  const int per = xcd_per(nblk);
  const dim3 grid(per * kXcds), block(256);
  const T* va = (sizeof(T) == 4) ? reinterpret_cast<const T*>(A->valf.p) : reinterpret_cast<const T*>(A->val.p);
  if (B == nullptr) {
    hipLaunchKernelGGL((k_spmm_shifted<T, false>), grid, block, 0, st, (int)n, per, A->rowptr.as<int>(),
                       A->colind.as<int>(), va, nullptr, nullptr, nullptr, ns, m0, zs, active, V, W);
  } else {
    const T* vb =
        (sizeof(T) == 4) ? reinterpret_cast<const T*>(B->valf.p) : reinterpret_cast<const T*>(B->val.p);
    hipLaunchKernelGGL((k_spmm_shifted<T, true>), grid, block, 0, st, (int)n, per, A->rowptr.as<int>(),
                       A->colind.as<int>(), va, B->rowptr.as<int>(), B->colind.as<int>(), vb, ns, m0, zs, active,
                       V, W);
  }
  IF_HIP(hipGetLastError());
}

template void launch_spmm_shifted<float>(hipStream_t, const ifeast_matrix*, const ifeast_matrix*, int, int,
                                         const float*, const int*, const float*, float*);
template void launch_spmm_shifted<double>(hipStream_t, const ifeast_matrix*, const ifeast_matrix*, int, int,
                                          const double*, const int*, const double*, double*);

void launch_spmm_real(hipStream_t st, const ifeast_matrix* M, int m, const double* X, double* Y) {
  const int64_t n = M->n;
  const int64_t nblk = (n + 3) / 4;
  const int per = xcd_per(nblk);
  hipLaunchKernelGGL(k_spmm_real, dim3(per * kXcds), dim3(256), 0, st, (int)n, per, M->rowptr.as<int>(),
                     M->colind.as<int>(), M->val.as<double>(), m, X, Y);
  IF_HIP(hipGetLastError());
}

}  // namespace ifeast
