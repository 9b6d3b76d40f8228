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

#include <cstdio>
#include <cstdlib>

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
// non-temporal 16-byte stores (results that are not read again by this kernel)
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef double nd2 __attribute__((ext_vector_type(2)));
__device__ inline void nt_store(const float4& v, float4* p) {
  const nf4 t = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(t, reinterpret_cast<nf4*>(p));
}
__device__ inline void nt_store(const double2& v, double2* p) {
  const nd2 t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<nd2*>(p));
}
template <class V> __device__ inline V vzero();
template <> __device__ inline float4 vzero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <> __device__ inline double2 vzero<double2>() { return make_double2(0.0, 0.0); }

// acc[u] += sum over the CSR entries [e0, e1) of val[e] * V[col[e]] at vector column vb + 64u.
// KC entries are fetched per round (row indices and values are wave-uniform scalar loads), then
// U x KC independent 16-byte loads are issued before any of them is used: a 7-point row is one
// round of KC = 8.  Entries past e1 repeat the last column with value 0 so every load stays in bounds.
template <class T, class V16, int U, int KC>
__device__ inline void row_gather(int e0, int e1, const int* __restrict__ ci, const T* __restrict__ va,
                                  const V16* __restrict__ Vv, int nvec, int vb, const bool (&on)[U], V16 (&acc)[U]) {
  for (int e = e0; e < e1; e += KC) {
    int c[KC];
    T a[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int ek = e + k < e1 ? e + k : e1 - 1;
      c[k] = ci[ek];
      a[k] = e + k < e1 ? va[ek] : T(0);
    }
    V16 x[U][KC];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < KC; ++k) x[u][k] = on[u] ? Vv[(int64_t)c[k] * nvec + vb + 64 * u] : vzero<V16>();
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < KC; ++k) axpy(a[k], x[u][k], acc[u]);
  }
}

// One wavefront per row; lane l handles the 16-byte vectors vb + 64u (u < U) of the row, looping
// over the row in strides of 64 U vectors.
template <class T, bool HAS_B, int U, int KC>
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
  const int nvec = ns * m0 / C;  // 16-byte vectors per row
  const V16* __restrict__ Vv = reinterpret_cast<const V16*>(V);
  V16* __restrict__ Wv = reinterpret_cast<V16*>(W);
  const int e0 = rp[row], e1 = rp[row + 1];
  for (int vb = lane; vb < nvec; vb += 64 * U) {
    bool on[U];
    int sh[U];
    V16 acc[U], self[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int vc = vb + 64 * u;
      sh[u] = vc < nvec ? (vc * C) / m0 : 0;
      on[u] = vc < nvec && (active == nullptr || active[sh[u]] != 0);
      acc[u] = vzero<V16>();
      self[u] = vzero<V16>();
    }
    row_gather<T, V16, U, KC>(e0, e1, ci, va, Vv, nvec, vb, on, acc);
    if (HAS_B) {
      row_gather<T, V16, U, KC>(brp[row], brp[row + 1], bci, bva, Vv, nvec, vb, on, self);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (on[u]) self[u] = Vv[(int64_t)row * nvec + vb + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (on[u])
        Wv[(int64_t)row * nvec + vb + 64 * u] = zs_minus(zs[2 * sh[u]], zs[2 * sh[u] + 1], self[u], acc[u]);
  }
}

// Column-sliced variant.  The block is cut into slices of LPR 16-byte vectors
// (32 complex FP32 numbers for LPR = 16); a group of LPR lanes handles one row of
// one slice and a wavefront 64 / LPR rows.  XCD x owns the rows [x R, (x+1) R) and
// sweeps them slice after slice, so the rows a stencil reads far from the
// diagonal (the neighbour planes of a 3-D grid) were fetched by the same XCD a
// few thousand rows earlier in the same slice and are still in its L2: the reuse
// distance in bytes shrinks by the number of slices.  Each group fetches KC CSR
// entries of its row with one coalesced load and broadcasts them with lane
// shuffles; W is stored with non-temporal stores so it does not evict V from L2.
template <class T, bool HAS_B, int LPR, int KC>
__device__ inline void slab_gather(int e0, int e1, int g, const int* __restrict__ ci, const T* __restrict__ va,
                                   const typename Vec16<T>::type* __restrict__ Vv, int nvec, int vc,
                                   typename Vec16<T>::type& acc) {
  static_assert(KC <= LPR, "one load per group fetches the round's entries");
  for (int e = e0; e < e1; e += KC) {
    const int my = e + g;
    const bool have = g < KC && my < e1;
    const int cl = have ? ci[my] : 0;
    const T al = have ? va[my] : T(0);
    int c[KC];
    T a[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      c[k] = __shfl(cl, k, LPR);
      a[k] = __shfl(al, k, LPR);
    }
    typename Vec16<T>::type x[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) x[k] = Vv[(int64_t)c[k] * nvec + vc];  // c = 0, a = 0 past the row's end
#pragma unroll
    for (int k = 0; k < KC; ++k) axpy(a[k], x[k], acc);
  }
}

template <class T, bool HAS_B, int LPR, int KC>
__global__ __launch_bounds__(256) void k_spmm_slab(int n, int rows_xcd, int rbx, int nslices,
                                                   const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const T* __restrict__ va, const int* __restrict__ brp,
                                                   const int* __restrict__ bci, const T* __restrict__ bva, int ns,
                                                   int m0, const T* __restrict__ zs, const int* __restrict__ active,
                                                   const T* __restrict__ V, T* __restrict__ W) {
  using V16 = typename Vec16<T>::type;
  constexpr int C = Vec16<T>::C;
  constexpr int RPW = 64 / LPR;  // rows per wavefront
  constexpr int RPB = 4 * RPW;   // rows per workgroup
  const int xcd = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
  const int slice = i / rbx, rb = i % rbx;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane % LPR;
  const int rlo = xcd * rows_xcd;
  const int rhi = min(n, rlo + rows_xcd);
  const int row = rlo + rb * RPB + wave * RPW + lane / LPR;
  const int nvec = ns * m0 / C;
  const int vc = slice * LPR + g;
  // whole groups leave together (the shuffles stay inside a group)
  if (slice >= nslices || row >= rhi) return;
  const bool live = vc < nvec;
  const int vcc = live ? vc : nvec - 1;  // lanes past the block width load a valid vector and store nothing
  const int s = (vcc * C) / m0;
  const V16* __restrict__ Vv = reinterpret_cast<const V16*>(V);
  V16 acc = vzero<V16>(), self = vzero<V16>();
  slab_gather<T, HAS_B, LPR, KC>(rp[row], rp[row + 1], g, ci, va, Vv, nvec, vcc, acc);
  if (HAS_B)
    slab_gather<T, HAS_B, LPR, KC>(brp[row], brp[row + 1], g, bci, bva, Vv, nvec, vcc, self);
  else
    self = Vv[(int64_t)row * nvec + vcc];
  if (live && (active == nullptr || active[s] != 0))
    nt_store(zs_minus(zs[2 * s], zs[2 * s + 1], self, acc), reinterpret_cast<V16*>(W) + (int64_t)row * nvec + vc);
}

// Whole rows for narrow blocks: a row of nvec <= 64 vectors is one group of nvec lanes and
// a wavefront takes floor(64 / nvec) consecutive rows (3 rows of 20 vectors for a real
// 80-column FP32 block), so every row is one contiguous run and few lanes idle.  Rows are
// placed per XCD as in k_spmm_slab; CSR entries are fetched by the group's first KC lanes
// and broadcast with lane shuffles.
template <class T, bool HAS_B, int KC>
__device__ inline void group_gather(int e0, int e1, int g0, int li, const int* __restrict__ ci,
                                    const T* __restrict__ va, const typename Vec16<T>::type* __restrict__ Vv,
                                    int nvec, int vc, typename Vec16<T>::type& acc) {
  for (int e = e0; e < e1; e += KC) {
    const int my = e + li;
    const bool have = li < KC && my < e1;
    const int cl = have ? ci[my] : 0;
    const T al = have ? va[my] : T(0);
    int c[KC];
    T a[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      c[k] = __shfl(cl, g0 + k);
      a[k] = __shfl(al, g0 + k);
    }
    typename Vec16<T>::type x[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) x[k] = Vv[(int64_t)c[k] * nvec + vc];
#pragma unroll
    for (int k = 0; k < KC; ++k) axpy(a[k], x[k], acc);
  }
}

// The same gather with every lane of the group loading the round's CSR entries itself (the
// group's lanes read one address, which the memory pipeline serves once) instead of shuffles.
template <class T, int KC>
__device__ inline void group_gather_direct(int e0, int e1, const int* __restrict__ ci, const T* __restrict__ va,
                                           const typename Vec16<T>::type* __restrict__ Vv, int nvec, int vc,
                                           typename Vec16<T>::type& acc) {
  for (int e = e0; e < e1; e += KC) {
    int c[KC];
    T a[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const bool have = e + k < e1;
      c[k] = ci[have ? e + k : e1 - 1];
      a[k] = have ? va[e + k] : T(0);
    }
    typename Vec16<T>::type x[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) x[k] = Vv[(int64_t)c[k] * nvec + vc];
#pragma unroll
    for (int k = 0; k < KC; ++k) axpy(a[k], x[k], acc);
  }
}

template <class T, bool HAS_B, int KC, bool DIRECT>
__global__ __launch_bounds__(256) void k_spmm_rows(int n, int rows_xcd, int rbx, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const T* __restrict__ va,
                                                   const int* __restrict__ brp, const int* __restrict__ bci,
                                                   const T* __restrict__ bva, int ns, int m0,
                                                   const T* __restrict__ zs, const int* __restrict__ active,
                                                   const T* __restrict__ V, T* __restrict__ W) {
  using V16 = typename Vec16<T>::type;
  constexpr int C = Vec16<T>::C;
  const int nvec = ns * m0 / C;
  const int gpw = 64 / nvec;  // row groups per wavefront
  const int xcd = blockIdx.x % kXcds, rb = blockIdx.x / kXcds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = lane / nvec, li = lane % nvec, g0 = grp * nvec;
  const int rlo = xcd * rows_xcd;
  const int rhi = min(n, rlo + rows_xcd);
  const int row = rlo + (rb * 4 + wave) * gpw + grp;
  // lanes past the last group, or groups past the XCD's rows, have nothing to do (each group
  // shuffles only within itself)
  if (grp >= gpw || row >= rhi) return;
  const int s = (li * C) / m0;
  const V16* __restrict__ Vv = reinterpret_cast<const V16*>(V);
  V16 acc = vzero<V16>(), self = vzero<V16>();
  if (DIRECT)
    group_gather_direct<T, KC>(rp[row], rp[row + 1], ci, va, Vv, nvec, li, acc);
  else
    group_gather<T, HAS_B, KC>(rp[row], rp[row + 1], g0, li, ci, va, Vv, nvec, li, acc);
  const bool shifted = zs[2 * s] != T(0) || zs[2 * s + 1] != T(0);
  if (HAS_B) {
    if (DIRECT)
      group_gather_direct<T, KC>(brp[row], brp[row + 1], bci, bva, Vv, nvec, li, self);
    else
      group_gather<T, HAS_B, KC>(brp[row], brp[row + 1], g0, li, bci, bva, Vv, nvec, li, self);
  } else if (shifted) {
    self = Vv[(int64_t)row * nvec + li];  // a zero shift (W = -A V) needs no self term
  }
  if (active == nullptr || active[s] != 0)
    nt_store(zs_minus(zs[2 * s], zs[2 * s + 1], self, acc), reinterpret_cast<V16*>(W) + (int64_t)row * nvec + li);
}

// Whole rows as in k_spmm_rows (B = I only), each wavefront taking G consecutive sets of
// floor(64 / nvec) rows and software-pipelining them: the row pointers of all G sets are loaded
// first, and the CSR entries of set s + 1 are loaded before the gathers of set s, so a set waits
// for one memory round trip (its gathers) instead of three (row pointers, entries, gathers).
// Rows with more than KC entries take their further rounds unpipelined.
template <class T, int KC, int G>
__global__ __launch_bounds__(256) void k_spmm_rows_pipe(int n, int rows_xcd, int rbx, const int* __restrict__ rp,
                                                        const int* __restrict__ ci, const T* __restrict__ va,
                                                        int ns, int m0, const T* __restrict__ zs,
                                                        const int* __restrict__ active, const T* __restrict__ V,
                                                        T* __restrict__ W) {
  using V16 = typename Vec16<T>::type;
  constexpr int C = Vec16<T>::C;
  const int nvec = ns * m0 / C;
  const int gpw = 64 / nvec;  // row groups per set
  const int xcd = blockIdx.x % kXcds, rb = blockIdx.x / kXcds;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = lane / nvec, li = lane % nvec, g0 = grp * nvec;
  const int rlo = xcd * rows_xcd;
  const int rhi = min(n, rlo + rows_xcd);
  const int row0 = rlo + (rb * 4 + wave) * G * gpw + grp;  // set s: row0 + s gpw
  if (grp >= gpw || row0 >= rhi) return;  // whole groups leave together
  // every lane of a group takes part in the group's shuffles; a stopped shift only skips its stores
  const int s_ = (li * C) / m0;
  const bool live = active == nullptr || active[s_] != 0;
  const bool shifted = zs[2 * s_] != T(0) || zs[2 * s_ + 1] != T(0);
  const V16* __restrict__ Vv = reinterpret_cast<const V16*>(V);
  int e0[G], e1[G];
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int row = row0 + q * gpw;
    e0[q] = row < rhi ? rp[row] : 0;
    e1[q] = row < rhi ? rp[row + 1] : 0;
  }
  int cl = 0;
  T al = T(0);
  auto entries = [&](int q, int& c, T& a) {
    const int my = e0[q] + li;
    const bool have = li < KC && my < e1[q];
    c = have ? ci[my] : 0;
    a = have ? va[my] : T(0);
  };
  entries(0, cl, al);
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int row = row0 + q * gpw;
    int cn = 0;
    T an = T(0);
    if (q + 1 < G) entries(q + 1, cn, an);
    if (row < rhi) {
      V16 acc = vzero<V16>();
      int c[KC];
      T a[KC];
#pragma unroll
      for (int k = 0; k < KC; ++k) {
        c[k] = __shfl(cl, g0 + k);
        a[k] = __shfl(al, g0 + k);
      }
      V16 x[KC];
#pragma unroll
      for (int k = 0; k < KC; ++k) x[k] = Vv[(int64_t)c[k] * nvec + li];
#pragma unroll
      for (int k = 0; k < KC; ++k) axpy(a[k], x[k], acc);
      if (e1[q] - e0[q] > KC)
        group_gather<T, false, KC>(e0[q] + KC, e1[q], g0, li, ci, va, Vv, nvec, li, acc);
      V16 self = vzero<V16>();
      if (shifted) self = Vv[(int64_t)row * nvec + li];
      if (live)
        nt_store(zs_minus(zs[2 * s_], zs[2 * s_ + 1], self, acc), reinterpret_cast<V16*>(W) + (int64_t)row * nvec + li);
    }
    cl = cn;
    al = an;
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

// Schedules the autotuner chooses from: whole rows per wavefront with U vectors per lane per
// pass, or column slices of LPR vectors; KC = CSR entries fetched per round.
struct Sched {
  bool slab;
  int U_or_LPR, KC;
  const char* name;
};
constexpr Sched kSched[] = {{false, 1, 8, "row-U1-K8"}, {false, 2, 4, "row-U2-K4"}, {false, 3, 4, "row-U3-K4"},
                            {true, 8, 8, "slab8-K8"},   {true, 16, 8, "slab16-K8"}, {true, 32, 8, "slab32-K8"},
                            {true, 16, 16, "slab16-K16"}, {true, 8, 4, "slab8-K4"},  {true, 0, 8, "rows-K8"},
                            {true, 0, 7, "rows-K7"},    {true, 0, 7, "rows-K7-direct"}, {true, 0, 4, "rows-K4-direct"},
                            {true, 0, 7, "rows-K7-pipe2"}, {true, 0, 7, "rows-K7-pipe4"}, {true, 0, 8, "rows-K8-pipe4"}};
constexpr int kNSched = sizeof(kSched) / sizeof(kSched[0]);

struct SpmmOperands {
  int n, ns, m0;
  const int *rp, *ci;
  const void* va;
  const int *brp, *bci;
  const void* bva;
  const void* zs;
  const int* active;
  const void* V;
  void* W;
};

template <class T, bool HAS_B, int U, int KC>
void launch_row(hipStream_t st, const SpmmOperands& o) {
  const int64_t nblk = (o.n + 3) / 4;
  const int per = xcd_per(nblk);
  hipLaunchKernelGGL((k_spmm_shifted<T, HAS_B, U, KC>), dim3(per * kXcds), dim3(256), 0, st, o.n, per, o.rp, o.ci,
                     (const T*)o.va, o.brp, o.bci, (const T*)o.bva, o.ns, o.m0, (const T*)o.zs, o.active,
                     (const T*)o.V, (T*)o.W);
}

template <class T, bool HAS_B, int LPR, int KC>
void launch_slab(hipStream_t st, const SpmmOperands& o) {
  constexpr int C = Vec16<T>::C;
  constexpr int RPB = 4 * (64 / LPR);
  const int nvec = o.ns * o.m0 / C;
  const int nslices = (nvec + LPR - 1) / LPR;
  const int rows_xcd = (o.n + kXcds - 1) / kXcds;
  const int rbx = (rows_xcd + RPB - 1) / RPB;
  const int64_t blocks = (int64_t)kXcds * nslices * rbx;
  IF_REQUIRE(blocks < (int64_t(1) << 31), "SpMM grid too large");
  hipLaunchKernelGGL((k_spmm_slab<T, HAS_B, LPR, KC>), dim3((unsigned)blocks), dim3(256), 0, st, o.n, rows_xcd, rbx,
                     nslices, o.rp, o.ci, (const T*)o.va, o.brp, o.bci, (const T*)o.bva, o.ns, o.m0,
                     (const T*)o.zs, o.active, (const T*)o.V, (T*)o.W);
}

template <class T, bool HAS_B, int KC, bool DIRECT>
void launch_rows(hipStream_t st, const SpmmOperands& o) {
  constexpr int C = Vec16<T>::C;
  const int nvec = o.ns * o.m0 / C;
  IF_REQUIRE(nvec >= KC && nvec <= 64, "SpMM rows schedule needs a block of 8..64 vectors per row");
  const int rpb = 4 * (64 / nvec);  // rows per workgroup
  const int rows_xcd = (o.n + kXcds - 1) / kXcds;
  const int rbx = (rows_xcd + rpb - 1) / rpb;
  hipLaunchKernelGGL((k_spmm_rows<T, HAS_B, KC, DIRECT>), dim3((unsigned)((int64_t)kXcds * rbx)), dim3(256), 0, st, o.n,
                     rows_xcd, rbx, o.rp, o.ci, (const T*)o.va, o.brp, o.bci, (const T*)o.bva, o.ns, o.m0,
                     (const T*)o.zs, o.active, (const T*)o.V, (T*)o.W);
}

template <class T, int KC, int G>
void launch_rows_pipe(hipStream_t st, const SpmmOperands& o) {
  constexpr int C = Vec16<T>::C;
  const int nvec = o.ns * o.m0 / C;
  IF_REQUIRE(nvec >= KC && nvec <= 64 && o.brp == nullptr, "SpMM pipelined rows schedule: 8..64 vectors per row, B = I");
  const int rpb = 4 * G * (64 / nvec);  // rows per workgroup
  const int rows_xcd = (o.n + kXcds - 1) / kXcds;
  const int rbx = (rows_xcd + rpb - 1) / rpb;
  hipLaunchKernelGGL((k_spmm_rows_pipe<T, KC, G>), dim3((unsigned)((int64_t)kXcds * rbx)), dim3(256), 0, st, o.n,
                     rows_xcd, rbx, o.rp, o.ci, (const T*)o.va, o.ns, o.m0, (const T*)o.zs, o.active, (const T*)o.V,
                     (T*)o.W);
}

// whether schedule idx can run a block of nvec 16-byte vectors per row (with B: has_b)
bool sched_fits(int idx, int nvec, bool has_b) {
  if (idx < 8) return true;
  if (idx >= 12 && has_b) return false;
  return nvec >= 8 && nvec <= 64;
}

template <class T, bool HAS_B>
void launch_sched(int idx, hipStream_t st, const SpmmOperands& o) {
  switch (idx) {
    case 0: launch_row<T, HAS_B, 1, 8>(st, o); break;
    case 1: launch_row<T, HAS_B, 2, 4>(st, o); break;
    case 2: launch_row<T, HAS_B, 3, 4>(st, o); break;
    case 3: launch_slab<T, HAS_B, 8, 8>(st, o); break;
    case 4: launch_slab<T, HAS_B, 16, 8>(st, o); break;
    case 5: launch_slab<T, HAS_B, 32, 8>(st, o); break;
    case 6: launch_slab<T, HAS_B, 16, 16>(st, o); break;
    case 7: launch_slab<T, HAS_B, 8, 4>(st, o); break;
    case 8: launch_rows<T, HAS_B, 8, false>(st, o); break;
    case 9: launch_rows<T, HAS_B, 7, false>(st, o); break;
    case 10: launch_rows<T, HAS_B, 7, true>(st, o); break;
    case 11: launch_rows<T, HAS_B, 4, true>(st, o); break;
    case 12: launch_rows_pipe<T, 7, 2>(st, o); break;
    case 13: launch_rows_pipe<T, 7, 4>(st, o); break;
    case 14: launch_rows_pipe<T, 8, 4>(st, o); break;
    default: throw Error{IFEAST_ERR_INVALID_ARG, "unknown SpMM schedule"};
  }
}

}  // namespace

const char* spmm_schedule_name(int idx) { return idx >= 0 && idx < kNSched ? kSched[idx].name : "?"; }

template <class T>
void launch_spmm_shifted(hipStream_t st, const ifeast_matrix* A, const ifeast_matrix* B, int ns, int m0,
                         const T* zs, const int* active, const T* V, T* W) {
  const int64_t n = A->n;
  SpmmOperands o;
  o.n = (int)n;
  o.ns = ns;
  o.m0 = m0;
  o.rp = A->rowptr.as<int>();
  o.ci = A->colind.as<int>();
  o.va = (sizeof(T) == 4) ? A->valf.p : A->val.p;
  o.brp = B ? B->rowptr.as<int>() : nullptr;
  o.bci = B ? B->colind.as<int>() : nullptr;
  o.bva = B ? ((sizeof(T) == 4) ? B->valf.p : B->val.p) : nullptr;
  o.zs = zs;
  o.active = active;
  o.V = V;
  o.W = W;
  auto run = [&](int idx) {
    if (B == nullptr)
      launch_sched<T, false>(idx, st, o);
    else
      launch_sched<T, true>(idx, st, o);
    IF_HIP(hipGetLastError());
  };
  // Autotuner: the first product of a given (matrix, B, width, precision) times every schedule on the
  // caller's stream (each launch computes the same W) and keeps the fastest for this matrix.
  const SpmmKey key{ns * m0, (int)sizeof(T), B != nullptr};
  int idx = -1;
  {
    std::lock_guard<std::mutex> lk(A->tune_mu);
    auto it = A->sched.find(key);
    if (it != A->sched.end()) idx = it->second;
  }
  if (idx < 0) {
    const char* forced = getenv("IFEAST_SPMM_SCHED");
    if (forced != nullptr) {
      idx = atoi(forced);
      IF_REQUIRE(idx >= 0 && idx < kNSched, "IFEAST_SPMM_SCHED out of range");
    } else {
      hipEvent_t e0, e1;
      IF_HIP(hipEventCreate(&e0));
      IF_HIP(hipEventCreate(&e1));
      float best = 1e30f;
      std::vector<float> times(kNSched, 0.f);
      const int nvec = ns * m0 / (sizeof(T) == 4 ? 2 : 1);
      for (int c = 0; c < kNSched; ++c) {
        if (!sched_fits(c, nvec, B != nullptr)) {
          times[c] = 0.f;
          continue;
        }
        run(c);  // warm
        IF_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r) run(c);
        IF_HIP(hipEventRecord(e1, st));
        IF_HIP(hipEventSynchronize(e1));
        IF_HIP(hipEventElapsedTime(&times[c], e0, e1));
        if (times[c] < best) {
          best = times[c];
          idx = c;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (getenv("IFEAST_VERBOSE") != nullptr) {
        fprintf(stderr, "[ifeast] spmm autotune n=%lld width=%d %s:", (long long)n, ns * m0,
                sizeof(T) == 4 ? "c32" : "c64");
        for (int c = 0; c < kNSched; ++c) fprintf(stderr, " %s=%.1fus", spmm_schedule_name(c), times[c] * 1e3f / 3);
        fprintf(stderr, " -> %s\n", spmm_schedule_name(idx));
      }
    }
    std::lock_guard<std::mutex> lk(A->tune_mu);
    A->sched[key] = idx;
  }
  KernelTimer* kt = current_timer();
  const int tok = kt ? kt->begin(st) : -1;
  run(idx);
  if (kt) {
    // algorithmic bytes: the CSR of A (and B) once, V read once and W written once for active shifts
    const int nact = kt->count(active, ns);
    const double csr = (double)(n + 1) * 4 + (double)A->nnz * (4 + sizeof(T)) +
                       (B ? (double)(n + 1) * 4 + (double)B->nnz * (4 + sizeof(T)) : 0.0);
    const double vw = 2.0 * (double)n * nact * m0 * 2 * sizeof(T);
    const double fl = (double)nact * m0 * 8.0 * ((double)A->nnz + (B ? (double)B->nnz : (double)n)) +
                      6.0 * (double)n * nact * m0;
    kt->end(tok, KC_SPMM, fl, csr + vw);
  }
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
