// Tall-skinny dense products on MFMA (gfx950 v_mfma_f32_16x16x4_f32 and
// v_mfma_f64_16x16x4_f64).
//
// Block Arnoldi (Sec. 3.1) orthogonalises each new block against the basis
// with Gram products H = V^H W and updates W -= V H; the Cholesky-QR of a
// block, the quadrature sum Q = sum_k w_k V_k y_k, the restart residual and
// the Rayleigh-Ritz products X = Q C are the same shapes.  Complex blocks are
// handled through their real views: an n x m complex row-major block with
// interleaved (re, im) is an n x 2m real block, so V^H W is read off the real
// product V_r^T W_r (2m x 2m) and V H is V_r times the 2m x 2m real form of H.
// Every product is therefore a real GEMM with one long dimension n.
//
// MFMA fragment layout used below (16x16x4, 64 lanes, lane l), as measured
// on gfx950 with an in-bounds probe of both builtins:
//   A operand: A[i = l % 16][k = l / 16]
//   B operand: B[k = l / 16][j = l % 16]
//   D (4 values v), f32: D[i = 4 * (l / 16) + v][j = l % 16]
//   D (4 values v), f64: D[i = l / 16 + 4 * v][j = l % 16]
#include "internal.h"

namespace ifeast {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <class T> struct Mfma;
template <> struct Mfma<float> {
  using acc = v4f;
  __device__ static inline acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  __device__ static inline acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int v) { return 4 * lk + v; }
};
template <> struct Mfma<double> {
  using acc = v4d;
  __device__ static inline acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int v) { return lk + 4 * v; }
};

constexpr int kXcds = 8;
__device__ inline int xcd_block(int bid, int per) { return (bid % kXcds) * per + bid / kXcds; }

// 16-byte vector of T for global loads
template <class T> struct V16T;
template <> struct V16T<float> { using t = float4; static constexpr int N = 4; };
template <> struct V16T<double> { using t = double2; static constexpr int N = 2; };
template <class T> __device__ inline void put16(T* dst, const typename V16T<T>::t& v);
template <> __device__ inline void put16<float>(float* d, const float4& v) { d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w; }
template <> __device__ inline void put16<double>(double* d, const double2& v) { d[0] = v.x; d[1] = v.y; }
template <class T> __device__ inline typename V16T<T>::t zero16();
template <> __device__ inline float4 zero16<float>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <> __device__ inline double2 zero16<double>() { return make_double2(0.0, 0.0); }

// LDS row stride: b32 fragment reads of 4 consecutive rows hit disjoint bank halves
template <class T> constexpr int lds_ld(int w) { return sizeof(T) == 4 ? w + ((16 - w % 32) + 32) % 32 : w; }

// ------------------------------------------------------------------ Gram
// G[item] = A_item^T B_item over a row split.  grid: x = row split,
// y = output tile, z = item.  The tile is (TB*16) x (TB*16); the 4 waves
// form a 2 x 2 grid, each owning H x H MFMA blocks (H = ceil(TB/2)).
template <class T> struct GramCfg { static constexpr int KC = 32; };
template <> struct GramCfg<double> { static constexpr int KC = 16; };

template <class T, int TB>
__global__ __launch_bounds__(256) void k_gram(GramArgs g, int nsplit, int64_t rows_per_split, int ntq,
                                              T* __restrict__ partial) {
  using V = typename V16T<T>::t;
  constexpr int VN = V16T<T>::N;
  constexpr int KC = GramCfg<T>::KC;
  constexpr int TP = TB * 16;
  constexpr int LD = lds_ld<T>(TP);
  constexpr int H = (TB + 1) / 2;
  constexpr int NV = KC * TP / VN;             // 16-byte vectors per operand tile
  constexpr int PER = (NV + 255) / 256;        // per thread
  __shared__ T sA[KC * LD];
  __shared__ T sB[KC * LD];

  const int item = blockIdx.z;
  const int s = item / g.ni, i = item % g.ni;
  if (g.active != nullptr && g.active[s] == 0) return;
  const int split = blockIdx.x;
  const int tp = blockIdx.y / ntq, tq = blockIdx.y % ntq;
  const int p0 = tp * TP, q0 = tq * TP;
  const int vp = min(TP, g.PW - p0), vq = min(TP, g.QW - q0);
  const int64_t r0 = (int64_t)split * rows_per_split;
  const int64_t r1 = min(g.n, r0 + rows_per_split);
  if (r0 >= r1) {
    // an empty split still owns its slot of partial sums
  }
  const T* __restrict__ A = (g.A_last != nullptr && i == g.ni - 1 ? static_cast<const T*>(g.A_last) + s * g.a_s
                                                                    : static_cast<const T*>(g.A) + s * g.a_s + i * g.a_i) +
                            p0;
  const T* __restrict__ B = static_cast<const T*>(g.B) + s * g.b_s + i * g.b_i + q0;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int wp = wave >> 1, wq = wave & 1;
  typename Mfma<T>::acc acc[H][H];
#pragma unroll
  for (int a = 0; a < H; ++a)
#pragma unroll
    for (int b = 0; b < H; ++b) acc[a][b] = Mfma<T>::zero();

  V ra[PER], rb[PER];
  auto fetch = [&](int64_t rc) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int v = tid + 256 * t;
      ra[t] = zero16<T>();
      rb[t] = zero16<T>();
      if (v < NV) {
        const int r = v / (TP / VN), c = (v % (TP / VN)) * VN;
        const int64_t row = rc + r;
        if (row < r1) {
          if (c < vp) ra[t] = *reinterpret_cast<const V*>(A + row * g.lda + c);
          if (c < vq) rb[t] = *reinterpret_cast<const V*>(B + row * g.ldb + c);
        }
      }
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t rc = r0; rc < r1; rc += KC) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int v = tid + 256 * t;
      if (v < NV) {
        const int r = v / (TP / VN), c = (v % (TP / VN)) * VN;
        put16<T>(sA + r * LD + c, ra[t]);
        put16<T>(sB + r * LD + c, rb[t]);
      }
    }
    __syncthreads();
    if (rc + KC < r1) fetch(rc + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T af[H], bf[H];
#pragma unroll
      for (int a = 0; a < H; ++a) af[a] = sA[(kk + lk) * LD + (wp * H + a) * 16 + li];
#pragma unroll
      for (int b = 0; b < H; ++b) bf[b] = sB[(kk + lk) * LD + (wq * H + b) * 16 + li];
#pragma unroll
      for (int a = 0; a < H; ++a)
#pragma unroll
        for (int b = 0; b < H; ++b)
          if ((wp * H + a) < TB && (wq * H + b) < TB) acc[a][b] = Mfma<T>::mma(af[a], bf[b], acc[a][b]);
    }
    __syncthreads();
  }

  T* out = partial + ((int64_t)item * nsplit + split) * g.PW * g.QW;
#pragma unroll
  for (int a = 0; a < H; ++a)
#pragma unroll
    for (int b = 0; b < H; ++b) {
      const int pb = wp * H + a, qb = wq * H + b;
      if (pb < TB && qb < TB && pb * 16 < vp && qb * 16 < vq) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int p = p0 + pb * 16 + Mfma<T>::row(lk, v);
          const int q = q0 + qb * 16 + li;
          out[(int64_t)p * g.QW + q] = acc[a][b][v];
        }
      }
    }
}

// Waves per workgroup of the split-K reduction.  The output is small (a few hundred workgroups of
// 64 elements), so the loads in flight per CU set its speed: sixteen waves striding the splits
// keep four times as many in flight as four did.
constexpr int kRedWaves = 16;

template <class T>
__global__ __launch_bounds__(64 * kRedWaves) void k_gram_reduce(int items, int nsplit, int PW, int QW, int ni,
                                                               const int* __restrict__ active,
                                                               const T* __restrict__ partial, double* __restrict__ G,
                                                               GramCombine cmb) {
  // 64 consecutive output elements per workgroup, one per lane, so every load of a wave reads 64
  // consecutive partial sums; wave w takes every kRedWaves-th split from w, and the waves' sums
  // are added in wave order (a fixed order: results are reproducible)
  __shared__ double red[kRedWaves][64];
  const int64_t per_item = (int64_t)PW * QW;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
  const bool live = idx < per_item * items;
  const int item = live ? (int)(idx / per_item) : 0;
  const bool on = live && !(active != nullptr && active[item / ni] == 0);
  double sum = 0.0;
  if (on) {
    const T* p = partial + (int64_t)item * nsplit * per_item + idx % per_item;
    // unrolled so that eight loads are in flight before the (in-order) additions
#pragma unroll 8
    for (int sp = wave; sp < nsplit; sp += kRedWaves) sum += (double)p[(int64_t)sp * per_item];
  }
  red[wave][lane] = sum;
  __syncthreads();
  if (wave != 0 || !on) return;
  sum = red[0][lane];
#pragma unroll
  for (int w = 1; w < kRedWaves; ++w) sum += red[w][lane];
  G[idx] = sum;
  if (cmb.Hm != nullptr) {
    // block column j of Hm (block rows i0 + item) and the update factors, as k_combine_real
    const int a = (int)((idx % per_item) / QW), b = (int)(idx % QW);
    double* h = cmb.Hm + (int64_t)(cmb.j * QW + b) * cmb.ldh + (int64_t)(cmb.i0 + item) * PW + a;
    *h = cmb.accumulate ? *h + sum : sum;
    static_cast<T*>(cmb.Hr)[idx] = (T)sum;
  }
}

// Gram of several blocks of a shift against the same right operand:
//   G[s, i] = A_{s,i}^T B_s,  i = 4 y .. 4 y + 3,  each (16 TB) x (16 TB).
// Wave w owns block i = 4 y + w and all TB x TB of its MFMA tiles; the B tile is staged once
// for the four waves, so B is read once per four blocks instead of once per block.  A group of
// two blocks gives each block 2 waves, splitting its 16-row tile blocks.
// grid: x = row split, y = group of four blocks, z = shift.
template <class T, int TB, int KC>
__global__ __launch_bounds__(256, 2) void k_gram4(GramArgs g, int nsplit, int64_t rows_per_split, T* __restrict__ partial) {
  using V = typename V16T<T>::t;
  constexpr int VN = V16T<T>::N;
  constexpr int TP = TB * 16;
  constexpr int LD = lds_ld<T>(TP);
  constexpr int NV = KC * TP / VN;             // 16-byte vectors per operand tile
  constexpr int PER = (NV + 255) / 256;
  __shared__ T sA[4][KC * LD];
  __shared__ T sB[KC * LD];
  const int s = blockIdx.z;
  if (g.active != nullptr && g.active[s] == 0) return;
  const int i0 = blockIdx.y * 4;
  const int nil = min(4, g.ni - i0);  // blocks in this group
  const int split = blockIdx.x;
  const int64_t r0 = (int64_t)split * rows_per_split;
  const int64_t r1 = min(g.n, r0 + rows_per_split);
  const T* __restrict__ A0 = static_cast<const T*>(g.A) + s * g.a_s + i0 * g.a_i;
  const T* __restrict__ B = static_cast<const T*>(g.B) + s * g.b_s;
  const T* Aq[4];  // the group's blocks (the shift's last one possibly from A_last)
#pragma unroll
  for (int q = 0; q < 4; ++q)
    Aq[q] = (g.A_last != nullptr && i0 + q == g.ni - 1) ? static_cast<const T*>(g.A_last) + s * g.a_s : A0 + q * g.a_i;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  // waves per block: with fewer than four blocks in the group, several waves share a block,
  // each taking a range [ra0, ra1) of its 16-row tile blocks
  const int wpb = nil >= 3 ? 1 : 4 / nil;
  const int q = wave / wpb, part = wave % wpb;
  const int ra0 = part * TB / wpb, ra1 = (part + 1) * TB / wpb;
  typename Mfma<T>::acc acc[TB][TB];
#pragma unroll
  for (int a = 0; a < TB; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) acc[a][b] = Mfma<T>::zero();
  V ra[4][PER], rb[PER];
  auto fetch = [&](int64_t rc) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int v = tid + 256 * t;
      const int r = v / (TP / VN), c = (v % (TP / VN)) * VN;
      const int64_t row = rc + r;
      const bool ok = v < NV && row < r1;
      rb[t] = ok ? *reinterpret_cast<const V*>(B + row * g.ldb + c) : zero16<T>();
#pragma unroll
      for (int q = 0; q < 4; ++q)
        ra[q][t] = (ok && q < nil) ? *reinterpret_cast<const V*>(Aq[q] + row * g.lda + c) : zero16<T>();
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t rc = r0; rc < r1; rc += KC) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int v = tid + 256 * t;
      if (v < NV) {
        const int r = v / (TP / VN), c = (v % (TP / VN)) * VN;
        put16<T>(sB + r * LD + c, rb[t]);
#pragma unroll
        for (int q = 0; q < 4; ++q) put16<T>(sA[q] + r * LD + c, ra[q][t]);
      }
    }
    __syncthreads();
    if (rc + KC < r1) fetch(rc + KC);
    if (q < nil) {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        T af[TB], bf[TB];
#pragma unroll
        for (int a = 0; a < TB; ++a) af[a] = (a >= ra0 && a < ra1) ? sA[q][(kk + lk) * LD + a * 16 + li] : T(0);
#pragma unroll
        for (int b = 0; b < TB; ++b) bf[b] = sB[(kk + lk) * LD + b * 16 + li];
#pragma unroll
        for (int a = 0; a < TB; ++a)
          if (a >= ra0 && a < ra1) {
#pragma unroll
            for (int b = 0; b < TB; ++b) acc[a][b] = Mfma<T>::mma(af[a], bf[b], acc[a][b]);
          }
      }
    }
    __syncthreads();
  }
  if (q >= nil) return;
  const int item = s * g.ni + i0 + q;
  T* out = partial + ((int64_t)item * nsplit + split) * TP * TP;
#pragma unroll
  for (int a = 0; a < TB; ++a)
    if (a >= ra0 && a < ra1) {
#pragma unroll
      for (int b = 0; b < TB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(int64_t)(a * 16 + Mfma<T>::row(lk, v)) * TP + b * 16 + li] = acc[a][b][v];
    }
}

// The same products with eight waves: G[s, i] = A_{s,i}^T B_s for the nil <= NIL blocks
// i = NIL y .. of a shift, each (16 TB) x (16 TB).  The nil * TB row blocks of 16 go round-robin
// to the waves (wave w: row blocks w, w + 8, ..), each wave taking all TB column blocks of its
// rows, so three blocks keep every wave busy and a wave holds at most ceil(NIL TB / 8) x TB
// MFMA tiles.  The B tile and the nil A tiles of a K chunk are staged once for the workgroup.
// NIL = 1 (one block against B) deals the TB x TB output tiles round-robin to the waves
// instead, so that all eight waves compute.
// grid: x = row split, y = group of NIL blocks, z = shift.
template <class T, int TB, int NIL, int KC, bool DB>
__global__ __launch_bounds__(512) void k_gram_rows(GramArgs g, int nsplit, int64_t rows_per_split,
                                                   T* __restrict__ partial) {
  using V = typename V16T<T>::t;
  constexpr int VN = V16T<T>::N;
  constexpr int TP = TB * 16;
  constexpr int LD = lds_ld<T>(TP);
  constexpr int NV = KC * TP / VN;  // 16-byte vectors per operand tile
  constexpr int NT = NIL + 1;       // staged tiles: the A blocks, then B
  constexpr int PER = (NT * NV + 511) / 512;
  constexpr int MAXR = (NIL * TB + 7) / 8;
  constexpr int NBUF = DB ? 2 : 1;  // DB: two LDS buffers, the next chunk stored while this one computes
  __shared__ T sT[NBUF * NT * KC * LD];
  const int s = blockIdx.z;
  if (g.active != nullptr && g.active[s] == 0) return;
  const int i0 = blockIdx.y * NIL;
  const int nil = min(NIL, g.ni - i0);
  const int split = blockIdx.x;
  const int64_t r0 = (int64_t)split * rows_per_split;
  const int64_t r1 = min(g.n, r0 + rows_per_split);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  // tile t < nil: A block i0 + t (the shift's last one possibly from A_last); t = NIL: B
  const T* const Ab = static_cast<const T*>(g.A) + s * g.a_s;
  const T* const Al = g.A_last != nullptr ? static_cast<const T*>(g.A_last) + s * g.a_s : nullptr;
  const T* const Bb = static_cast<const T*>(g.B) + s * g.b_s;
  // the group's last block is B itself (A_last == B, one shift): its Gram with B is symmetric
  const bool sym = NIL != 1 && Al != nullptr && g.A_last == g.B && g.a_s == 0 && g.b_s == 0 && i0 + NIL >= g.ni;
  constexpr bool TILES = NIL == 1;
  constexpr int MAXT = (TB * TB + 7) / 8;  // tiles per wave (NIL = 1)
  typename Mfma<T>::acc acc[TILES ? 1 : MAXR][TB];
  typename Mfma<T>::acc acct[TILES ? MAXT : 1];
#pragma unroll
  for (int r = 0; r < (TILES ? 1 : MAXR); ++r)
#pragma unroll
    for (int b = 0; b < TB; ++b) acc[r][b] = Mfma<T>::zero();
#pragma unroll
  for (int t = 0; t < (TILES ? MAXT : 1); ++t) acct[t] = Mfma<T>::zero();
  V pre[PER];
  auto fetch = [&](int64_t rc) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 512 * u;
      const int t = e / NV, v = e % NV;
      const int r = v / (TP / VN), c = (v % (TP / VN)) * VN;
      const int64_t row = rc + r;
      pre[u] = zero16<T>();
      if (t < NT && (t == NIL || t < nil) && row < r1) {
        // the tile's source, computed (an indexed pointer array would live in scratch)
        const T* p = t == NIL ? Bb : ((Al != nullptr && i0 + t == g.ni - 1) ? Al : Ab + (i0 + t) * g.a_i);
        const int64_t ld = t == NIL ? g.ldb : g.lda;
        pre[u] = *reinterpret_cast<const V*>(p + row * ld + c);
      }
    }
  };
  auto stage = [&](T* buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 512 * u;
      const int t = e / NV, v = e % NV;
      if (t < NT) {
        const int r = v / (TP / VN), c = (v % (TP / VN)) * VN;
        put16<T>(buf + (t * KC + r) * LD + c, pre[u]);
      }
    }
  };
  auto compute = [&](const T* buf) {
    const T* sB = buf + NIL * KC * LD;
    if constexpr (TILES) {
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
          const int tile = wave + 8 * t;
          if (tile < TB * TB) {
            const int rb = tile / TB, cb = tile % TB;
            const T af = buf[(kk + lk) * LD + rb * 16 + li];
            const T bf = sB[(kk + lk) * LD + cb * 16 + li];
            acct[t] = Mfma<T>::mma(af, bf, acct[t]);
          }
        }
      }
      return;
    }
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T bf[TB];
#pragma unroll
      for (int b = 0; b < TB; ++b) bf[b] = sB[(kk + lk) * LD + b * 16 + li];
#pragma unroll
      for (int r = 0; r < MAXR; ++r) {
        const int rb = wave + 8 * r;
        if (rb < nil * TB) {
          const int blk = rb / TB, lr = rb % TB;
          const T af = buf[(blk * KC + kk + lk) * LD + lr * 16 + li];
          // the last block's self Gram is symmetric: only its tiles on and above the diagonal
          const int bmin = (sym && blk == nil - 1) ? lr : 0;
#pragma unroll
          for (int b = 0; b < TB; ++b)
            if (b >= bmin) acc[r][b] = Mfma<T>::mma(af, bf[b], acc[r][b]);
        }
      }
    }
  };
  if (r0 < r1) fetch(r0);
  if constexpr (DB) {
    // one barrier per chunk: chunk c computes from buffer c & 1 while the loads of chunk c + 1
    // are in flight, then stages them into the other buffer (last read in chunk c - 1)
    if (r0 < r1) stage(sT);
    __syncthreads();
    int cur = 0;
    for (int64_t rc = r0; rc < r1; rc += KC) {
      const bool more = rc + KC < r1;
      if (more) fetch(rc + KC);
      compute(sT + cur * NT * KC * LD);
      if (more) stage(sT + (cur ^ 1) * NT * KC * LD);
      __syncthreads();
      cur ^= 1;
    }
  } else {
    for (int64_t rc = r0; rc < r1; rc += KC) {
      stage(sT);
      __syncthreads();
      if (rc + KC < r1) fetch(rc + KC);
      compute(sT);
      __syncthreads();
    }
  }
  if constexpr (TILES) {
    T* out = partial + ((int64_t)(s * g.ni + i0) * nsplit + split) * TP * TP;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      const int tile = wave + 8 * t;
      if (tile >= TB * TB) continue;
      const int rb = tile / TB, cb = tile % TB;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(int64_t)(rb * 16 + Mfma<T>::row(lk, v)) * TP + cb * 16 + li] = acct[t][v];
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    const int rb = wave + 8 * r;
    if (rb >= nil * TB) continue;
    const int blk = rb / TB, lr = rb % TB;
    T* out = partial + ((int64_t)(s * g.ni + i0 + blk) * nsplit + split) * TP * TP;
    const bool sb = sym && blk == nil - 1;
#pragma unroll
    for (int b = 0; b < TB; ++b) {
      if (sb && b < lr) continue;  // written below, as the transpose of tile (b, lr)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = lr * 16 + Mfma<T>::row(lk, v), col = b * 16 + li;
        out[(int64_t)row * TP + col] = acc[r][b][v];
        if (sb && b > lr) out[(int64_t)col * TP + row] = acc[r][b][v];
      }
    }
  }
}

inline int gram_tb(int W) {
  // tile blocks per dimension: at most 10 (160 reals), as few tiles as possible
  const int nb = W / 16;
  const int nt = (nb + 9) / 10;
  return (nb + nt - 1) / nt;
}

// Workgroups of k_gram<T, tb> resident on the whole device at once.
template <class T>
int gram_capacity(int tb);

// Row splits per (item, tile): enough workgroups to fill the device twice, and a total that
// does not exceed two full waves of resident workgroups (a third, nearly empty wave would
// cost as much as a full one).  At least 1024 rows per split.
// min_rows: smallest row range of one split (1024; 512 for the four-block kernel and for one
// or two tiles, which otherwise leave too few workgroups in flight: measured on the device).
inline int gram_nsplit(int64_t n, int items, int tiles, int cap, int64_t min_rows = 1024) {
  const int64_t per = (int64_t)items * tiles;
  const int64_t target = 2 * (int64_t)std::max(cap, 1);
  const int64_t want = std::max<int64_t>(1, target / per);
  const int64_t maxs = std::max<int64_t>(1, n / min_rows);
  return (int)std::min(want, maxs);
}

// ------------------------------------------------------------------ apply
// O_item = beta O_item + alpha sum_b A_b Bm_b.  grid: x = 64 RB-row tile (XCD
// renumbered), y = output column tile, z = item.  Wave w owns rows
// [16 RB w, 16 RB (w+1)) of the tile (RB MFMA row blocks) and TBQ column blocks.
template <class T> struct ApplyCfg { static constexpr int KC = 32; };
template <> struct ApplyCfg<double> { static constexpr int KC = 16; };

template <class T, class TO, int TBQ, int RB = 2, int KCX = ApplyCfg<T>::KC>
__global__ __launch_bounds__(256) void k_apply(ApplyArgs a, int per) {
  using V = typename V16T<T>::t;
  constexpr int VN = V16T<T>::N;
  constexpr int KC = KCX;
  constexpr int RT = 64 * RB;  // 4 waves x RB row blocks of 16
  constexpr int TQ = TBQ * 16;
  constexpr int LDA_S = KC + 4;
  constexpr int LDB_S = lds_ld<T>(TQ);
  constexpr int NVA = RT * KC / VN, PERA = (NVA + 255) / 256;
  constexpr int NVB = KC * TQ / VN, PERB = (NVB + 255) / 256;
  __shared__ T sA[RT * LDA_S];
  __shared__ T sB[KC * LDB_S];

  const int item = blockIdx.z;
  if (a.active_item != nullptr && a.active_item[item] == 0) return;
  const int64_t nrt = (a.n + RT - 1) / RT;
  const int64_t rt = xcd_block(blockIdx.x, per);
  if (rt >= nrt) return;
  const int64_t r0 = rt * RT;
  const int q0 = blockIdx.y * TQ;
  const int vq = min(TQ, a.OW - q0);

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  typename Mfma<T>::acc acc[RB][TBQ];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int t = 0; t < TBQ; ++t) acc[r][t] = Mfma<T>::zero();

  const T* __restrict__ Abase = static_cast<const T*>(a.A) + item * a.a_item;
  const T* __restrict__ Bbase = static_cast<const T*>(a.Bm) + item * a.bm_item;
  const int nkc = (a.KW + KC - 1) / KC;
  // flattened (block, k-chunk) loop with register prefetch
  V ra[PERA], rb[PERB];
  auto fetch = [&](int b, int k0) {
    const int sb = b / a.nbi, ib = b % a.nbi;
    const T* __restrict__ Ab = (a.A_last != nullptr && b == a.nb - 1)
                                   ? static_cast<const T*>(a.A_last) + item * a.a_item
                                   : Abase + sb * a.a_s + ib * a.a_i;
    const T* __restrict__ Bb = Bbase + (int64_t)b * a.KW * a.OW;
#pragma unroll
    for (int t = 0; t < PERA; ++t) {
      const int v = tid + 256 * t;
      ra[t] = zero16<T>();
      if (v < NVA) {
        const int r = v / (KC / VN), c = (v % (KC / VN)) * VN;
        const int64_t row = r0 + r;
        if (row < a.n && k0 + c < a.KW) ra[t] = *reinterpret_cast<const V*>(Ab + row * a.lda + k0 + c);
      }
    }
#pragma unroll
    for (int t = 0; t < PERB; ++t) {
      const int v = tid + 256 * t;
      rb[t] = zero16<T>();
      if (v < NVB) {
        const int r = v / (TQ / VN), c = (v % (TQ / VN)) * VN;
        if (k0 + r < a.KW && c < vq) rb[t] = *reinterpret_cast<const V*>(Bb + (int64_t)(k0 + r) * a.OW + q0 + c);
      }
    }
  };
  auto skip = [&](int b) { return a.active_sb != nullptr && a.active_sb[b / a.nbi] == 0; };
  int b = 0, kc = 0;
  while (b < a.nb && skip(b)) ++b;
  if (b < a.nb) fetch(b, 0);
  while (b < a.nb) {
#pragma unroll
    for (int t = 0; t < PERA; ++t) {
      const int v = tid + 256 * t;
      if (v < NVA) {
        const int r = v / (KC / VN), c = (v % (KC / VN)) * VN;
        put16<T>(sA + r * LDA_S + c, ra[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < PERB; ++t) {
      const int v = tid + 256 * t;
      if (v < NVB) {
        const int r = v / (TQ / VN), c = (v % (TQ / VN)) * VN;
        put16<T>(sB + r * LDB_S + c, rb[t]);
      }
    }
    __syncthreads();
    // next (block, chunk)
    int nb_ = b, nk = kc + 1;
    if (nk >= nkc) {
      nk = 0;
      ++nb_;
      while (nb_ < a.nb && skip(nb_)) ++nb_;
    }
    if (nb_ < a.nb) fetch(nb_, nk * KC);
    // block 0 with a lower (upper) triangular coefficient: the output column tiles right (left) of
    // this K chunk get nothing from it
    const int tri_from = (a.lower0 && b == 0) ? kc * KC + KC - 1 : (1 << 30);
    const int tri_to = (a.upper0 && b == 0) ? kc * KC - 15 : -(1 << 30);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      T af[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) af[r] = sA[(wave * 16 * RB + r * 16 + li) * LDA_S + kk + lk];
#pragma unroll
      for (int t = 0; t < TBQ; ++t) {
        if (t * 16 < vq && q0 + t * 16 <= tri_from && q0 + t * 16 >= tri_to) {
          const T bv = sB[(kk + lk) * LDB_S + t * 16 + li];
          // transposed product: the MFMA computes (A Bm)^T blocks, so a lane ends up holding
          // consecutive output columns of one row
#pragma unroll
          for (int r = 0; r < RB; ++r) acc[r][t] = Mfma<T>::mma(bv, af[r], acc[r][t]);
        }
      }
    }
    __syncthreads();
    b = nb_;
    kc = nk;
  }

  TO* __restrict__ O = static_cast<TO*>(a.O) + item * a.o_item;
  // lane (li, lk) holds output row li of each 16-row block and its columns Mfma<T>::row(lk, v)
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int64_t row = r0 + wave * 16 * RB + r * 16 + li;
    if (row >= a.n) continue;
    TO* __restrict__ orow = O + row * a.ldo + q0;
#pragma unroll
    for (int t = 0; t < TBQ; ++t) {
      if (t * 16 >= vq) continue;
      if constexpr (sizeof(T) == 4) {
        // four consecutive columns 16 t + 4 lk .. + 3
        TO* o = orow + t * 16 + 4 * lk;
        TO val[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) val[v] = (TO)(a.alpha * (double)acc[r][t][v]);
        if constexpr (sizeof(TO) == 4) {
          float4* o4 = reinterpret_cast<float4*>(o);
          float4 w = make_float4(val[0], val[1], val[2], val[3]);
          if (a.beta != 0.0) {
            const float4 old = *o4;
            const float bt = (float)a.beta;
            w = make_float4(bt * old.x + w.x, bt * old.y + w.y, bt * old.z + w.z, bt * old.w + w.w);
          }
          *o4 = w;
        } else {
          double2* o2 = reinterpret_cast<double2*>(o);
          double2 w0 = make_double2(val[0], val[1]), w1 = make_double2(val[2], val[3]);
          if (a.beta != 0.0) {
            const double2 p0 = o2[0], p1 = o2[1];
            w0 = make_double2(a.beta * p0.x + w0.x, a.beta * p0.y + w0.y);
            w1 = make_double2(a.beta * p1.x + w1.x, a.beta * p1.y + w1.y);
          }
          o2[0] = w0;
          o2[1] = w1;
        }
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          TO* o = orow + t * 16 + Mfma<T>::row(lk, v);
          const TO val = (TO)(a.alpha * (double)acc[r][t][v]);
          *o = (a.beta == 0.0) ? val : (TO)(a.beta * (double)(*o)) + val;
        }
      }
    }
  }
}

}  // namespace

namespace {
template <class T, int TB>
int gram_capacity_of() {
  // without a device (host-only footprint queries) assume a large device: the row-split
  // count, and with it the partial-sum buffer, only grows with the capacity
  static int cap = -1;
  if (cap < 0) {
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_gram<T, TB>), 256, 0) !=
            hipSuccess ||
        occ < 1 || cus < 1)
      return 2048;
    cap = occ * cus;
  }
  return cap;
}

template <class T, int TB>
int gram4_capacity_of() {
  static int cap = -1;
  if (cap < 0) {
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_gram4<T, TB, 16>), 256, 0) !=
            hipSuccess ||
        occ < 1 || cus < 1)
      return 2048;
    cap = occ * cus;
  }
  return cap;
}

template <class T>
int gram4_capacity(int tb) {
  switch (tb) {
    case 1: return gram4_capacity_of<T, 1>();
    case 2: return gram4_capacity_of<T, 2>();
    case 3: return gram4_capacity_of<T, 3>();
    case 4: return gram4_capacity_of<T, 4>();
    default: return gram4_capacity_of<T, 5>();
  }
}

// Workgroups of the eight-wave single-block Gram resident on the whole device at once.
template <class T, int TB>
int gram_rows1_capacity_of() {
  static int cap = -1;
  if (cap < 0) {
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_gram_rows<T, TB, 1, 32, true>),
                                                     512, 0) != hipSuccess ||
        occ < 1 || cus < 1)
      return 1024;
    cap = occ * cus;
  }
  return cap;
}
template <class T>
int gram_rows1_capacity(int tb) {
  switch (tb) {
    case 1: return gram_rows1_capacity_of<T, 1>();
    case 2: return gram_rows1_capacity_of<T, 2>();
    case 3: return gram_rows1_capacity_of<T, 3>();
    case 4: return gram_rows1_capacity_of<T, 4>();
    default: return gram_rows1_capacity_of<T, 5>();
  }
}

// k_gram4 applies to square products of at most 80 columns whose right operand is shared by
// the blocks of a shift
// (FP64 at 80 columns would spill at two waves per SIMD: it keeps the one-block kernel)
template <class T>
bool gram4_fits(const GramArgs& g) {
  const int maxw = sizeof(T) == 4 ? 80 : 64;
  return g.PW == g.QW && g.PW % 16 == 0 && g.PW <= maxw && g.ni >= 2 && g.b_i == 0;
}

template <class T>
int gram_capacity(int tb) {
  switch (tb) {
    case 1: return gram_capacity_of<T, 1>();
    case 2: return gram_capacity_of<T, 2>();
    case 3: return gram_capacity_of<T, 3>();
    case 4: return gram_capacity_of<T, 4>();
    case 5: return gram_capacity_of<T, 5>();
    case 6: return gram_capacity_of<T, 6>();
    case 7: return gram_capacity_of<T, 7>();
    case 8: return gram_capacity_of<T, 8>();
    case 9: return gram_capacity_of<T, 9>();
    default: return gram_capacity_of<T, 10>();
  }
}
}  // namespace

// Largest tile (in 16-column blocks) of the Gram kernel; 0 = as wide as the operands allow.
int g_gram_variant = 0;
// K chunk of the four-block Gram kernel (32, or 16).
int g_gram4_kc = 32;
// FP32 multi-block Grams: the eight-wave kernel (1) or the four-wave one (0).
int g_gram_rows = 1;
// FP32 single-block square Grams: the eight-wave kernel with the tiles dealt to the waves (1) or
// the four-wave tile kernel (0).
int g_gram_rows1 = 1;

template <class T>
size_t gram_partial_bytes(int64_t n, int PW, int QW, int items) {
  // the largest over the tilings launch_gram may choose (the four-block kernel when one shift
  // has all the items: the fewest groups, the most row splits)
  size_t best = 0;
  if (PW == QW && PW % 16 == 0 && PW <= (sizeof(T) == 4 ? 80 : 64) && items >= 2) {
    const int groups = (items + 3) / 4;
    const int ns = gram_nsplit(n, groups, 1, gram4_capacity<T>(PW / 16), 512);
    best = (size_t)items * ns * PW * QW * sizeof(T);
  }
  const int tb0 = std::max(gram_tb(PW), gram_tb(QW));
  for (int tb = 1; tb <= tb0; ++tb) {
    const int tiles = ((PW / 16 + tb - 1) / tb) * ((QW / 16 + tb - 1) / tb);
    const int ns = gram_nsplit(n, items, tiles, gram_capacity<T>(tb), items * tiles <= 2 ? 512 : 1024);
    best = std::max(best, (size_t)items * ns * PW * QW * sizeof(T));
  }
  return best;
}

template <class T>
void launch_gram(hipStream_t st, const GramArgs& g, void* partial, size_t partial_bytes) {
  IF_REQUIRE(g.PW % 16 == 0 && g.QW % 16 == 0, "gram: widths must be multiples of 16");
  if constexpr (sizeof(T) == 4) {
    // one square block per shift (FP32, at most 80 columns): the eight-wave kernel with the output
    // tiles dealt to the waves
    if (g_gram_rows1 && g_gram_variant >= 0 && g.ni == 1 && g.PW == g.QW && g.PW <= 80 && g.b_i == 0) {
      const int tb = g.PW / 16;
      int nsplit = gram_nsplit(g.n, g.ns, 1, gram_rows1_capacity<T>(tb), 512);
      nsplit = (int)std::max<size_t>(1, std::min<size_t>(nsplit, partial_bytes / ((size_t)g.ns * g.PW * g.QW * sizeof(T))));
      int64_t rps = (g.n + nsplit - 1) / nsplit;
      rps = (rps + 31) / 32 * 32;
      T* part = static_cast<T*>(partial);
      KernelTimer* kt = g.kclass >= 0 ? current_timer() : nullptr;
      const int tok = kt ? kt->begin(st) : -1;
      const dim3 grid(nsplit, 1, g.ns), block(512);
      switch (tb) {
        case 1: hipLaunchKernelGGL((k_gram_rows<T, 1, 1, 32, true>), grid, block, 0, st, g, nsplit, rps, part); break;
        case 2: hipLaunchKernelGGL((k_gram_rows<T, 2, 1, 32, true>), grid, block, 0, st, g, nsplit, rps, part); break;
        case 3: hipLaunchKernelGGL((k_gram_rows<T, 3, 1, 32, true>), grid, block, 0, st, g, nsplit, rps, part); break;
        case 4: hipLaunchKernelGGL((k_gram_rows<T, 4, 1, 32, true>), grid, block, 0, st, g, nsplit, rps, part); break;
        default: hipLaunchKernelGGL((k_gram_rows<T, 5, 1, 32, true>), grid, block, 0, st, g, nsplit, rps, part); break;
      }
      IF_HIP(hipGetLastError());
      if (kt) {
        const int nact = kt->count(g.active, g.ns);
        const double rb = g.A == g.B ? 0.0 : (double)g.n * g.QW * sizeof(T) * nact;
        kt->end(tok, g.kclass, 2.0 * g.n * g.PW * g.QW * nact, (double)g.n * g.PW * sizeof(T) * nact + rb);
      }
      const int64_t total = (int64_t)g.ns * g.PW * g.QW;
      hipLaunchKernelGGL((k_gram_reduce<T>), dim3((unsigned)((total + 63) / 64)), dim3(64 * kRedWaves), 0, st, g.ns,
                         nsplit, g.PW, g.QW, 1, g.active, part, g.G, g.cmb);
      IF_HIP(hipGetLastError());
      return;
    }
  }
  if (gram4_fits<T>(g) && g_gram_variant >= 0) {
    const int tb = g.PW / 16;
    const int groups = (g.ni + 3) / 4;
    const int items = g.ns * g.ni;
    int nsplit = gram_nsplit(g.n, g.ns * groups, 1, gram4_capacity<T>(tb), 512);
    // with slots held by concurrent work, one round on the rest (a second, nearly empty round
    // would cost as much as the first)
    if (g.reserve > 0) nsplit = std::min(nsplit, std::max(1, gram4_capacity<T>(tb) / (g.ns * groups) - g.reserve));
    IF_REQUIRE((size_t)items * nsplit * g.PW * g.QW * sizeof(T) <= partial_bytes, "gram: partial buffer too small");
    // K chunk (rows per staged tile): 32 (measured fastest, two waves per SIMD still fit) or 16
    const int kc = g_gram4_kc == 16 ? 16 : 32;
    int64_t rps = (g.n + nsplit - 1) / nsplit;
    rps = (rps + 31) / 32 * 32;
    const dim3 grid(nsplit, groups, g.ns), block(256);
    T* part = static_cast<T*>(partial);
    KernelTimer* kt = g.kclass >= 0 ? current_timer() : nullptr;
    const int tok = kt ? kt->begin(st) : -1;
#define IF_G4(TB_, KC_) hipLaunchKernelGGL((k_gram4<T, TB_, KC_>), grid, block, 0, st, g, nsplit, rps, part)
#define IF_GR(TB_, NIL_)                                                                                        \
  hipLaunchKernelGGL((k_gram_rows<T, TB_, NIL_, 32, (NIL_ < 4)>), dim3(nsplit, (g.ni + NIL_ - 1) / NIL_, g.ns),   \
                     dim3(512), 0, st, g, nsplit, rps, part)
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      if (g_gram_rows) {
        // eight waves, row blocks round-robin: groups of three blocks when there are exactly three
        const int nil = g.ni == 2 ? 2 : (g.ni == 3 ? 3 : 4);
#define IF_GR_TB(TB_) \
  if (nil == 2) IF_GR(TB_, 2); else if (nil == 3) IF_GR(TB_, 3); else IF_GR(TB_, 4);
        switch (tb) {
          case 1: IF_GR_TB(1) break;
          case 2: IF_GR_TB(2) break;
          case 3: IF_GR_TB(3) break;
          case 4: IF_GR_TB(4) break;
          default: IF_GR_TB(5) break;
        }
#undef IF_GR_TB
        done = true;
      }
    }
    if (done) {
    } else if (kc == 32) {
      switch (tb) {
        case 1: IF_G4(1, 32); break;
        case 2: IF_G4(2, 32); break;
        case 3: IF_G4(3, 32); break;
        case 4: IF_G4(4, 32); break;
        default: IF_G4(5, 32); break;
      }
    } else {
      switch (tb) {
        case 1: IF_G4(1, 16); break;
        case 2: IF_G4(2, 16); break;
        case 3: IF_G4(3, 16); break;
        case 4: IF_G4(4, 16); break;
        default: IF_G4(5, 16); break;
      }
    }
#undef IF_G4
#undef IF_GR
    IF_HIP(hipGetLastError());
    if (kt) {
      const int nact = kt->count(g.active, g.ns);
      const double eff = (double)nact * g.ni;
      // the self Gram (A == B, one block, or B as the last block) reads B once, as an A block; the
      // eight-wave kernel forms that last block's symmetric product from its upper triangle, which
      // counts n m0 (m0 + 1) flops
      const double rb = ((g.A == g.B && g.ni == 1) || g.A_last == g.B) ? 0.0 : (double)g.n * g.QW * sizeof(T) * nact;
      const bool symk = sizeof(T) == 4 && g_gram_rows && g.A_last == g.B && g.a_s == 0 && g.b_s == 0;
      const double fl = symk ? 2.0 * g.n * g.PW * g.QW * (eff - 1) + (double)g.n * g.PW * (g.QW + 1)
                             : 2.0 * g.n * g.PW * g.QW * eff;
      kt->end(tok, g.kclass, fl, (double)g.n * g.PW * sizeof(T) * eff + rb);
    }
    const int64_t total = (int64_t)items * g.PW * g.QW;
    hipLaunchKernelGGL((k_gram_reduce<T>), dim3((unsigned)((total + 63) / 64)), dim3(64 * kRedWaves), 0, st, items,
                       nsplit, g.PW, g.QW, g.ni, g.active, part, g.G, g.cmb);
    IF_HIP(hipGetLastError());
    return;
  }
  // one square tile size for both dimensions
  int tb = std::max(gram_tb(g.PW), gram_tb(g.QW));
  if (g_gram_variant > 0 && tb > g_gram_variant) tb = g_gram_variant;
  if (g.tb_cap > 0 && tb > g.tb_cap) tb = g.tb_cap;
  const int ntp = (g.PW / 16 + tb - 1) / tb, ntq = (g.QW / 16 + tb - 1) / tb;
  const int items = g.ns * g.ni;
  const int nsplit = gram_nsplit(g.n, items, ntp * ntq, gram_capacity<T>(tb), items * ntp * ntq <= 2 ? 512 : 1024);
  IF_REQUIRE((size_t)items * nsplit * g.PW * g.QW * sizeof(T) <= partial_bytes, "gram: partial buffer too small");
  constexpr int KC = GramCfg<T>::KC;
  int64_t rps = (g.n + nsplit - 1) / nsplit;
  rps = (rps + KC - 1) / KC * KC;
  const dim3 grid(nsplit, ntp * ntq, items), block(256);
  T* part = static_cast<T*>(partial);
  KernelTimer* kt = g.kclass >= 0 ? current_timer() : nullptr;
  const int tok = kt ? kt->begin(st) : -1;
  switch (tb) {
    case 1: hipLaunchKernelGGL((k_gram<T, 1>), grid, block, 0, st, g, nsplit, rps, ntq, part); break;
    case 2: hipLaunchKernelGGL((k_gram<T, 2>), grid, block, 0, st, g, nsplit, rps, ntq, part); break;
    case 3: hipLaunchKernelGGL((k_gram<T, 3>), grid, block, 0, st, g, nsplit, rps, ntq, part); break;
    case 4: hipLaunchKernelGGL((k_gram<T, 4>), grid, block, 0, st, g, nsplit, rps, ntq, part); break;
    case 5: hipLaunchKernelGGL((k_gram<T, 5>), grid, block, 0, st, g, nsplit, rps, ntq, part); break;
    case 6: hipLaunchKernelGGL((k_gram<T, 6>), grid, block, 0, st, g, nsplit, rps, ntq, part); break;
    case 7: hipLaunchKernelGGL((k_gram<T, 7>), grid, block, 0, st, g, nsplit, rps, ntq, part); break;
    case 8: hipLaunchKernelGGL((k_gram<T, 8>), grid, block, 0, st, g, nsplit, rps, ntq, part); break;
    case 9: hipLaunchKernelGGL((k_gram<T, 9>), grid, block, 0, st, g, nsplit, rps, ntq, part); break;
    case 10: hipLaunchKernelGGL((k_gram<T, 10>), grid, block, 0, st, g, nsplit, rps, ntq, part); break;
    default: throw Error{IFEAST_ERR_INVALID_ARG, "gram: unsupported tile"};
  }
  IF_HIP(hipGetLastError());
  if (kt) {
    // algorithmic: every active item's A block once; B once per item, or once per shift when the
    // blocks of a shift share it (b_i == 0); the self Gram (A == B, one block, or B as the last
    // block) reads B once, as an A block
    const int nact = kt->count(g.active, g.ns);
    const double eff = (double)nact * g.ni;
    const double ra = (double)g.n * g.PW * sizeof(T) * eff;
    const double rb = ((g.A == g.B && g.ni == 1) || g.A_last == g.B)
                          ? 0.0
                          : (double)g.n * g.QW * sizeof(T) * (g.b_i == 0 ? nact : eff);
    kt->end(tok, g.kclass, 2.0 * g.n * g.PW * g.QW * eff, ra + rb);
  }
  const int64_t total = (int64_t)items * g.PW * g.QW;
  hipLaunchKernelGGL((k_gram_reduce<T>), dim3((unsigned)((total + 63) / 64)), dim3(64 * kRedWaves), 0, st, items,
                     nsplit, g.PW, g.QW, g.ni, g.active, part, g.G, g.cmb);
  IF_HIP(hipGetLastError());
}

// Row blocks per wave and K chunk of the FP32 update kernel (FP64: g_apply_rb64); -1 selects the
// built-in choice measured fastest: one row block per wave for 144- and 160-column tiles (the most
// resident waves), two row blocks with a 32-row K chunk for 96- to 128-column tiles (one row block
// there is unrolled into more than 256 registers and runs one wave per SIMD: 14x slower at 128
// columns), two with a 16-row K chunk up to 80 columns.
int g_apply_variant = -1;
// Row blocks per wave of the FP64 update kernel (1 or 2); <= 0 selects the built-in choice (1).
int g_apply_rb64 = 0;

template <class T, class TO, int RB, int KC>
void launch_apply_rt(hipStream_t st, const ApplyArgs& a, int tbq, int ntq, KernelTimer* kt, int& tok) {
  constexpr int RT = 64 * RB;
  const int64_t nrt = (a.n + RT - 1) / RT;
  const int per = (int)((nrt + kXcds - 1) / kXcds);
  const dim3 grid(per * kXcds, ntq, a.items), block(256);
  tok = kt ? kt->begin(st) : -1;
  switch (tbq) {
    case 1: hipLaunchKernelGGL((k_apply<T, TO, 1, RB, KC>), grid, block, 0, st, a, per); break;
    case 2: hipLaunchKernelGGL((k_apply<T, TO, 2, RB, KC>), grid, block, 0, st, a, per); break;
    case 3: hipLaunchKernelGGL((k_apply<T, TO, 3, RB, KC>), grid, block, 0, st, a, per); break;
    case 4: hipLaunchKernelGGL((k_apply<T, TO, 4, RB, KC>), grid, block, 0, st, a, per); break;
    case 5: hipLaunchKernelGGL((k_apply<T, TO, 5, RB, KC>), grid, block, 0, st, a, per); break;
    case 6: hipLaunchKernelGGL((k_apply<T, TO, 6, RB, KC>), grid, block, 0, st, a, per); break;
    case 7: hipLaunchKernelGGL((k_apply<T, TO, 7, RB, KC>), grid, block, 0, st, a, per); break;
    case 8: hipLaunchKernelGGL((k_apply<T, TO, 8, RB, KC>), grid, block, 0, st, a, per); break;
    case 9: hipLaunchKernelGGL((k_apply<T, TO, 9, RB, KC>), grid, block, 0, st, a, per); break;
    case 10: hipLaunchKernelGGL((k_apply<T, TO, 10, RB, KC>), grid, block, 0, st, a, per); break;
    default: throw Error{IFEAST_ERR_INVALID_ARG, "apply: unsupported tile"};
  }
}

template <class T, class TO>
void launch_apply(hipStream_t st, const ApplyArgs& a) {
  IF_REQUIRE(a.OW % 16 == 0, "apply: output width must be a multiple of 16");
  const int nbq = a.OW / 16;
  const int ntq = (nbq + 9) / 10;
  const int tbq = (nbq + ntq - 1) / ntq;
  KernelTimer* kt = a.kclass >= 0 ? current_timer() : nullptr;
  int tok = -1;
  constexpr int KC0 = ApplyCfg<T>::KC;
  if (sizeof(T) == 4) {
    int var = g_apply_variant;
    if (var < 0) var = tbq >= 9 ? 3 : (tbq >= 6 ? 0 : 6);
    switch (var) {
      case 0: launch_apply_rt<T, TO, 2, 32>(st, a, tbq, ntq, kt, tok); break;
      case 1: launch_apply_rt<T, TO, 1, 64>(st, a, tbq, ntq, kt, tok); break;
      case 2: launch_apply_rt<T, TO, 1, 16>(st, a, tbq, ntq, kt, tok); break;
      case 3: launch_apply_rt<T, TO, 1, 32>(st, a, tbq, ntq, kt, tok); break;
      case 4: launch_apply_rt<T, TO, 4, 32>(st, a, tbq, ntq, kt, tok); break;
      case 5: launch_apply_rt<T, TO, 4, 16>(st, a, tbq, ntq, kt, tok); break;
      default: launch_apply_rt<T, TO, 2, 16>(st, a, tbq, ntq, kt, tok); break;
    }
  } else {
    // FP64: one row block per wave (measured faster than two at every tile width: 7 % at 80
    // columns, 15 % at 160, 35 % at 128 of a complex 256-column output, where two hold more than
    // 256 registers)
    int rb = g_apply_rb64;
    if (rb < 1) rb = 1;
    if (rb == 1)
      launch_apply_rt<T, TO, 1, KC0>(st, a, tbq, ntq, kt, tok);
    else
      launch_apply_rt<T, TO, 2, KC0>(st, a, tbq, ntq, kt, tok);
  }
  IF_HIP(hipGetLastError());
  if (kt) {
    // algorithmic: each active (item, block) reads its n x KW slab once; O is written once per
    // active item (and read first when beta != 0)
    const double it = kt->count(a.active_item, a.items);
    const double bl = a.active_sb ? (double)kt->count(a.active_sb, a.nb / a.nbi) * a.nbi : (double)a.nb;
    const double fl = 2.0 * a.n * a.KW * a.OW * it * bl;
    const double by = (double)a.n * a.KW * sizeof(T) * it * bl + (double)a.n * a.OW * sizeof(TO) * it * (a.beta != 0.0 ? 2 : 1);
    kt->end(tok, a.kclass, fl, by);
  }
}

template size_t gram_partial_bytes<float>(int64_t, int, int, int);
template size_t gram_partial_bytes<double>(int64_t, int, int, int);
template void launch_gram<float>(hipStream_t, const GramArgs&, void*, size_t);
template void launch_gram<double>(hipStream_t, const GramArgs&, void*, size_t);
template void launch_apply<float, float>(hipStream_t, const ApplyArgs&);
template void launch_apply<float, double>(hipStream_t, const ApplyArgs&);
template void launch_apply<double, double>(hipStream_t, const ApplyArgs&);

}  // namespace ifeast
