// Device kernels of the multigrid Laplacian solve (gfx950, wave64).
//
// Data layout: every n x W block is node-major (node u's W values are
// contiguous).  The W columns are split into NS slices of WS = W / NS
// columns and workgroup b works on slice b mod NS: the hardware deals
// workgroups to the 8 XCDs round-robin, so each XCD touches only its own
// column slice of every gathered row and its private L2 holds 1/NS of the
// block (8 slices of 64 columns at W = 512, 4 at W = 256 with two XCDs per
// slice, 32-column slices below).  Inside a slice a "row group" of LPR
// lanes owns one row at a time, each lane V consecutive columns
// (WS = LPR * V), so a neighbour's
// slice row is one coalesced WS*sizeof(T)-byte read.  The row groups of a
// workgroup walk a contiguous range of row tiles.
//
// The operator is the graph Laplacian L = D - A (Sec. 2); the smoother is
// weighted Jacobi S = omega D^-1; P is piecewise constant over aggregates.
// Partial sums (dot products, norms) are accumulated in FP64 per lane,
// combined across row groups through LDS in a fixed order and written per
// workgroup; a separate finalize kernel adds them in a fixed order, so every
// reduction is deterministic and free of atomics.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kern.hpp"
#include "rng.hpp"

namespace cfc {
namespace dev {

// Column slicing and lane shape of a W-wide block.
template <int W, int NSX = slices_of(W)> struct Shape {
  // column slices: at most one per XCD, 32 columns wide up to W = 128 (a
  // slice row of >= 128 B in FP32 fills whole cache lines) and 64 columns
  // from W = 256, so that the bfloat16 rows the operator product gathers
  // are 128 B too: on R-MAT-20 at W = 256, 4 slices of 64 columns measured
  // 3.05 ms per product against 3.98 ms for 8 slices of 32 (random 64-byte
  // reads use HBM worse than 128-byte ones)
  static constexpr int NS = NSX;
  static constexpr int WS = W / NS;           // columns per slice
  static constexpr int V = WS >= 4 ? 4 : 1;   // columns per lane
  static constexpr int LPR = WS / V;          // lanes per row group
  static constexpr int RG = kBlock / LPR;     // row groups per workgroup
};

// Slice of this workgroup and its index rb among the grb workgroups of that
// slice.  Workgroup b runs on XCD b mod 8; the 8/NS XCDs that share a slice
// each take a contiguous part of the row range (rb blocks in order), so a
// row's neighbours are most often in the same XCD's L2.
template <int W, int NSX = slices_of(W)>
__device__ __forceinline__ void slice_of_block(int& slice, int& rb, int& grb) {
  constexpr int NS = Shape<W, NSX>::NS;
  constexpr int XPS = 8 / NS;  // XCDs per slice
  const int b = blockIdx.x;
  slice = b % NS;
  grb = gridDim.x / NS;
  if ((gridDim.x & 7) == 0 && grb % XPS == 0)
    rb = ((b & 7) / NS) * (grb / XPS) + (b >> 3);
  else
    rb = b / NS;
}

template <typename T, int V>
struct alignas((sizeof(T) * V) >= 16 ? 16 : sizeof(T) * V) Vec {
  T v[V];
};

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> ld(const T* p) {
  return *reinterpret_cast<const Vec<T, V>*>(p);
}
template <typename T, int V>
__device__ __forceinline__ void st(T* p, const Vec<T, V>& x) {
  *reinterpret_cast<Vec<T, V>*>(p) = x;
}

// bfloat16 storage of the preconditioned residual z = S r on the depth-one
// path: z is rounded once (to nearest, ties to even) where it is formed, and
// that rounded z is what every later use sees (its own row, its
// neighbours' gathers, r.z), so the CG recurrences stay consistent
// (q = L p holds to FP32 rounding) while the gathered rows are half as wide.
typedef unsigned short bf16_t;

__device__ __forceinline__ bf16_t f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return bf16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(unsigned(h) << 16); }

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> ld_bf(const bf16_t* p) {
  const Vec<bf16_t, V> h = ld<bf16_t, V>(p);
  Vec<T, V> r;
#pragma unroll
  for (int i = 0; i < V; ++i) r.v[i] = T(bf2f(h.v[i]));
  return r;
}

// FP8 storage of z (OCP e4m3, finite range +-448) on the same paths: each
// row's column slice (the LPR lanes of one row group) shares one FP32 scale
// max|z| / 448, stored after the n x W bytes (float[n][NS] at
// f8_scale_off(n, W)).  As with bfloat16, z is rounded once where it is
// formed and every later use sees the dequantised value.  The kernels that
// write or gather it run with half the regular number of column slices
// (NSX = NS / 2), so a gathered slice row is 128 bytes plus its scale.
typedef unsigned char f8_t;
constexpr float kF8Max = 448.0f;

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> ld_f8(const f8_t* p, float scale) {
  Vec<T, V> r;
  if constexpr (V == 4) {
    const int w = *reinterpret_cast<const int*>(p);
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(w, false);
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(w, true);
    r.v[0] = T(lo[0] * scale);
    r.v[1] = T(lo[1] * scale);
    r.v[2] = T(hi[0] * scale);
    r.v[3] = T(hi[1] * scale);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) r.v[i] = T(__builtin_amdgcn_cvt_f32_fp8(int(p[i]), 0) * scale);
  }
  return r;
}

// Round a row group's slice of z to FP8: the scale is the largest finite
// |z| of the slice over 448 (slices whose largest |z| is below 1e-30 are
// stored as zeros); values are clamped to +-448 (NaN stays NaN) and z is
// replaced by the dequantised values.  Lane 0 of the row group stores the
// scale.
template <typename T, int W, int NSX = slices_of(W)>
__device__ __forceinline__ void st_f8(Vec<T, Shape<W, NSX>::V>& z, f8_t* dst, float* sc_dst) {
  constexpr int LPR = Shape<W, NSX>::LPR, V = Shape<W, NSX>::V;
  float m = 0.0f;
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const float a = fabsf(float(z.v[i]));
    if (a <= 3.0e38f) m = fmaxf(m, a);
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  const float inv = m > 1e-30f ? kF8Max / m : 0.0f;
  const float scale = m > 1e-30f ? m / kF8Max : 0.0f;
  float y[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const float t = float(z.v[i]) * inv;
    y[i] = t > kF8Max ? kF8Max : (t < -kF8Max ? -kF8Max : t);
  }
  if constexpr (V == 4) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(y[0], y[1], 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(y[2], y[3], w, true);
    *reinterpret_cast<int*>(dst) = w;
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) dst[i] = f8_t(__builtin_amdgcn_cvt_pk_fp8_f32(y[i], 0.0f, 0, false) & 0xff);
  }
  if (threadIdx.x % LPR == 0) *sc_dst = scale;
  z = ld_f8<T, V>(dst, scale);
}

// Streaming (non-temporal) row access for values read or written once per
// kernel: they should not displace the rows that neighbours gather again.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> ld_nt(const T* p) {
  Vec<T, V> r;
  if constexpr ((sizeof(T) * V) % 16 == 0) {
    constexpr int C = sizeof(T) * V / 16;
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
    u32x4* o = reinterpret_cast<u32x4*>(&r);
#pragma unroll
    for (int c = 0; c < C; ++c) o[c] = __builtin_nontemporal_load(q + c);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) r.v[i] = __builtin_nontemporal_load(p + i);
  }
  return r;
}

template <typename T, int V>
__device__ __forceinline__ void st_nt(T* p, const Vec<T, V>& x) {
  if constexpr ((sizeof(T) * V) % 16 == 0) {
    constexpr int C = sizeof(T) * V / 16;
    u32x4* q = reinterpret_cast<u32x4*>(p);
    const u32x4* i = reinterpret_cast<const u32x4*>(&x);
#pragma unroll
    for (int c = 0; c < C; ++c) __builtin_nontemporal_store(i[c], q + c);
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) __builtin_nontemporal_store(x.v[k], p + k);
  }
}

// Contiguous range of row tiles for row-block rb of G row-blocks.
__device__ __forceinline__ void block_tiles(int ntiles, int rb, int G, int& tb, int& te) {
  const int per = (ntiles + G - 1) / G;
  tb = min(rb * per, ntiles);
  te = min(tb + per, ntiles);
}

// Sum acc over the row groups of the workgroup and store the WS slice
// columns to out (which points at the slice's first column).
template <int W, int NSX = slices_of(W)>
__device__ __forceinline__ void block_store(const double* acc, double* lds, double* out) {
  constexpr int LPR = Shape<W, NSX>::LPR, V = Shape<W, NSX>::V, RG = Shape<W, NSX>::RG,
                WS = Shape<W, NSX>::WS;
  const int rg = threadIdx.x / LPR, c0 = (threadIdx.x % LPR) * V;
#pragma unroll
  for (int i = 0; i < V; ++i) lds[rg * WS + c0 + i] = acc[i];
  __syncthreads();
  for (int c = threadIdx.x; c < WS; c += kBlock) {
    double s = 0;
    for (int g = 0; g < RG; ++g) s += lds[g * WS + c];
    out[c] = s;
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ T wt(const T* w, int e) {
  return w ? w[e] : T(1);
}

// nb += sum over edges e = e0 + s, e0 + s + S, ... < e1 of w_e * f(col_e),
// kGatherDepth neighbour rows in flight, added in edge order (so the depth
// does not change the result).  f returns the neighbour's WS-slice values.
#ifndef CFC_GATHER_DEPTH
#define CFC_GATHER_DEPTH 4
#endif
constexpr int kGatherDepth = CFC_GATHER_DEPTH;
// rows in flight in the FP32 heavy-row pre-pass, whose segments are long
// (R-MAT-20's operator product 3.89 against 3.97 ms at 4; the FP64
// residual's pre-pass was slower at 8)
#ifndef CFC_HEAVY_GATHER_DEPTH
#define CFC_HEAVY_GATHER_DEPTH 8
#endif
constexpr int kHeavyGatherDepth = CFC_HEAVY_GATHER_DEPTH;

template <typename T, int W, int NSX = slices_of(W), int D = kGatherDepth, class F>
__device__ __forceinline__ void gather_acc(T* nb, const int* __restrict__ col, const T* __restrict__ w,
                                           int e0, int e1, int s, int S, F&& f) {
  constexpr int V = Shape<W, NSX>::V;
  int e = e0 + s;
  for (; e + (D - 1) * S < e1; e += D * S) {
    int v[D];
    T wv[D];
    Vec<T, V> x[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      v[j] = col[e + j * S];
      wv[j] = wt(w, e + j * S);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) x[j] = f(v[j]);
#pragma unroll
    for (int i = 0; i < V; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) nb[i] += wv[j] * x[j].v[i];
  }
  for (; e < e1; e += S) {
    const int v0 = col[e];
    const T w0 = wt(w, e);
    const Vec<T, V> x0 = f(v0);
#pragma unroll
    for (int i = 0; i < V; ++i) nb[i] += w0 * x0.v[i];
  }
}

// Split decomposition: SPLIT row groups share each unit (row or aggregate),
// each taking every SPLIT-th edge; a tile holds RG / SPLIT units.  After the
// gathers, wg_combine hands each unit's leading row group (split 0) the sum
// over its SPLIT groups, in a fixed order.
template <int W, int SPLIT, int NSX = slices_of(W)>
struct Deco {
  static_assert(Shape<W, NSX>::RG % SPLIT == 0, "split must divide the row groups");
  static constexpr int PER_TILE = Shape<W, NSX>::RG / SPLIT;
  __device__ static int unit(int t, int rg) { return t * PER_TILE + rg / SPLIT; }
  __device__ static int split(int rg) { return rg % SPLIT; }
  __device__ static bool leader(int rg) { return rg % SPLIT == 0; }
};

template <typename T, int W, int SPLIT, int NSX = slices_of(W)>
__device__ __forceinline__ void wg_combine(T* nb, T* lds) {
  constexpr int LPR = Shape<W, NSX>::LPR, V = Shape<W, NSX>::V, WS = Shape<W, NSX>::WS;
  const int rg = threadIdx.x / LPR, c = (threadIdx.x % LPR) * V;
#pragma unroll
  for (int i = 0; i < V; ++i) lds[rg * WS + c + i] = nb[i];
  __syncthreads();
  if (rg % SPLIT == 0) {
#pragma unroll
    for (int i = 0; i < V; ++i) {
      T s = 0;
      for (int g = 0; g < SPLIT; ++g) s += lds[(rg + g) * WS + c + i];
      nb[i] = s;
    }
  }
  __syncthreads();
}

// nb += the segment partials of heavy row u (fixed order); no-op for a light row.
template <typename T, int W, int NSX = slices_of(W)>
__device__ __forceinline__ void add_heavy(const LevelArgs& L, int u, T* nb, int c0) {
  if (!L.heavy) return;
  const int h = L.heavy[u];
  if (h < 0) return;
  constexpr int V = Shape<W, NSX>::V;
  if (L.hsum) {
    const Vec<T, V> x = ld<T, V>(static_cast<const T*>(L.hsum) + (size_t)h * W + c0);
#pragma unroll
    for (int i = 0; i < V; ++i) nb[i] += x.v[i];
    return;
  }
  const T* hp = static_cast<const T*>(L.hpart);
  for (int sgi = L.hseg[h]; sgi < L.hseg[h + 1]; ++sgi) {
    const Vec<T, V> x = ld<T, V>(hp + (size_t)sgi * W + c0);
#pragma unroll
    for (int i = 0; i < V; ++i) nb[i] += x.v[i];
  }
}

// Heavy-row pre-pass: one workgroup per (segment, column slice); its row
// groups split the segment's edges and row group 0 stores the sum
// hpart[seg] = sum_e w_e f(col_e) with f chosen by KIND.
enum HeavyKind {
  HK_SPMM = 0, HK_RESTRICT = 1, HK_RESTRICT_UPD = 2, HK_PROLONG = 3, HK_RES64 = 4, HK_BF16 = 5,
  HK_RES32 = 6,  // T = double, the gathered block is FP32
  HK_F8 = 7      // the gathered block is FP8 with per-row-slice scales
};

template <typename T, int W, int KIND, int NSX = slices_of(W)>
__global__ __launch_bounds__(kBlock) void k_heavy(LevelArgs L, const T* __restrict__ a,
                                                  const T* __restrict__ q, const T* __restrict__ xc,
                                                  const double* __restrict__ scal) {
  constexpr int LPR = Shape<W, NSX>::LPR, V = Shape<W, NSX>::V, RG = Shape<W, NSX>::RG, WS = Shape<W, NSX>::WS;
  constexpr int HD = sizeof(T) == 4 ? kHeavyGatherDepth : kGatherDepth;
  __shared__ T ldc[RG * WS];
  int slice, sgi, nsg;
  slice_of_block<W, NSX>(slice, sgi, nsg);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const T* w = static_cast<const T*>(L.hw);
  const T* sd = static_cast<const T*>(L.sd);
  const T mu = T(L.mu);
  const float* zsc = KIND == HK_F8 ? reinterpret_cast<const float*>(
                                         reinterpret_cast<const f8_t*>(a) + f8_scale_off(L.n, W))
                                   : nullptr;
  T alpha[V];
#pragma unroll
  for (int i = 0; i < V; ++i) alpha[i] = KIND == HK_RESTRICT_UPD ? T(scal[S_ALPHA * W + c0 + i]) : T(0);
  for (; sgi < L.nseg; sgi += nsg) {
    T nb[V];
#pragma unroll
    for (int i = 0; i < V; ++i) nb[i] = 0;
    gather_acc<T, W, NSX, HD>(nb, L.hcol, w, L.seg_e[sgi], L.seg_e[sgi + 1], rg, RG, [&](int v) {
      if constexpr (KIND == HK_F8)
        return ld_f8<T, V>(reinterpret_cast<const f8_t*>(a) + (size_t)v * W + c0,
                           zsc[(size_t)v * Shape<W, NSX>::NS + slice]);
      if constexpr (KIND == HK_BF16)
        return ld_bf<T, V>(reinterpret_cast<const bf16_t*>(a) + (size_t)v * W + c0);
      if constexpr (KIND == HK_RES32) {
        const Vec<float, V> f = ld<float, V>(reinterpret_cast<const float*>(a) + (size_t)v * W + c0);
        Vec<T, V> r;
#pragma unroll
        for (int i = 0; i < V; ++i) r.v[i] = T(f.v[i]);
        return r;
      }
      Vec<T, V> r = ld<T, V>(a + (size_t)v * W + c0);
      if constexpr (KIND == HK_RESTRICT || KIND == HK_RESTRICT_UPD) {
        if constexpr (KIND == HK_RESTRICT_UPD) {
          const Vec<T, V> qv = ld<T, V>(q + (size_t)v * W + c0);
#pragma unroll
          for (int i = 0; i < V; ++i) r.v[i] -= alpha[i] * qv.v[i];
        }
        const T f = sd[v];
#pragma unroll
        for (int i = 0; i < V; ++i) r.v[i] *= f;
      } else if constexpr (KIND == HK_PROLONG) {
        const T f = sd[v];
        const Vec<T, V> xv = ld<T, V>(xc + (size_t)L.agg[v] * W + c0);
#pragma unroll
        for (int i = 0; i < V; ++i) r.v[i] = f * r.v[i] + mu * xv.v[i];
      }
      return r;
    });
    wg_combine<T, W, RG, NSX>(nb, ldc);
    if (rg == 0) {
      Vec<T, V> o;
#pragma unroll
      for (int i = 0; i < V; ++i) o.v[i] = nb[i];
      st<T, V>(static_cast<T*>(L.hpart) + (size_t)sgi * W + c0, o);
    }
  }
}

// hsum[h] = the segment partials of heavy row h added in segment order, one
// row group per heavy row with 8 partials in flight (the largest rows have
// hundreds of segments; left to the main kernels, the row groups that hold
// them would set those kernels' duration).
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_heavy_sum(LevelArgs L) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = Shape<W>::RG, WS = Shape<W>::WS;
  constexpr int D = 8;
  int slice, rb, grb;
  slice_of_block<W>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const T* hp = static_cast<const T*>(L.hpart);
  // strided rows: the longest rows (first in a hubs-first order) spread over
  // the workgroups
  const int ntiles = (L.nheavy + RG - 1) / RG;
  for (int t = rb; t < ntiles; t += grb) {
    const int h = t * RG + rg;
    if (h >= L.nheavy) continue;
    T s[V];
#pragma unroll
    for (int i = 0; i < V; ++i) s[i] = 0;
    const int k1 = L.hseg[h + 1];
    int k = L.hseg[h];
    for (; k + D <= k1; k += D) {
      Vec<T, V> x[D];
#pragma unroll
      for (int j = 0; j < D; ++j) x[j] = ld<T, V>(hp + (size_t)(k + j) * W + c0);
#pragma unroll
      for (int j = 0; j < D; ++j)
#pragma unroll
        for (int i = 0; i < V; ++i) s[i] += x[j].v[i];
    }
    for (; k < k1; ++k) {
      const Vec<T, V> x = ld<T, V>(hp + (size_t)k * W + c0);
#pragma unroll
      for (int i = 0; i < V; ++i) s[i] += x.v[i];
    }
    Vec<T, V> o;
#pragma unroll
    for (int i = 0; i < V; ++i) o.v[i] = s[i];
    st<T, V>(static_cast<T*>(L.hsum) + (size_t)h * W + c0, o);
  }
}

// ---------------------------------------------------------------------------
// PCG step on level 0: q = L z + beta q, p = z + beta p; partial p.q.
// JAC = 1: the preconditioner is one Jacobi step, and z = S r is formed on
// the fly from the residual passed in place of z (saves storing z).
// JAC = 2: z is passed as its bfloat16 copy (bf16_t[n][W]); JAC = 3: as
// its FP8 copy with per-row-slice scales.
// x (nullable, depth one): the previous iteration's x += alpha p_old is
// applied here, where p_old is read anyway, instead of in the update kernel.
template <typename T, int W, int JAC, int SPLIT, int NSX = slices_of(W)>
__global__ __launch_bounds__(kBlock) void k_spmm_pq(LevelArgs L, const T* __restrict__ z,
                                                    T* __restrict__ p, T* __restrict__ q,
                                                    T* __restrict__ x,
                                                    const double* __restrict__ scal, int first,
                                                    double* __restrict__ part) {
  constexpr int LPR = Shape<W, NSX>::LPR, V = Shape<W, NSX>::V, RG = Shape<W, NSX>::RG, WS = Shape<W, NSX>::WS;
  using D = Deco<W, SPLIT, NSX>;
  __shared__ double lds[RG * WS];
  __shared__ T ldc[SPLIT > 1 ? RG * WS : 1];
  int slice, rb, grb;
  slice_of_block<W, NSX>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const T* w = static_cast<const T*>(L.w);
  const T* deg = static_cast<const T*>(L.deg);
  const T* sd = static_cast<const T*>(L.sd);
  const f8_t* z8 = reinterpret_cast<const f8_t*>(z);
  const float* zsc = reinterpret_cast<const float*>(z8 + f8_scale_off(L.n, W));
  const bool xf = x && !first;
  T beta[V], alpha[V];
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    beta[i] = first ? T(0) : T(scal[S_BETA * W + c0 + i]);
    alpha[i] = xf ? T(scal[S_ALPHA * W + c0 + i]) : T(0);
    acc[i] = 0;
  }
  int tb, te;
  block_tiles((L.n + D::PER_TILE - 1) / D::PER_TILE, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = D::unit(t, rg);
    T nb[V];
#pragma unroll
    for (int i = 0; i < V; ++i) nb[i] = 0;
    if (u < L.n)
      gather_acc<T, W, NSX>(nb, L.col, w, L.rowptr[u], L.rowptr[u + 1], D::split(rg), SPLIT, [&](int v) {
        if constexpr (JAC == 3)
          return ld_f8<T, V>(z8 + (size_t)v * W + c0, zsc[(size_t)v * Shape<W, NSX>::NS + slice]);
        if constexpr (JAC == 2)
          return ld_bf<T, V>(reinterpret_cast<const bf16_t*>(z) + (size_t)v * W + c0);
        Vec<T, V> zv = ld<T, V>(z + (size_t)v * W + c0);
        if constexpr (JAC == 1) {
          const T f = sd[v];
#pragma unroll
          for (int i = 0; i < V; ++i) zv.v[i] *= f;
        }
        return zv;
      });
    if constexpr (SPLIT > 1) wg_combine<T, W, SPLIT, NSX>(nb, ldc);
    if (u < L.n && D::leader(rg)) {
      add_heavy<T, W, NSX>(L, u, nb, c0);
      const size_t o = (size_t)u * W + c0;
      Vec<T, V> zu;
      if constexpr (JAC == 3)
        zu = ld_f8<T, V>(z8 + o, zsc[(size_t)u * Shape<W, NSX>::NS + slice]);
      else if constexpr (JAC == 2)
        zu = ld_bf<T, V>(reinterpret_cast<const bf16_t*>(z) + o);
      else
        zu = ld<T, V>(z + o);
      if constexpr (JAC == 1) {
        const T f = sd[u];
#pragma unroll
        for (int i = 0; i < V; ++i) zu.v[i] *= f;
      }
      const T du = deg[u];
      Vec<T, V> pn, qn;
      if (first) {
        pn = zu;
#pragma unroll
        for (int i = 0; i < V; ++i) qn.v[i] = du * zu.v[i] - nb[i];
      } else {
        const Vec<T, V> po = ld_nt<T, V>(p + o), qo = ld_nt<T, V>(q + o);
#pragma unroll
        for (int i = 0; i < V; ++i) {
          pn.v[i] = zu.v[i] + beta[i] * po.v[i];
          qn.v[i] = (du * zu.v[i] - nb[i]) + beta[i] * qo.v[i];
        }
        if (xf) {
          Vec<T, V> xo = ld_nt<T, V>(x + o);
#pragma unroll
          for (int i = 0; i < V; ++i) xo.v[i] += alpha[i] * po.v[i];
          st_nt<T, V>(x + o, xo);
        }
      }
      st_nt<T, V>(p + o, pn);
      st<T, V>(q + o, qn);
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] += double(pn.v[i]) * double(qn.v[i]);
    }
  }
  block_store<W, NSX>(acc, lds, part + (size_t)rb * W + slice * WS);
}

// ---------------------------------------------------------------------------
// Update (r -= alpha q, x += alpha p) and/or pre-smooth + residual + restrict:
// bc[I] = sum_{u in I} (b - L S b)_u with b = r_out, which, the rows of an
// aggregate being contiguous, is (1 - omega) sum_{u in I} b_u plus the sum,
// over every edge leaving a row of I, of w_e * omega / D_vv * b_v.
// Units are aggregates when RESTRICT, else rows.  xf: x is updated by the
// next product kernel instead (x = 0 on the first iteration, p not read, no
// sum-x partials).
template <typename T, int W, bool UPDATE, bool RESTRICT, int SPLIT>
__global__ __launch_bounds__(kBlock) void k_update_restrict(
    LevelArgs L, const T* __restrict__ r_in, const T* __restrict__ q, const T* __restrict__ p,
    T* __restrict__ x, T* __restrict__ r_out, T* __restrict__ bc, const double* __restrict__ scal,
    int first, double* __restrict__ part_rr, double* __restrict__ part_cs, int xf) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = Shape<W>::RG, WS = Shape<W>::WS;
  using D = Deco<W, SPLIT>;
  __shared__ double lds[UPDATE ? RG * WS : 1];
  __shared__ T ldc[SPLIT > 1 ? RG * WS : 1];
  int slice, rb, grb;
  slice_of_block<W>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const T* w = static_cast<const T*>(L.w);
  const T* sd = static_cast<const T*>(L.sd);
  const T om1 = T(1.0 - L.omega);
  T alpha[V];
  double rr[V], cs[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    alpha[i] = UPDATE ? T(scal[S_ALPHA * W + c0 + i]) : T(0);
    rr[i] = 0;
    cs[i] = 0;
  }
  const int units = RESTRICT ? L.nagg : L.n;
  int tb, te;
  block_tiles((units + D::PER_TILE - 1) / D::PER_TILE, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int I = D::unit(t, rg);
    const bool valid = I < units;
    T s[V];
#pragma unroll
    for (int i = 0; i < V; ++i) s[i] = 0;
    if (valid) {
      const int r0 = RESTRICT ? L.aggptr[I] : I;
      const int r1 = RESTRICT ? L.aggptr[I + 1] : I + 1;
      for (int u = r0 + D::split(rg); u < r1; u += SPLIT) {
        const size_t o = (size_t)u * W + c0;
        Vec<T, V> rn = ld<T, V>(r_in + o);
        if (UPDATE) {
          const Vec<T, V> qu = ld<T, V>(q + o);
          Vec<T, V> xu, pu;
          if (!xf) {
            pu = ld_nt<T, V>(p + o);
            if (!first) xu = ld_nt<T, V>(x + o);
          }
#pragma unroll
          for (int i = 0; i < V; ++i) {
            rn.v[i] -= alpha[i] * qu.v[i];
            if (xf)
              xu.v[i] = 0;
            else
              xu.v[i] = first ? alpha[i] * pu.v[i] : xu.v[i] + alpha[i] * pu.v[i];
            rr[i] += double(rn.v[i]) * double(rn.v[i]);
            cs[i] += double(xu.v[i]);
          }
          if (!xf || first) st_nt<T, V>(x + o, xu);
          st<T, V>(r_out + o, rn);
        }
#pragma unroll
        for (int i = 0; i < V; ++i) s[i] += om1 * rn.v[i];
        if (RESTRICT) add_heavy<T, W>(L, u, s, c0);
      }
      if (RESTRICT)
        gather_acc<T, W>(s, L.col, w, L.rowptr[r0], L.rowptr[r1], D::split(rg), SPLIT, [&](int v) {
          Vec<T, V> r = ld<T, V>(r_in + (size_t)v * W + c0);
          const T f = sd[v];
          if (UPDATE) {
            const Vec<T, V> qv = ld<T, V>(q + (size_t)v * W + c0);
#pragma unroll
            for (int i = 0; i < V; ++i) r.v[i] -= alpha[i] * qv.v[i];
          }
#pragma unroll
          for (int i = 0; i < V; ++i) r.v[i] *= f;
          return r;
        });
    }
    if (RESTRICT) {
      if constexpr (SPLIT > 1) wg_combine<T, W, SPLIT>(s, ldc);
      if (valid && D::leader(rg)) {
        Vec<T, V> sv;
#pragma unroll
        for (int i = 0; i < V; ++i) sv.v[i] = s[i];
        st<T, V>(bc + (size_t)I * W + c0, sv);
      }
    }
  }
  if (UPDATE) {
    block_store<W>(rr, lds, part_rr + (size_t)rb * W + slice * WS);
    if (!xf) block_store<W>(cs, lds, part_cs + (size_t)rb * W + slice * WS);
  }
}

// ---------------------------------------------------------------------------
// Prolongation + post-smoothing: xt = S b + mu xc[agg], x = xt + S (b - L xt).
template <typename T, int W, bool DOT, int SPLIT>
__global__ __launch_bounds__(kBlock) void k_prolong_smooth(LevelArgs L, const T* __restrict__ b,
                                                           const T* __restrict__ xc,
                                                           T* __restrict__ x,
                                                           double* __restrict__ part) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = Shape<W>::RG, WS = Shape<W>::WS;
  using D = Deco<W, SPLIT>;
  __shared__ double lds[DOT ? RG * WS : 1];
  __shared__ T ldc[SPLIT > 1 ? RG * WS : 1];
  int slice, rb, grb;
  slice_of_block<W>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const T* w = static_cast<const T*>(L.w);
  const T* sd = static_cast<const T*>(L.sd);
  const T* deg = static_cast<const T*>(L.deg);
  const T mu = T(L.mu);
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = 0;
  int tb, te;
  block_tiles((L.n + D::PER_TILE - 1) / D::PER_TILE, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = D::unit(t, rg);
    T nb[V];
#pragma unroll
    for (int i = 0; i < V; ++i) nb[i] = 0;
    if (u < L.n)
      gather_acc<T, W>(nb, L.col, w, L.rowptr[u], L.rowptr[u + 1], D::split(rg), SPLIT, [&](int v) {
        const T sv = sd[v];
        const Vec<T, V> bv = ld<T, V>(b + (size_t)v * W + c0);
        const Vec<T, V> xv = ld<T, V>(xc + (size_t)L.agg[v] * W + c0);
        Vec<T, V> r;
#pragma unroll
        for (int i = 0; i < V; ++i) r.v[i] = sv * bv.v[i] + mu * xv.v[i];
        return r;
      });
    if constexpr (SPLIT > 1) wg_combine<T, W, SPLIT>(nb, ldc);
    if (u < L.n && D::leader(rg)) {
      add_heavy<T, W>(L, u, nb, c0);
      const size_t o = (size_t)u * W + c0;
      const Vec<T, V> bu = ld<T, V>(b + o);
      const Vec<T, V> cu = ld<T, V>(xc + (size_t)L.agg[u] * W + c0);
      const T sdu = sd[u], du = deg[u];
      Vec<T, V> xo;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const T xt = sdu * bu.v[i] + mu * cu.v[i];
        const T lx = du * xt - nb[i];
        xo.v[i] = xt + sdu * (bu.v[i] - lx);
        if (DOT) acc[i] += double(bu.v[i]) * double(xo.v[i]);
      }
      st_nt<T, V>(x + o, xo);
    }
  }
  if (DOT) block_store<W>(acc, lds, part + (size_t)rb * W + slice * WS);
}

// ---------------------------------------------------------------------------
// Smoother-only "solve" on the deepest level a truncated V-cycle uses:
// x = S b (one Jacobi step from zero, S = omega D^-1); partial b.x if part.
// ZF = 1: x is stored as bfloat16 (bf16_t[n][W]), ZF = 2: as FP8 with
// per-row-slice scales; the partial uses the rounded values.
template <typename T, int W, bool DOT, int ZF, int NSX = slices_of(W)>
__global__ __launch_bounds__(kBlock) void k_jacobi(LevelArgs L, const T* __restrict__ b,
                                                   void* __restrict__ xv, double* __restrict__ part) {
  constexpr bool BF = ZF == 1;
  constexpr int LPR = Shape<W, NSX>::LPR, V = Shape<W, NSX>::V, RG = Shape<W, NSX>::RG, WS = Shape<W, NSX>::WS;
  __shared__ double lds[DOT ? RG * WS : 1];
  int slice, rb, grb;
  slice_of_block<W, NSX>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const T* sd = static_cast<const T*>(L.sd);
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = 0;
  int tb, te;
  block_tiles((L.n + RG - 1) / RG, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u >= L.n) continue;
    const size_t o = (size_t)u * W + c0;
    const Vec<T, V> bu = ld<T, V>(b + o);
    const T su = sd[u];
    Vec<T, V> xo;
    Vec<bf16_t, V> xh;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      xo.v[i] = su * bu.v[i];
      if constexpr (BF) {
        xh.v[i] = f2bf(float(xo.v[i]));
        xo.v[i] = T(bf2f(xh.v[i]));
      }
    }
    if constexpr (ZF == 2) {
      f8_t* x8 = static_cast<f8_t*>(xv);
      st_f8<T, W, NSX>(xo, x8 + o, reinterpret_cast<float*>(x8 + f8_scale_off(L.n, W)) +
                                  (size_t)u * Shape<W, NSX>::NS + slice);
    }
#pragma unroll
    for (int i = 0; i < V; ++i)
      if (DOT) acc[i] += double(bu.v[i]) * double(xo.v[i]);
    if constexpr (BF)
      st<bf16_t, V>(static_cast<bf16_t*>(xv) + o, xh);
    else if (ZF == 0 && xv)
      st<T, V>(static_cast<T*>(xv) + o, xo);
  }
  if (DOT) block_store<W, NSX>(acc, lds, part + (size_t)rb * W + slice * WS);
}

// Jacobi-preconditioned CG update on level 0 (a V-cycle of depth one):
// r_out = r_in - alpha q, x = (first ? 0 : x) + alpha p, z = S r_out;
// partials |r_out|^2, sum x, r_out . z.  ZF = 1: z is stored (non-null) as
// bfloat16, ZF = 2: as FP8 with per-row-slice scales; r_out . z uses the
// rounded z.  xf: x is updated by the
// product kernel of the next iteration instead (this kernel reads neither x
// nor p, writes x = 0 on the first iteration and no sum-x partials).
template <typename T, int W, int ZF, int NSX = slices_of(W)>
__global__ __launch_bounds__(kBlock) void k_update_jacobi(LevelArgs L, const T* __restrict__ r_in,
                                                          const T* __restrict__ q, const T* __restrict__ p,
                                                          T* __restrict__ x, T* __restrict__ r_out,
                                                          void* __restrict__ z, const double* __restrict__ scal,
                                                          int first, double* __restrict__ part_rr,
                                                          double* __restrict__ part_cs,
                                                          double* __restrict__ part_rz, int xf) {
  constexpr int LPR = Shape<W, NSX>::LPR, V = Shape<W, NSX>::V, RG = Shape<W, NSX>::RG, WS = Shape<W, NSX>::WS;
  constexpr bool BF = ZF == 1;
  __shared__ double lds[RG * WS];
  int slice, rb, grb;
  slice_of_block<W, NSX>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const T* sd = static_cast<const T*>(L.sd);
  T alpha[V];
  double rr[V], cs[V], rz[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    alpha[i] = T(scal[S_ALPHA * W + c0 + i]);
    rr[i] = cs[i] = rz[i] = 0;
  }
  int tb, te;
  block_tiles((L.n + RG - 1) / RG, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u >= L.n) continue;
    const size_t o = (size_t)u * W + c0;
    Vec<T, V> rn = ld_nt<T, V>(r_in + o);
    const Vec<T, V> qu = ld_nt<T, V>(q + o);
    Vec<T, V> xu, zu, pu;
    Vec<bf16_t, V> zh;
    if (!xf) {
      pu = ld_nt<T, V>(p + o);
      if (!first) xu = ld_nt<T, V>(x + o);
    }
    const T su = sd[u];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      rn.v[i] -= alpha[i] * qu.v[i];
      if (xf)
        xu.v[i] = 0;
      else
        xu.v[i] = first ? alpha[i] * pu.v[i] : xu.v[i] + alpha[i] * pu.v[i];
      zu.v[i] = su * rn.v[i];
      if constexpr (BF) {
        zh.v[i] = f2bf(float(zu.v[i]));
        zu.v[i] = T(bf2f(zh.v[i]));
      }
    }
    if constexpr (ZF == 2) {
      f8_t* z8 = static_cast<f8_t*>(z);
      st_f8<T, W, NSX>(zu, z8 + o, reinterpret_cast<float*>(z8 + f8_scale_off(L.n, W)) +
                                  (size_t)u * Shape<W, NSX>::NS + slice);
    }
#pragma unroll
    for (int i = 0; i < V; ++i) {
      rr[i] += double(rn.v[i]) * double(rn.v[i]);
      cs[i] += double(xu.v[i]);
      rz[i] += double(rn.v[i]) * double(zu.v[i]);
    }
    if (!xf || first) st_nt<T, V>(x + o, xu);
    st_nt<T, V>(r_out + o, rn);
    if constexpr (BF)
      st<bf16_t, V>(static_cast<bf16_t*>(z) + o, zh);
    else if (ZF == 0 && z)
      st<T, V>(static_cast<T*>(z) + o, zu);
  }
  block_store<W, NSX>(rr, lds, part_rr + (size_t)rb * W + slice * WS);
  if (!xf) block_store<W, NSX>(cs, lds, part_cs + (size_t)rb * W + slice * WS);
  block_store<W, NSX>(rz, lds, part_rz + (size_t)rb * W + slice * WS);
}

// Last CG update of x when the product kernel carries the x updates:
// x += alpha p; partial column sums of x.
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_xfinal(int n, T* __restrict__ x, const T* __restrict__ p,
                                                   const double* __restrict__ scal,
                                                   double* __restrict__ part_cs) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = Shape<W>::RG, WS = Shape<W>::WS;
  __shared__ double lds[RG * WS];
  int slice, rb, grb;
  slice_of_block<W>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  T alpha[V];
  double cs[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    alpha[i] = T(scal[S_ALPHA * W + c0 + i]);
    cs[i] = 0;
  }
  int tb, te;
  block_tiles((n + RG - 1) / RG, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u >= n) continue;
    const size_t o = (size_t)u * W + c0;
    Vec<T, V> xu = ld_nt<T, V>(x + o);
    const Vec<T, V> pu = ld_nt<T, V>(p + o);
#pragma unroll
    for (int i = 0; i < V; ++i) {
      xu.v[i] += alpha[i] * pu.v[i];
      cs[i] += double(xu.v[i]);
    }
    st_nt<T, V>(x + o, xu);
  }
  block_store<W>(cs, lds, part_cs + (size_t)rb * W + slice * WS);
}

// ---------------------------------------------------------------------------
// Coarsest level: x = Lc^+ b with FP64 MFMA (16x16x4 tiles, one per wave).
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T, int W>
__global__ __launch_bounds__(256) void k_coarse_mfma(int nc, int ncp, const double* __restrict__ A,
                                                     const T* __restrict__ b, T* __restrict__ x) {
  const int wave = blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  constexpr int NTC = W / 16;
  const int tr = wave / NTC, tc = wave % NTC;
  if (tr * 16 >= ncp) return;
  const int i0 = tr * 16, j0 = tc * 16;
  // operand layout of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l holds
  // A[l%16][l/16] and B[l/16][l%16]; result register r of lane l is
  // D[l/16 + 4r][l%16].
  const int ar = i0 + (lane & 15), kk = lane >> 4, bj = j0 + (lane & 15);
  const double* Ar = A + (size_t)ar * ncp + kk;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < ncp; k0 += 4) {
    const double a = Ar[k0];
    const int k = k0 + kk;
    const double bb = k < nc ? double(b[(size_t)k * W + bj]) : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = i0 + (lane >> 4) + 4 * r;
    if (row < nc) x[(size_t)row * W + bj] = T(acc[r]);
  }
}

// Narrow blocks (W < 16): one thread per output element.
template <typename T, int W>
__global__ __launch_bounds__(256) void k_coarse_simple(int nc, int ncp, const double* __restrict__ A,
                                                       const T* __restrict__ b, T* __restrict__ x) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nc * W) return;
  const int i = id / W, j = id % W;
  double s = 0;
  for (int k = 0; k < nc; ++k) s += A[(size_t)i * ncp + k] * double(b[(size_t)k * W + j]);
  x[(size_t)i * W + j] = T(s);
}

// Partial column dots a.b over rows.
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_dot(int n, const T* __restrict__ a, const T* __restrict__ b,
                                                double* __restrict__ part) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = Shape<W>::RG, WS = Shape<W>::WS;
  __shared__ double lds[RG * WS];
  int slice, rb, grb;
  slice_of_block<W>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = 0;
  int tb, te;
  block_tiles((n + RG - 1) / RG, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u >= n) continue;
    const Vec<T, V> x = ld<T, V>(a + (size_t)u * W + c0);
    const Vec<T, V> y = b ? ld<T, V>(b + (size_t)u * W + c0) : Vec<T, V>{};
#pragma unroll
    for (int i = 0; i < V; ++i) acc[i] += b ? double(x.v[i]) * double(y.v[i]) : double(x.v[i]);
  }
  block_store<W>(acc, lds, part + (size_t)rb * W + slice * WS);
}

// ---------------------------------------------------------------------------
// FP64 residual r = b - L x (Eq. 1), stored as TO; partial |r|^2 (FP64).
// x is FP64, or (TX = float) an FP32 block whose values the FP64 arithmetic
// takes exactly.
template <typename TX, int V>
__device__ __forceinline__ Vec<double, V> ld_f64(const TX* p) {
  if constexpr (sizeof(TX) == 8) {
    return ld<double, V>(p);
  } else {
    const Vec<TX, V> f = ld<TX, V>(p);
    Vec<double, V> r;
#pragma unroll
    for (int i = 0; i < V; ++i) r.v[i] = double(f.v[i]);
    return r;
  }
}

template <typename TO, int W, typename TX, int SPLIT>
__global__ __launch_bounds__(kBlock) void k_residual64(LevelArgs L, const TX* __restrict__ x,
                                                       RhsArgs rhs, TO* r_out,
                                                       double* __restrict__ part) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = Shape<W>::RG, WS = Shape<W>::WS;
  using D = Deco<W, SPLIT>;
  __shared__ double lds[RG * WS];
  __shared__ double ldc[SPLIT > 1 ? RG * WS : 1];
  int slice, rb, grb;
  slice_of_block<W>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const double* w = static_cast<const double*>(L.w);
  const double* deg = static_cast<const double*>(L.deg);
  int ps[V], pt[V];
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    ps[i] = rhs.kind == 1 ? rhs.ps[c0 + i] : -1;
    pt[i] = rhs.kind == 1 ? rhs.pt[c0 + i] : -1;
    acc[i] = 0;
  }
  int tb, te;
  block_tiles((L.n + D::PER_TILE - 1) / D::PER_TILE, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = D::unit(t, rg);
    double nb[V];
#pragma unroll
    for (int i = 0; i < V; ++i) nb[i] = 0;
    if (x && u < L.n)
      gather_acc<double, W>(nb, L.col, w, L.rowptr[u], L.rowptr[u + 1], D::split(rg), SPLIT,
                            [&](int v) { return ld_f64<TX, V>(x + (size_t)v * W + c0); });
    if constexpr (SPLIT > 1) wg_combine<double, W, SPLIT>(nb, ldc);
    if (u < L.n && D::leader(rg)) {
      if (x) add_heavy<double, W>(L, u, nb, c0);
      const size_t o = (size_t)u * W + c0;
      double a[V];
      if (x) {
        const Vec<double, V> xu = ld_f64<TX, V>(x + o);
        const double du = deg[u];
#pragma unroll
        for (int i = 0; i < V; ++i) a[i] = du * xu.v[i] - nb[i];
      } else {
#pragma unroll
        for (int i = 0; i < V; ++i) a[i] = 0;
      }
      double bv[V];
      if (rhs.kind == 0) {
        const Vec<double, V> bb = ld_nt<double, V>(rhs.dense + o);
#pragma unroll
        for (int i = 0; i < V; ++i) bv[i] = bb.v[i];
      } else if (rhs.kind == 2) {
        const Vec<float, V> bb = ld_nt<float, V>(rhs.dense32 + o);
#pragma unroll
        for (int i = 0; i < V; ++i) bv[i] = double(bb.v[i]);
      } else {
#pragma unroll
        for (int i = 0; i < V; ++i) bv[i] = (u == ps[i] ? 1.0 : 0.0) - (u == pt[i] ? 1.0 : 0.0);
      }
      Vec<TO, V> ro;
      Vec<double, V> r64;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const double r = bv[i] - a[i];
        r64.v[i] = r;
        ro.v[i] = TO(r);
        acc[i] += r * r;
      }
      st_nt<TO, V>(r_out + o, ro);
      if (rhs.r64_out) st_nt<double, V>(rhs.r64_out + o, r64);
    }
  }
  block_store<W>(acc, lds, part + (size_t)rb * W + slice * WS);
}

// x64 = (first ? 0 : x64) + d - mean(d), mean(d) = cs / n.
template <typename TI, int W>
__global__ __launch_bounds__(kBlock) void k_xupdate64(int n, double* __restrict__ x64,
                                                      const TI* __restrict__ d,
                                                      const double* __restrict__ scal, int first) {
  const size_t total = (size_t)n * W;
  const double inv = 1.0 / double(n);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int c = int(i % W);
    const double m = scal[S_CS * W + c] * inv;
    x64[i] = (first ? 0.0 : x64[i]) + double(d[i]) - m;
  }
}

// ---------------------------------------------------------------------------
// Projection right-hand sides (Sec. 5.2, Algorithm 1): column j of the block
// is system i = i0 + j, y_i[u] = sum over edges {u,v} of B(e,u) q_i(e) sqrt(w_e)
// with B(e, lo) = +1, B(e, hi) = -1 and q_i(e) = +-1/sqrt(k) from the sign
// word of (seed, i/64, lo, hi), bit i%64 (set = -1), keyed on graph ids.
// r (nullable): the same values in the inner precision TO, with partial sums
// of y^2 (the refinement's first residual, r = y, and its norms).
template <typename TO, int W>
__global__ __launch_bounds__(kBlock) void k_jl_rhs(LevelArgs L, const int* __restrict__ iperm,
                                                   uint64_t seed, int64_t i0, int64_t k,
                                                   double* __restrict__ Y, TO* __restrict__ r,
                                                   double* __restrict__ part) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = Shape<W>::RG, WS = Shape<W>::WS;
  __shared__ double lds[RG * WS];
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = 0;
  int slice, rb, grb;
  slice_of_block<W>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const double* w = static_cast<const double*>(L.w);
  const double inv_sqrt_k = 1.0 / sqrt(double(k));
  const int64_t sys0 = i0 + c0;
  const uint64_t word = uint64_t(sys0) >> 6;
  int tb, te;
  block_tiles((L.n + RG - 1) / RG, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u >= L.n) continue;
    const uint64_t gu = uint64_t(iperm[u]);
    double a[V];
#pragma unroll
    for (int i = 0; i < V; ++i) a[i] = 0;
    const int hh = L.heavy ? L.heavy[u] : -1;
    const int e0 = hh >= 0 ? L.hptr[hh] : L.rowptr[u];
    const int e1 = hh >= 0 ? L.hptr[hh + 1] : L.rowptr[u + 1];
    const int* cl = hh >= 0 ? L.hcol : L.col;
    const double* wl = hh >= 0 ? static_cast<const double*>(L.hw) : w;
    // The row group's columns lie in one 64-column sign word (WS divides 64
    // and every slice starts on a multiple of WS), so lane j hashes edge
    // eb + j once and the group shares the words through shuffles.
    const int lane = threadIdx.x % LPR;
    for (int eb = e0; eb < e1; eb += LPR) {
      const int e = eb + lane;
      uint64_t h = 0;
      double sg = 0;
      if (e < e1) {
        const uint64_t gv = uint64_t(iperm[cl[e]]);
        const uint64_t lo = gu < gv ? gu : gv, hi = gu < gv ? gv : gu;
        const double sw = wl ? sqrt(wl[e]) : 1.0;
        sg = gu < gv ? sw : -sw;
        h = jl_word(seed, word, lo, hi);
      }
      const unsigned hl = (unsigned)h, hu = (unsigned)(h >> 32);
      const int cnt = min(LPR, e1 - eb);
      for (int j = 0; j < cnt; ++j) {
        const uint64_t hj = ((uint64_t)(unsigned)__shfl((int)hu, j, LPR) << 32) |
                            (uint64_t)(unsigned)__shfl((int)hl, j, LPR);
        const double sgj = __shfl(sg, j, LPR);
#pragma unroll
        for (int i = 0; i < V; ++i) {
          const int bit = int((hj >> ((sys0 + i) & 63)) & 1u);
          a[i] += bit ? -sgj : sgj;
        }
      }
    }
    Vec<double, V> yo;
#pragma unroll
    for (int i = 0; i < V; ++i) yo.v[i] = (sys0 + i < k) ? a[i] * inv_sqrt_k : 0.0;
    st<double, V>(Y + (size_t)u * W + c0, yo);
    if (r) {
      Vec<TO, V> ro;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        ro.v[i] = TO(yo.v[i]);
        acc[i] += yo.v[i] * yo.v[i];
      }
      st_nt<TO, V>(r + (size_t)u * W + c0, ro);
    }
  }
  if (r) block_store<W>(acc, lds, part + (size_t)rb * W + slice * WS);
}

// Whole-row shape (no column slicing) for per-row reductions over all W columns.
template <int W> struct RowShape {
  static constexpr int V = W >= 512 ? W / 64 : (W >= 4 ? 4 : 1);
  static constexpr int LPR = W / V;
  static constexpr int RG = kBlock / LPR;
};

// N[u] += |x_u|^2 over the first ncols columns.
template <int W>
__global__ __launch_bounds__(kBlock) void k_jl_rownorm(int n, const double* __restrict__ x, int ncols,
                                                       double* __restrict__ N) {
  constexpr int LPR = RowShape<W>::LPR, V = RowShape<W>::V, RG = RowShape<W>::RG;
  const int rg = threadIdx.x / LPR, lane = threadIdx.x % LPR, c0 = lane * V;
  int tb, te;
  block_tiles((n + RG - 1) / RG, blockIdx.x, gridDim.x, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    const bool ok = u < n;
    double s = 0;
    if (ok) {
      const Vec<double, V> xu = ld<double, V>(x + (size_t)u * W + c0);
#pragma unroll
      for (int i = 0; i < V; ++i)
        if (c0 + i < ncols) s += xu.v[i] * xu.v[i];
    }
    for (int off = LPR / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, LPR);
    if (ok && lane == 0) N[u] += s;
  }
}

// ---------------------------------------------------------------------------
// Elimination level (LAMG's elimination stage): with the kept rows C first
// and the eliminated rows F an independent set, L = [L_CC L_CF; L_FC D_F]
// and one exact block step of the preconditioner is
//   forward  t_C = r_C - L_CF D_F^-1 r_F      (t_c = r_c + sum_f w_cf / d_f r_f)
//   coarse   z_C = M_S^-1 t_C                  (M_S: the cycle on the Schur
//                                               complement, the next level)
//   back     z_F = D_F^-1 (r_F - L_FC z_C)     (z_f = (r_f + sum_c w_fc z_c) / d_f)
// which is symmetric whenever M_S is.

// t = r + F r over the kept rows (F = the forward operator); with JAC the
// next level is smoothed once in place: out = sd1 * t, partial sums r . out;
// without JAC, partial sums t . t when part is given.  BF (with JAC): out is
// stored as bfloat16 and the partials use the rounded values.
template <typename T, int W, bool JAC, bool BF>
__global__ __launch_bounds__(kBlock) void k_elim_fwd(LevelArgs F, const T* __restrict__ r,
                                                     void* __restrict__ out, const T* __restrict__ sd1,
                                                     double* __restrict__ part) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = Shape<W>::RG, WS = Shape<W>::WS;
  __shared__ double lds[RG * WS];
  int slice, rb, grb;
  slice_of_block<W>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const T* w = static_cast<const T*>(F.w);
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = 0;
  int tb, te;
  block_tiles((F.n + RG - 1) / RG, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u >= F.n) continue;
    T nb[V];
#pragma unroll
    for (int i = 0; i < V; ++i) nb[i] = 0;
    gather_acc<T, W>(nb, F.col, w, F.rowptr[u], F.rowptr[u + 1], 0, 1,
                     [&](int v) { return ld<T, V>(r + (size_t)v * W + c0); });
    add_heavy<T, W>(F, u, nb, c0);
    const size_t o = (size_t)u * W + c0;
    const Vec<T, V> ru = ld<T, V>(r + o);
    Vec<T, V> ov;
    Vec<bf16_t, V> oh;
    if constexpr (JAC) {
      const T su = sd1[u];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        ov.v[i] = su * (ru.v[i] + nb[i]);
        if constexpr (BF) {
          oh.v[i] = f2bf(float(ov.v[i]));
          ov.v[i] = T(bf2f(oh.v[i]));
        }
        acc[i] += double(ru.v[i]) * double(ov.v[i]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) {
        ov.v[i] = ru.v[i] + nb[i];
        acc[i] += double(ov.v[i]) * double(ov.v[i]);
      }
    }
    if constexpr (BF)
      st<bf16_t, V>(static_cast<bf16_t*>(out) + o, oh);
    else
      st<T, V>(static_cast<T*>(out) + o, ov);
  }
  if (JAC || part) block_store<W>(acc, lds, part + (size_t)rb * W + slice * WS);
}

// z_f for the eliminated rows, then partial sums of r . z over the eliminated
// rows (ALL = false) or over every row (ALL = true).  BF: z is held as
// bfloat16 (the kept rows' z_c read as stored, z_f rounded when stored and
// in the partials).
template <typename T, int W, bool ALL, bool BF>
__global__ __launch_bounds__(kBlock) void k_elim_back(LevelArgs L, const T* __restrict__ r,
                                                      void* __restrict__ zv, double* __restrict__ part) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = Shape<W>::RG, WS = Shape<W>::WS;
  __shared__ double lds[RG * WS];
  int slice, rb, grb;
  slice_of_block<W>(slice, rb, grb);
  const int rg = threadIdx.x / LPR, c0 = slice * WS + (threadIdx.x % LPR) * V;
  const T* ew = static_cast<const T*>(L.ew);
  const T* einv = static_cast<const T*>(L.einv);
  T* z = static_cast<T*>(zv);
  bf16_t* zh = static_cast<bf16_t*>(zv);
  auto zrow = [&](int a) {
    if constexpr (BF)
      return ld_bf<T, V>(zh + (size_t)a * W + c0);
    else
      return ld<T, V>(z + (size_t)a * W + c0);
  };
  const int base = ALL ? 0 : L.nC;
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = 0;
  int tb, te;
  block_tiles((L.n - base + RG - 1) / RG, rb, grb, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = base + t * RG + rg;
    if (u >= L.n) continue;
    const size_t o = (size_t)u * W + c0;
    const Vec<T, V> ru = ld<T, V>(r + o);
    Vec<T, V> zu;
    if (u >= L.nC) {
      const int i = u - L.nC;
      const int4 nb = reinterpret_cast<const int4*>(L.enb)[i];
      const int a[kElimDeg] = {nb.x, nb.y, nb.z, nb.w};
      const T di = einv[i];
      zu = ru;
#pragma unroll
      for (int j = 0; j < kElimDeg; ++j) {
        if (a[j] < 0) break;  // neighbours first, then -1
        const T wa = ew[kElimDeg * i + j];
        const Vec<T, V> za = zrow(a[j]);
#pragma unroll
        for (int k = 0; k < V; ++k) zu.v[k] += wa * za.v[k];
      }
#pragma unroll
      for (int k = 0; k < V; ++k) zu.v[k] *= di;
      if constexpr (BF) {
        Vec<bf16_t, V> h;
#pragma unroll
        for (int k = 0; k < V; ++k) {
          h.v[k] = f2bf(float(zu.v[k]));
          zu.v[k] = T(bf2f(h.v[k]));
        }
        st<bf16_t, V>(zh + o, h);
      } else {
        st<T, V>(z + o, zu);
      }
    } else {
      zu = zrow(u);
    }
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] += double(ru.v[k]) * double(zu.v[k]);
  }
  block_store<W>(acc, lds, part + (size_t)rb * W + slice * WS);
}

// ---------------------------------------------------------------------------
// Electrical currents of a block of unit s_j -> t_j flows (Sec. 2): column j
// of the FP64 block x holds potentials with L x_j = e_{s_j} - e_{t_j}, so
// edge {u, v} carries w_uv (x_u[j] - x_v[j]).  The throughput of node u in
// flow j is half the absolute current over its edges, counted only when u is
// neither s_j nor t_j.  One row group per row (or heavy-row segment), lanes
// across the columns; the lane sum over columns is reduced across the row
// group, so each row's total is written by one lane in a fixed order.

// sum over edges e0..e1 of w_e |x_u - x_col(e)| per column (4 rows in flight)
template <int W>
__device__ __forceinline__ void tp_lane(const double* __restrict__ x, const int* __restrict__ col,
                                        const double* __restrict__ w, int e0, int e1, int c0,
                                        const Vec<double, RowShape<W>::V>& xu,
                                        double (&acc)[RowShape<W>::V]) {
  constexpr int V = RowShape<W>::V;
  int e = e0;
  for (; e + 4 <= e1; e += 4) {
    Vec<double, V> xv[4];
    double we[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      xv[k] = ld<double, V>(x + (size_t)col[e + k] * W + c0);
      we[k] = w ? w[e + k] : 1.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] += we[k] * fabs(xu.v[i] - xv[k].v[i]);
  }
  for (; e < e1; ++e) {
    const Vec<double, V> xv = ld<double, V>(x + (size_t)col[e] * W + c0);
    const double we = w ? w[e] : 1.0;
#pragma unroll
    for (int i = 0; i < V; ++i) acc[i] += we * fabs(xu.v[i] - xv.v[i]);
  }
}

// lane sum over the columns that count for row u
template <int W>
__device__ __forceinline__ double tp_masked(int u, const double (&acc)[RowShape<W>::V],
                                            const int (&ps)[RowShape<W>::V],
                                            const int (&pt)[RowShape<W>::V]) {
  double s = 0;
#pragma unroll
  for (int i = 0; i < RowShape<W>::V; ++i)
    if (ps[i] >= 0 && u != ps[i] && u != pt[i]) s += acc[i];
  return s;
}

template <int W>
__device__ __forceinline__ void tp_pairs(const int* __restrict__ ps, const int* __restrict__ pt,
                                         int ncols, int c0, int (&a)[RowShape<W>::V],
                                         int (&b)[RowShape<W>::V]) {
#pragma unroll
  for (int i = 0; i < RowShape<W>::V; ++i) {
    const bool ok = c0 + i < ncols;
    a[i] = ok ? ps[c0 + i] : -1;
    b[i] = ok ? pt[c0 + i] : -1;
  }
}

// heavy rows: seg_part[seg] = lane-and-column sum over the segment's edges.
// A whole workgroup takes one segment (its RG row groups split the edges),
// since the few long rows would otherwise leave most of the chip idle.
template <int W>
__global__ __launch_bounds__(kBlock) void k_tp_seg(LevelArgs L, const double* __restrict__ x,
                                                   int ncols, const int* __restrict__ ps,
                                                   const int* __restrict__ pt,
                                                   double* __restrict__ seg_part) {
  constexpr int LPR = RowShape<W>::LPR, V = RowShape<W>::V, RG = RowShape<W>::RG;
  __shared__ double red[RG];
  const int rg = threadIdx.x / LPR, lane = threadIdx.x % LPR, c0 = lane * V;
  int a[V], b[V];
  tp_pairs<W>(ps, pt, ncols, c0, a, b);
  const double* hw = static_cast<const double*>(L.hw);
  for (int sg = blockIdx.x; sg < L.nseg; sg += gridDim.x) {
    const int u = L.seg_row[sg];
    const int e0 = L.seg_e[sg], e1 = L.seg_e[sg + 1];
    const int len = e1 - e0, per = (len + RG - 1) / RG;
    const int f0 = e0 + min(len, rg * per), f1 = e0 + min(len, (rg + 1) * per);
    const Vec<double, V> xu = ld<double, V>(x + (size_t)u * W + c0);
    double acc[V];
#pragma unroll
    for (int i = 0; i < V; ++i) acc[i] = 0;
    tp_lane<W>(x, L.hcol, hw, f0, f1, c0, xu, acc);
    double s = tp_masked<W>(u, acc, a, b);
    for (int off = LPR / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, LPR);
    if (lane == 0) red[rg] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0;
      for (int i = 0; i < RG; ++i) t += red[i];
      seg_part[sg] = t;
    }
    __syncthreads();
  }
}

// tp[u] += throughput of row u summed over the block's flows
template <int W>
__global__ __launch_bounds__(kBlock) void k_tp_rows(LevelArgs L, const double* __restrict__ x,
                                                    int ncols, const int* __restrict__ ps,
                                                    const int* __restrict__ pt,
                                                    const double* __restrict__ seg_part,
                                                    double* __restrict__ tp) {
  constexpr int LPR = RowShape<W>::LPR, V = RowShape<W>::V, RG = RowShape<W>::RG;
  const int rg = threadIdx.x / LPR, lane = threadIdx.x % LPR, c0 = lane * V;
  int a[V], b[V];
  tp_pairs<W>(ps, pt, ncols, c0, a, b);
  const double* w = static_cast<const double*>(L.w);
  int tb, te;
  block_tiles((L.n + RG - 1) / RG, blockIdx.x, gridDim.x, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    const bool ok = u < L.n;
    const int hh = ok && L.heavy ? L.heavy[u] : -1;
    double s = 0;
    if (ok && hh < 0) {
      const Vec<double, V> xu = ld<double, V>(x + (size_t)u * W + c0);
      double acc[V];
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] = 0;
      tp_lane<W>(x, L.col, w, L.rowptr[u], L.rowptr[u + 1], c0, xu, acc);
      s = tp_masked<W>(u, acc, a, b);
    }
    for (int off = LPR / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, LPR);
    if (ok && lane == 0) {
      if (hh >= 0)
        for (int sg = L.hseg[hh]; sg < L.hseg[hh + 1]; ++sg) s += seg_part[sg];
      tp[u] += 0.5 * s;
    }
  }
}

// out[i] += sum over the first ncols columns of (x_{a_i} - x_{b_i})^2: the
// squared sketch distance of Sec. 5.2 between the endpoints of edge i.
template <int W>
__global__ __launch_bounds__(kBlock) void k_edge_sq(int ne, const int* __restrict__ ea,
                                                    const int* __restrict__ eb,
                                                    const double* __restrict__ x, int ncols,
                                                    double* __restrict__ out) {
  constexpr int LPR = RowShape<W>::LPR, V = RowShape<W>::V, RG = RowShape<W>::RG;
  const int rg = threadIdx.x / LPR, lane = threadIdx.x % LPR, c0 = lane * V;
  int tb, te;
  block_tiles((ne + RG - 1) / RG, blockIdx.x, gridDim.x, tb, te);
  for (int t = tb; t < te; ++t) {
    const int i = t * RG + rg;
    const bool ok = i < ne;
    double s = 0;
    if (ok) {
      const Vec<double, V> xa = ld<double, V>(x + (size_t)ea[i] * W + c0);
      const Vec<double, V> xb = ld<double, V>(x + (size_t)eb[i] * W + c0);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const double d = xa.v[k] - xb.v[k];
        if (c0 + k < ncols) s += d * d;
      }
    }
    for (int off = LPR / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, LPR);
    if (ok && lane == 0) out[i] += s;
  }
}

// ---------------------------------------------------------------------------
// host launchers
inline int grid_units(int units, int rg) { return grid_for(units, rg); }

template <typename T, int W>
struct Launch {
  static constexpr int RG = Shape<W>::RG;
  static constexpr int NS = Shape<W>::NS;
  // The kernels that write or gather z in FP8 use half as many column
  // slices (128 columns from W = 256), so that a gathered FP8 slice row is
  // 128 bytes, as a bfloat16 one is with the regular slicing.
  static constexpr int NS8 = NS >= 2 ? NS / 2 : 1;
  static constexpr int RG8 = Shape<W, NS8>::RG;

  // workgroups per slice for a kernel over `units` units of level L
  static int rows_grid(const LevelArgs& L, int units) {
    return grid_for(units, RG / std::min(std::max(L.split, 1), RG));
  }
  // the same for the FP8 product (row splits of at most 4)
  static int rows_grid8(const LevelArgs& L, int units) {
    return grid_for(units, RG8 / (L.split >= 4 ? 4 : 1), NS / NS8);
  }

#define CFC_LAUNCH(K, units, ...)                                                              \
  do {                                                                                         \
    const int g_ = rows_grid(L, units);                                                        \
    if (!g_) return;                                                                           \
    const int sp_ = std::min(std::max(L.split, 1), RG);                                        \
    if (sp_ >= 16)                                                                             \
      hipLaunchKernelGGL((K<__VA_ARGS__, 16>), dim3(g_ * NS), dim3(kBlock), 0, s, ARGS);       \
    else if (sp_ >= 4)                                                                         \
      hipLaunchKernelGGL((K<__VA_ARGS__, 4>), dim3(g_ * NS), dim3(kBlock), 0, s, ARGS);        \
    else                                                                                       \
      hipLaunchKernelGGL((K<__VA_ARGS__, 1>), dim3(g_ * NS), dim3(kBlock), 0, s, ARGS);        \
  } while (0)

  // the per-row sums of the segment partials (when the level has hsum)
  template <typename TT>
  static void heavy_sum(const LevelArgs& L, hipStream_t s) {
    if (!L.nseg || !L.hsum) return;
    const int g = std::min((L.nheavy + RG - 1) / RG, kMaxGrid);
    hipLaunchKernelGGL((k_heavy_sum<TT, W>), dim3(g * NS), dim3(kBlock), 0, s, L);
  }
  template <int KIND>
  static void heavy(const LevelArgs& L, const void* a, const void* q, const void* xc,
                    const double* scal, hipStream_t s) {
    if (!L.nseg) return;
    const int g = std::min(L.nseg, 4 * kMaxGrid);
    hipLaunchKernelGGL((k_heavy<T, W, KIND>), dim3(g * NS), dim3(kBlock), 0, s, L, (const T*)a,
                       (const T*)q, (const T*)xc, scal);
    heavy_sum<T>(L, s);
  }

  static void spmm_pq(const LevelArgs& L, const void* z, void* p, void* q, void* x,
                      const double* scal, int first, double* part, int jac, hipStream_t s) {
#define ARGS L, (const T*)z, (T*)p, (T*)q, (T*)x, scal, first, part
    if (jac == 3) {
      if (L.nseg) {
        const int gh = std::min(L.nseg, 4 * kMaxGrid);
        hipLaunchKernelGGL((k_heavy<T, W, HK_F8, NS8>), dim3(gh * NS8), dim3(kBlock), 0, s, L,
                           (const T*)z, (const T*)nullptr, (const T*)nullptr, scal);
        heavy_sum<T>(L, s);
      }
      const int g8 = rows_grid8(L, L.n);
      if (!g8) return;
      if (L.split >= 4)
        hipLaunchKernelGGL((k_spmm_pq<T, W, 3, 4, NS8>), dim3(g8 * NS8), dim3(kBlock), 0, s, ARGS);
      else
        hipLaunchKernelGGL((k_spmm_pq<T, W, 3, 1, NS8>), dim3(g8 * NS8), dim3(kBlock), 0, s, ARGS);
    } else if (jac == 2) {
      heavy<HK_BF16>(L, z, nullptr, nullptr, scal, s);
      CFC_LAUNCH(k_spmm_pq, L.n, T, W, 2);
    } else if (jac) {
      heavy<HK_RESTRICT>(L, z, nullptr, nullptr, scal, s);  // sum of w_e sd_v r_v
      CFC_LAUNCH(k_spmm_pq, L.n, T, W, 1);
    } else {
      heavy<HK_SPMM>(L, z, nullptr, nullptr, scal, s);
      CFC_LAUNCH(k_spmm_pq, L.n, T, W, 0);
    }
#undef ARGS
  }
  static void update_restrict(const LevelArgs& L, const void* r_in, const void* q, const void* p,
                              void* x, void* r_out, void* bc, const double* scal, int first,
                              int do_update, double* prr, double* pcs, int xf, hipStream_t s) {
    const bool R = L.nagg > 0;
    if (R && do_update) heavy<HK_RESTRICT_UPD>(L, r_in, q, nullptr, scal, s);
    else if (R) heavy<HK_RESTRICT>(L, r_in, nullptr, nullptr, scal, s);
#define ARGS L, (const T*)r_in, (const T*)q, (const T*)p, (T*)x, (T*)r_out, (T*)bc, scal, first, prr, pcs, xf
    if (do_update && R)
      CFC_LAUNCH(k_update_restrict, L.nagg, T, W, true, true);
    else if (do_update)
      CFC_LAUNCH(k_update_restrict, L.n, T, W, true, false);
    else if (R)
      CFC_LAUNCH(k_update_restrict, L.nagg, T, W, false, true);
#undef ARGS
  }
  static void restrict_(const LevelArgs& L, const void* b, void* bc, hipStream_t s) {
    heavy<HK_RESTRICT>(L, b, nullptr, nullptr, nullptr, s);
#define ARGS L, (const T*)b, (const T*)nullptr, (const T*)nullptr, (T*)nullptr, (T*)nullptr, (T*)bc, \
             (const double*)nullptr, 0, (double*)nullptr, (double*)nullptr, 0
    CFC_LAUNCH(k_update_restrict, L.nagg, T, W, false, true);
#undef ARGS
  }
  static void prolong_smooth(const LevelArgs& L, const void* b, const void* xc, void* x,
                             double* part, hipStream_t s) {
    heavy<HK_PROLONG>(L, b, nullptr, xc, nullptr, s);
#define ARGS L, (const T*)b, (const T*)xc, (T*)x, part
    if (part)
      CFC_LAUNCH(k_prolong_smooth, L.n, T, W, true);
    else
      CFC_LAUNCH(k_prolong_smooth, L.n, T, W, false);
#undef ARGS
  }
  static void jacobi(const LevelArgs& L, const void* b, void* x, double* part, int zf, hipStream_t s) {
    const int g = grid_units(L.n, RG);
    if (!g) return;
    if (zf == 2 && part)
      hipLaunchKernelGGL((k_jacobi<T, W, true, 2, NS8>), dim3(grid_for(L.n, RG8, NS / NS8) * NS8), dim3(kBlock),
                         0, s, L, (const T*)b, x, part);
    else if (zf && part)
      hipLaunchKernelGGL((k_jacobi<T, W, true, 1>), dim3(g * NS), dim3(kBlock), 0, s, L,
                         (const T*)b, x, part);
    else if (part)
      hipLaunchKernelGGL((k_jacobi<T, W, true, 0>), dim3(g * NS), dim3(kBlock), 0, s, L,
                         (const T*)b, x, part);
    else
      hipLaunchKernelGGL((k_jacobi<T, W, false, 0>), dim3(g * NS), dim3(kBlock), 0, s, L,
                         (const T*)b, x, part);
  }
  static void update_jacobi(const LevelArgs& L, const void* r_in, const void* q, const void* p,
                            void* x, void* r_out, void* z, const double* scal, int first,
                            double* prr, double* pcs, double* prz, int zf, int xf, hipStream_t s) {
    const int g = grid_units(L.n, RG);
    if (!g) return;
#define UJ(ZF)                                                                                       \
  hipLaunchKernelGGL((k_update_jacobi<T, W, ZF>), dim3(g * NS), dim3(kBlock), 0, s, L, (const T*)r_in, \
                     (const T*)q, (const T*)p, (T*)x, (T*)r_out, z, scal, first, prr, pcs, prz, xf)
    if (zf == 2)
      hipLaunchKernelGGL((k_update_jacobi<T, W, 2, NS8>), dim3(grid_for(L.n, RG8, NS / NS8) * NS8), dim3(kBlock),
                         0, s, L, (const T*)r_in, (const T*)q, (const T*)p, (T*)x, (T*)r_out, z, scal,
                         first, prr, pcs, prz, xf);
    else if (zf)
      UJ(1);
    else
      UJ(0);
#undef UJ
  }
  static void xfinal(int n, void* x, const void* p, const double* scal, double* pcs, hipStream_t s) {
    const int g = grid_units(n, RG);
    if (!g) return;
    hipLaunchKernelGGL((k_xfinal<T, W>), dim3(g * NS), dim3(kBlock), 0, s, n, (T*)x, (const T*)p, scal,
                       pcs);
  }
  static void coarse(int nc, int ncp, const double* A, const void* b, void* x, hipStream_t s) {
#ifndef CFC_COARSE_NO_MFMA
    if constexpr (W >= 16) {
      const int waves = (ncp / 16) * (W / 16);
      hipLaunchKernelGGL((k_coarse_mfma<T, W>), dim3((waves + 3) / 4), dim3(256), 0, s, nc, ncp, A,
                         (const T*)b, (T*)x);
    } else
#endif
    {
      hipLaunchKernelGGL((k_coarse_simple<T, W>), dim3((nc * W + 255) / 256), dim3(256), 0, s, nc,
                         ncp, A, (const T*)b, (T*)x);
    }
  }
  static void dot(int n, const void* a, const void* b, double* part, hipStream_t s) {
    const int g = grid_units(n, RG);
    if (!g) return;
    hipLaunchKernelGGL((k_dot<T, W>), dim3(g * NS), dim3(kBlock), 0, s, n, (const T*)a, (const T*)b,
                       part);
  }
  static void residual64(const LevelArgs& L, const void* x, int x_fp32, RhsArgs rhs, void* r_out,
                         double* part, hipStream_t s) {
    const dim3 gh(std::min(L.nseg, 4 * kMaxGrid) * NS);
    if (x && L.nseg && x_fp32)
      hipLaunchKernelGGL((k_heavy<double, W, HK_RES32>), gh, dim3(kBlock), 0, s, L, (const double*)x,
                         (const double*)nullptr, (const double*)nullptr, (const double*)nullptr);
    else if (x && L.nseg)
      hipLaunchKernelGGL((k_heavy<double, W, HK_RES64>), gh, dim3(kBlock), 0, s, L, (const double*)x,
                         (const double*)nullptr, (const double*)nullptr, (const double*)nullptr);
    if (x) heavy_sum<double>(L, s);
    if (x_fp32) {
#define ARGS L, (const float*)x, rhs, (T*)r_out, part
      CFC_LAUNCH(k_residual64, L.n, T, W, float);
#undef ARGS
    } else {
#define ARGS L, (const double*)x, rhs, (T*)r_out, part
      CFC_LAUNCH(k_residual64, L.n, T, W, double);
#undef ARGS
    }
  }
  static void xupdate64(int n, double* x64, const void* d, const double* scal, int first,
                        hipStream_t s) {
    const size_t total = (size_t)n * W;
    int g = (int)std::min<size_t>((total + kBlock - 1) / kBlock, 8192);
    if (!g) return;
    hipLaunchKernelGGL((k_xupdate64<T, W>), dim3(g), dim3(kBlock), 0, s, n, x64, (const T*)d, scal,
                       first);
  }
  static int jl_rhs(const LevelArgs& L, const int* iperm, uint64_t seed, int64_t i0, int64_t k,
                    double* Y, void* r, double* part, hipStream_t s) {
    const int g = grid_units(L.n, RG);
    if (!g) return 0;
    hipLaunchKernelGGL((k_jl_rhs<T, W>), dim3(g * NS), dim3(kBlock), 0, s, L, iperm, seed, i0, k, Y,
                       (T*)r, part);
    return g;
  }
  static void jl_rownorm(int n, const double* x64, int ncols, double* N, double* part,
                         hipStream_t s) {
    const int g = grid_units(n, RowShape<W>::RG);
    if (!g) return;
    hipLaunchKernelGGL((k_jl_rownorm<W>), dim3(g), dim3(kBlock), 0, s, n, x64, ncols, N);
    if (!part) return;
    // column sums of the block, sliced like the other partial sums
    const int gc = grid_units(n, RG);
    hipLaunchKernelGGL((k_dot<double, W>), dim3(gc * NS), dim3(kBlock), 0, s, n, x64,
                       (const double*)nullptr, part);
  }
  static int elim_grid(int units) { return std::min(grid_units(units, RG), kMaxGrid / 2); }
  static void elim_fwd(const LevelArgs& L, const void* r, void* out, const void* sd1,
                       double* part, int jac, hipStream_t s) {
    heavy<HK_SPMM>(L, r, nullptr, nullptr, nullptr, s);
    const int g = elim_grid(L.n);
    if (!g) return;
    if (jac == 2)
      hipLaunchKernelGGL((k_elim_fwd<T, W, true, true>), dim3(g * NS), dim3(kBlock), 0, s, L,
                         (const T*)r, out, (const T*)sd1, part);
    else if (jac)
      hipLaunchKernelGGL((k_elim_fwd<T, W, true, false>), dim3(g * NS), dim3(kBlock), 0, s, L,
                         (const T*)r, out, (const T*)sd1, part);
    else
      hipLaunchKernelGGL((k_elim_fwd<T, W, false, false>), dim3(g * NS), dim3(kBlock), 0, s, L,
                         (const T*)r, out, (const T*)sd1, part);
  }
  static void elim_back(const LevelArgs& L, const void* r, void* z, double* part, int allrows,
                        int bf, hipStream_t s) {
    const int g = elim_grid(allrows ? L.n : L.n - L.nC);
    if (!g) return;
    if (allrows && bf)
      hipLaunchKernelGGL((k_elim_back<T, W, true, true>), dim3(g * NS), dim3(kBlock), 0, s, L,
                         (const T*)r, z, part);
    else if (allrows)
      hipLaunchKernelGGL((k_elim_back<T, W, true, false>), dim3(g * NS), dim3(kBlock), 0, s, L,
                         (const T*)r, z, part);
    else if (bf)
      hipLaunchKernelGGL((k_elim_back<T, W, false, true>), dim3(g * NS), dim3(kBlock), 0, s, L,
                         (const T*)r, z, part);
    else
      hipLaunchKernelGGL((k_elim_back<T, W, false, false>), dim3(g * NS), dim3(kBlock), 0, s, L,
                         (const T*)r, z, part);
  }
  static void throughput(const LevelArgs& L, const double* x64, int ncols, const int* ps,
                         const int* pt, double* seg_part, double* tp, hipStream_t s) {
    if (L.nseg) {
      const int gs = std::min(L.nseg, 4 * kMaxGrid);
      hipLaunchKernelGGL((k_tp_seg<W>), dim3(gs), dim3(kBlock), 0, s, L, x64, ncols, ps, pt, seg_part);
    }
    const int g = grid_units(L.n, RowShape<W>::RG);
    if (!g) return;
    hipLaunchKernelGGL((k_tp_rows<W>), dim3(g), dim3(kBlock), 0, s, L, x64, ncols, ps, pt,
                       (const double*)seg_part, tp);
  }
  static void edge_sq(int ne, const int* a, const int* b, const double* x64, int ncols, double* out,
                      hipStream_t s) {
    const int g = grid_units(ne, RowShape<W>::RG);
    if (!g) return;
    hipLaunchKernelGGL((k_edge_sq<W>), dim3(g), dim3(kBlock), 0, s, ne, a, b, x64, ncols, out);
  }
  static void zero(void* p, size_t bytes, hipStream_t s) { zero_fill(p, bytes, s); }

  static KernTable table() {
    KernTable t;
    t.W = W;
    t.esize = sizeof(T);
    t.rg = RG;
    t.rows_grid = &rows_grid;
    t.rg8 = RG8;
    t.ns8 = NS8;
    t.rows_grid8 = &rows_grid8;
    t.spmm_pq = &spmm_pq;
    t.update_restrict = &update_restrict;
    t.restrict_ = &restrict_;
    t.prolong_smooth = &prolong_smooth;
    t.coarse = &coarse;
    t.jacobi = &jacobi;
    t.update_jacobi = &update_jacobi;
    t.xfinal = &xfinal;
    t.dot = &dot;
    t.residual64 = &residual64;
    t.xupdate64 = &xupdate64;
    t.jl_rhs = &jl_rhs;
    t.jl_rownorm = &jl_rownorm;
    t.zero = &zero;
    t.throughput = &throughput;
    t.elim_fwd = &elim_fwd;
    t.elim_back = &elim_back;
    t.elim_grid = &elim_grid;
    t.edge_sq = &edge_sq;
    return t;
  }
};

}  // namespace dev
}  // namespace cfc

#define CFC_DEFINE_TABLES(WW)                                                 \
  namespace cfc {                                                             \
  const KernTable* kern_table_##WW(bool fp64) {                               \
    static const KernTable tf = dev::Launch<float, WW>::table();              \
    static const KernTable td = dev::Launch<double, WW>::table();             \
    return fp64 ? &td : &tf;                                                  \
  }                                                                           \
  }
