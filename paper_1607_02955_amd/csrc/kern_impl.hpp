// Device kernels of the multigrid Laplacian solve (gfx950, wave64).
//
// Data layout: every n x W block is node-major (node u's W values are
// contiguous).  A "row group" of LPR lanes owns one row at a time, each lane
// V consecutive columns (W = LPR * V), so a neighbour's row is one coalesced
// W*sizeof(T)-byte read.  Workgroups walk a contiguous range of row tiles,
// and the tile ranges are dealt out XCD by XCD (hardware deals workgroups to
// the 8 XCDs round-robin), so rows that are close in the aggregate-nested
// numbering share an L2.
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

template <int W> struct Shape;
template <> struct Shape<1> { static constexpr int LPR = 1, V = 1; };
template <> struct Shape<32> { static constexpr int LPR = 8, V = 4; };
template <> struct Shape<64> { static constexpr int LPR = 16, V = 4; };
template <> struct Shape<128> { static constexpr int LPR = 32, V = 4; };
template <> struct Shape<256> { static constexpr int LPR = 64, V = 4; };
template <> struct Shape<512> { static constexpr int LPR = 64, V = 8; };

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

// Contiguous tile range of this workgroup; consecutive ranges go to one XCD.
__device__ __forceinline__ void block_tiles(int ntiles, int& tb, int& te) {
  const int G = gridDim.x, b = blockIdx.x;
  const int vb = ((G & 7) == 0) ? (b & 7) * (G >> 3) + (b >> 3) : b;
  const int per = (ntiles + G - 1) / G;
  tb = min(vb * per, ntiles);
  te = min(tb + per, ntiles);
}

// Sum acc over the row groups of the workgroup and store W values to out.
template <int W>
__device__ __forceinline__ void block_store(const double* acc, double* lds, double* out) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = kBlock / LPR;
  const int rg = threadIdx.x / LPR, c0 = (threadIdx.x % LPR) * V;
#pragma unroll
  for (int i = 0; i < V; ++i) lds[rg * W + c0 + i] = acc[i];
  __syncthreads();
  for (int c = threadIdx.x; c < W; c += kBlock) {
    double s = 0;
    for (int g = 0; g < RG; ++g) s += lds[g * W + c];
    out[c] = s;
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ T wt(const T* w, int e) {
  return w ? w[e] : T(1);
}

// a -= sum_e w_e x[col_e]   (rows e0..e1), four gathers in flight.
template <typename T, int W>
__device__ __forceinline__ void gather_sub(T* a, const T* __restrict__ x, const int* __restrict__ col,
                                           const T* __restrict__ w, int e0, int e1, int c0) {
  constexpr int V = Shape<W>::V;
  int e = e0;
  for (; e + 4 <= e1; e += 4) {
    const int v0 = col[e], v1 = col[e + 1], v2 = col[e + 2], v3 = col[e + 3];
    const T w0 = wt(w, e), w1 = wt(w, e + 1), w2 = wt(w, e + 2), w3 = wt(w, e + 3);
    const Vec<T, V> x0 = ld<T, V>(x + (size_t)v0 * W + c0);
    const Vec<T, V> x1 = ld<T, V>(x + (size_t)v1 * W + c0);
    const Vec<T, V> x2 = ld<T, V>(x + (size_t)v2 * W + c0);
    const Vec<T, V> x3 = ld<T, V>(x + (size_t)v3 * W + c0);
#pragma unroll
    for (int i = 0; i < V; ++i) {
      a[i] -= w0 * x0.v[i];
      a[i] -= w1 * x1.v[i];
      a[i] -= w2 * x2.v[i];
      a[i] -= w3 * x3.v[i];
    }
  }
  for (; e < e1; ++e) {
    const int v0 = col[e];
    const T w0 = wt(w, e);
    const Vec<T, V> x0 = ld<T, V>(x + (size_t)v0 * W + c0);
#pragma unroll
    for (int i = 0; i < V; ++i) a[i] -= w0 * x0.v[i];
  }
}

// ---------------------------------------------------------------------------
// PCG step on level 0: q = L z + beta q, p = z + beta p; partial p.q
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_spmm_pq(LevelArgs L, const T* __restrict__ z,
                                                    T* __restrict__ p, T* __restrict__ q,
                                                    const double* __restrict__ scal, int first,
                                                    double* __restrict__ part) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = kBlock / LPR;
  __shared__ double lds[RG * W];
  const int rg = threadIdx.x / LPR, c0 = (threadIdx.x % LPR) * V;
  const T* w = static_cast<const T*>(L.w);
  const T* deg = static_cast<const T*>(L.deg);
  T beta[V];
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) {
    beta[i] = first ? T(0) : T(scal[S_BETA * W + c0 + i]);
    acc[i] = 0;
  }
  int tb, te;
  block_tiles((L.n + RG - 1) / RG, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u < L.n) {
      const size_t o = (size_t)u * W + c0;
      const Vec<T, V> zu = ld<T, V>(z + o);
      T a[V];
      const T du = deg[u];
#pragma unroll
      for (int i = 0; i < V; ++i) a[i] = du * zu.v[i];
      gather_sub<T, W>(a, z, L.col, w, L.rowptr[u], L.rowptr[u + 1], c0);
      Vec<T, V> pn, qn;
      if (first) {
        pn = zu;
#pragma unroll
        for (int i = 0; i < V; ++i) qn.v[i] = a[i];
      } else {
        const Vec<T, V> po = ld<T, V>(p + o), qo = ld<T, V>(q + o);
#pragma unroll
        for (int i = 0; i < V; ++i) {
          pn.v[i] = zu.v[i] + beta[i] * po.v[i];
          qn.v[i] = a[i] + beta[i] * qo.v[i];
        }
      }
      st<T, V>(p + o, pn);
      st<T, V>(q + o, qn);
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] += double(pn.v[i]) * double(qn.v[i]);
    }
  }
  block_store<W>(acc, lds, part + (size_t)blockIdx.x * W);
}

// ---------------------------------------------------------------------------
// Update (r -= alpha q, x += alpha p) and/or pre-smooth + residual + restrict.
// Units are aggregates when RESTRICT (their rows are contiguous), else rows.
template <typename T, int W, bool UPDATE, bool RESTRICT>
__global__ __launch_bounds__(kBlock) void k_update_restrict(
    LevelArgs L, const T* __restrict__ r_in, const T* __restrict__ q, const T* __restrict__ p,
    T* __restrict__ x, T* __restrict__ r_out, T* __restrict__ bc, const double* __restrict__ scal,
    int first, double* __restrict__ part_rr, double* __restrict__ part_cs) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = kBlock / LPR;
  __shared__ double lds[RG * W];
  const int rg = threadIdx.x / LPR, c0 = (threadIdx.x % LPR) * V;
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
  block_tiles((units + RG - 1) / RG, tb, te);
  for (int t = tb; t < te; ++t) {
    const int I = t * RG + rg;
    if (I >= units) continue;
    const int r0 = RESTRICT ? L.aggptr[I] : I;
    const int r1 = RESTRICT ? L.aggptr[I + 1] : I + 1;
    T s[V];
#pragma unroll
    for (int i = 0; i < V; ++i) s[i] = 0;
    for (int u = r0; u < r1; ++u) {
      const size_t o = (size_t)u * W + c0;
      Vec<T, V> rn = ld<T, V>(r_in + o);
      if (UPDATE) {
        const Vec<T, V> qu = ld<T, V>(q + o), pu = ld<T, V>(p + o);
        Vec<T, V> xu;
        if (!first) xu = ld<T, V>(x + o);
#pragma unroll
        for (int i = 0; i < V; ++i) {
          rn.v[i] -= alpha[i] * qu.v[i];
          xu.v[i] = first ? alpha[i] * pu.v[i] : xu.v[i] + alpha[i] * pu.v[i];
          rr[i] += double(rn.v[i]) * double(rn.v[i]);
          cs[i] += double(xu.v[i]);
        }
        st<T, V>(x + o, xu);
        st<T, V>(r_out + o, rn);
      }
      if (RESTRICT) {
        T a[V];
#pragma unroll
        for (int i = 0; i < V; ++i) a[i] = om1 * rn.v[i];
        const int e1 = L.rowptr[u + 1];
        int e = L.rowptr[u];
        for (; e + 2 <= e1; e += 2) {
          const int v0 = L.col[e], v1 = L.col[e + 1];
          const T f0 = wt(w, e) * sd[v0], f1 = wt(w, e + 1) * sd[v1];
          Vec<T, V> a0 = ld<T, V>(r_in + (size_t)v0 * W + c0);
          Vec<T, V> a1 = ld<T, V>(r_in + (size_t)v1 * W + c0);
          if (UPDATE) {
            const Vec<T, V> q0 = ld<T, V>(q + (size_t)v0 * W + c0);
            const Vec<T, V> q1 = ld<T, V>(q + (size_t)v1 * W + c0);
#pragma unroll
            for (int i = 0; i < V; ++i) {
              a0.v[i] -= alpha[i] * q0.v[i];
              a1.v[i] -= alpha[i] * q1.v[i];
            }
          }
#pragma unroll
          for (int i = 0; i < V; ++i) {
            a[i] += f0 * a0.v[i];
            a[i] += f1 * a1.v[i];
          }
        }
        if (e < e1) {
          const int v0 = L.col[e];
          const T f0 = wt(w, e) * sd[v0];
          Vec<T, V> a0 = ld<T, V>(r_in + (size_t)v0 * W + c0);
          if (UPDATE) {
            const Vec<T, V> q0 = ld<T, V>(q + (size_t)v0 * W + c0);
#pragma unroll
            for (int i = 0; i < V; ++i) a0.v[i] -= alpha[i] * q0.v[i];
          }
#pragma unroll
          for (int i = 0; i < V; ++i) a[i] += f0 * a0.v[i];
        }
#pragma unroll
        for (int i = 0; i < V; ++i) s[i] += a[i];
      }
    }
    if (RESTRICT) {
      Vec<T, V> sv;
#pragma unroll
      for (int i = 0; i < V; ++i) sv.v[i] = s[i];
      st<T, V>(bc + (size_t)I * W + c0, sv);
    }
  }
  if (UPDATE) {
    block_store<W>(rr, lds, part_rr + (size_t)blockIdx.x * W);
    block_store<W>(cs, lds, part_cs + (size_t)blockIdx.x * W);
  }
}

// ---------------------------------------------------------------------------
// Prolongation + post-smoothing: xt = S b + mu xc[agg], x = xt + S (b - L xt).
template <typename T, int W, bool DOT>
__global__ __launch_bounds__(kBlock) void k_prolong_smooth(LevelArgs L, const T* __restrict__ b,
                                                           const T* __restrict__ xc,
                                                           T* __restrict__ x,
                                                           double* __restrict__ part) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = kBlock / LPR;
  __shared__ double lds[DOT ? RG * W : 1];
  const int rg = threadIdx.x / LPR, c0 = (threadIdx.x % LPR) * V;
  const T* w = static_cast<const T*>(L.w);
  const T* sd = static_cast<const T*>(L.sd);
  const T* deg = static_cast<const T*>(L.deg);
  const T mu = T(L.mu);
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = 0;
  int tb, te;
  block_tiles((L.n + RG - 1) / RG, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u >= L.n) continue;
    const size_t o = (size_t)u * W + c0;
    const Vec<T, V> bu = ld<T, V>(b + o);
    const Vec<T, V> cu = ld<T, V>(xc + (size_t)L.agg[u] * W + c0);
    const T sdu = sd[u], du = deg[u];
    T xt[V], a[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      xt[i] = sdu * bu.v[i] + mu * cu.v[i];
      a[i] = du * xt[i];
    }
    const int e1 = L.rowptr[u + 1];
    int e = L.rowptr[u];
    for (; e + 2 <= e1; e += 2) {
      const int v0 = L.col[e], v1 = L.col[e + 1];
      const T w0 = wt(w, e), w1 = wt(w, e + 1);
      const T s0 = sd[v0], s1 = sd[v1];
      const int g0 = L.agg[v0], g1 = L.agg[v1];
      const Vec<T, V> b0 = ld<T, V>(b + (size_t)v0 * W + c0);
      const Vec<T, V> b1 = ld<T, V>(b + (size_t)v1 * W + c0);
      const Vec<T, V> x0 = ld<T, V>(xc + (size_t)g0 * W + c0);
      const Vec<T, V> x1 = ld<T, V>(xc + (size_t)g1 * W + c0);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        a[i] -= w0 * (s0 * b0.v[i] + mu * x0.v[i]);
        a[i] -= w1 * (s1 * b1.v[i] + mu * x1.v[i]);
      }
    }
    if (e < e1) {
      const int v0 = L.col[e];
      const T w0 = wt(w, e), s0 = sd[v0];
      const Vec<T, V> b0 = ld<T, V>(b + (size_t)v0 * W + c0);
      const Vec<T, V> x0 = ld<T, V>(xc + (size_t)L.agg[v0] * W + c0);
#pragma unroll
      for (int i = 0; i < V; ++i) a[i] -= w0 * (s0 * b0.v[i] + mu * x0.v[i]);
    }
    Vec<T, V> xo;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      xo.v[i] = xt[i] + sdu * (bu.v[i] - a[i]);
      if (DOT) acc[i] += double(bu.v[i]) * double(xo.v[i]);
    }
    st<T, V>(x + o, xo);
  }
  if (DOT) block_store<W>(acc, lds, part + (size_t)blockIdx.x * W);
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
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = kBlock / LPR;
  __shared__ double lds[RG * W];
  const int rg = threadIdx.x / LPR, c0 = (threadIdx.x % LPR) * V;
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = 0;
  int tb, te;
  block_tiles((n + RG - 1) / RG, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u >= n) continue;
    const Vec<T, V> x = ld<T, V>(a + (size_t)u * W + c0), y = ld<T, V>(b + (size_t)u * W + c0);
#pragma unroll
    for (int i = 0; i < V; ++i) acc[i] += double(x.v[i]) * double(y.v[i]);
  }
  block_store<W>(acc, lds, part + (size_t)blockIdx.x * W);
}

// ---------------------------------------------------------------------------
// FP64 residual r = b - L x (Eq. 1), stored as TO; partial |r|^2 (FP64).
template <typename TO, int W>
__global__ __launch_bounds__(kBlock) void k_residual64(LevelArgs L, const double* __restrict__ x,
                                                       RhsArgs rhs, TO* __restrict__ r_out,
                                                       double* __restrict__ part) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = kBlock / LPR;
  __shared__ double lds[RG * W];
  const int rg = threadIdx.x / LPR, c0 = (threadIdx.x % LPR) * V;
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
  block_tiles((L.n + RG - 1) / RG, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u >= L.n) continue;
    const size_t o = (size_t)u * W + c0;
    double a[V];
#pragma unroll
    for (int i = 0; i < V; ++i) a[i] = 0;
    if (x) {
      const Vec<double, V> xu = ld<double, V>(x + o);
      const double du = deg[u];
#pragma unroll
      for (int i = 0; i < V; ++i) a[i] = du * xu.v[i];
      gather_sub<double, W>(a, x, L.col, w, L.rowptr[u], L.rowptr[u + 1], c0);
    }
    double bv[V];
    if (rhs.kind == 0) {
      const Vec<double, V> bb = ld<double, V>(rhs.dense + o);
#pragma unroll
      for (int i = 0; i < V; ++i) bv[i] = bb.v[i];
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) bv[i] = (u == ps[i] ? 1.0 : 0.0) - (u == pt[i] ? 1.0 : 0.0);
    }
    Vec<TO, V> ro;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      const double r = bv[i] - a[i];
      ro.v[i] = TO(r);
      acc[i] += r * r;
    }
    st<TO, V>(r_out + o, ro);
  }
  block_store<W>(acc, lds, part + (size_t)blockIdx.x * W);
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
template <int W>
__global__ __launch_bounds__(kBlock) void k_jl_rhs(LevelArgs L, const int* __restrict__ iperm,
                                                   uint64_t seed, int64_t i0, int64_t k,
                                                   double* __restrict__ Y) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = kBlock / LPR;
  const int rg = threadIdx.x / LPR, c0 = (threadIdx.x % LPR) * V;
  const double* w = static_cast<const double*>(L.w);
  const double inv_sqrt_k = 1.0 / sqrt(double(k));
  const int64_t sys0 = i0 + c0;
  const uint64_t word = uint64_t(sys0) >> 6;
  int tb, te;
  block_tiles((L.n + RG - 1) / RG, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    if (u >= L.n) continue;
    const uint64_t gu = uint64_t(iperm[u]);
    double a[V];
#pragma unroll
    for (int i = 0; i < V; ++i) a[i] = 0;
    for (int e = L.rowptr[u]; e < L.rowptr[u + 1]; ++e) {
      const uint64_t gv = uint64_t(iperm[L.col[e]]);
      const uint64_t lo = gu < gv ? gu : gv, hi = gu < gv ? gv : gu;
      const double sw = w ? sqrt(w[e]) : 1.0;
      const double sg = gu < gv ? sw : -sw;
      const uint64_t h = jl_word(seed, word, lo, hi);
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const int bit = int((h >> ((sys0 + i) & 63)) & 1u);
        a[i] += bit ? -sg : sg;
      }
    }
    Vec<double, V> yo;
#pragma unroll
    for (int i = 0; i < V; ++i) yo.v[i] = (sys0 + i < k) ? a[i] * inv_sqrt_k : 0.0;
    st<double, V>(Y + (size_t)u * W + c0, yo);
  }
}

// N[u] += |x_u|^2 over the first ncols columns; partial column sums.
template <int W>
__global__ __launch_bounds__(kBlock) void k_jl_rownorm(int n, const double* __restrict__ x, int ncols,
                                                       double* __restrict__ N,
                                                       double* __restrict__ part) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = kBlock / LPR;
  __shared__ double lds[RG * W];
  const int rg = threadIdx.x / LPR, lane = threadIdx.x % LPR, c0 = lane * V;
  double acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = 0;
  int tb, te;
  block_tiles((n + RG - 1) / RG, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    const bool ok = u < n;
    double s = 0;
    if (ok) {
      const Vec<double, V> xu = ld<double, V>(x + (size_t)u * W + c0);
#pragma unroll
      for (int i = 0; i < V; ++i)
        if (c0 + i < ncols) {
          s += xu.v[i] * xu.v[i];
          acc[i] += xu.v[i];
        }
    }
    for (int off = LPR / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, LPR);
    if (ok && lane == 0) N[u] += s;
  }
  block_store<W>(acc, lds, part + (size_t)blockIdx.x * W);
}

// T[u] += x_u . s with s the column sums held in scal[S_CS].
template <int W>
__global__ __launch_bounds__(kBlock) void k_jl_rowdot(int n, const double* __restrict__ x, int ncols,
                                                      const double* __restrict__ scal,
                                                      double* __restrict__ Tv) {
  constexpr int LPR = Shape<W>::LPR, V = Shape<W>::V, RG = kBlock / LPR;
  const int rg = threadIdx.x / LPR, lane = threadIdx.x % LPR, c0 = lane * V;
  double sc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) sc[i] = (c0 + i < ncols) ? scal[S_CS * W + c0 + i] : 0.0;
  int tb, te;
  block_tiles((n + RG - 1) / RG, tb, te);
  for (int t = tb; t < te; ++t) {
    const int u = t * RG + rg;
    const bool ok = u < n;
    double s = 0;
    if (ok) {
      const Vec<double, V> xu = ld<double, V>(x + (size_t)u * W + c0);
#pragma unroll
      for (int i = 0; i < V; ++i) s += xu.v[i] * sc[i];
    }
    for (int off = LPR / 2; off >= 1; off >>= 1) s += __shfl_xor(s, off, LPR);
    if (ok && lane == 0) Tv[u] += s;
  }
}

// ---------------------------------------------------------------------------
// host launchers
inline int grid_units(int units, int rg) { return grid_for(units, rg); }

template <typename T, int W>
struct Launch {
  static constexpr int RG = kBlock / Shape<W>::LPR;

  static void spmm_pq(const LevelArgs& L, const void* z, void* p, void* q, const double* scal,
                      int first, double* part, hipStream_t s) {
    const int g = grid_units(L.n, RG);
    if (!g) return;
    hipLaunchKernelGGL((k_spmm_pq<T, W>), dim3(g), dim3(kBlock), 0, s, L, (const T*)z, (T*)p,
                       (T*)q, scal, first, part);
  }
  static void update_restrict(const LevelArgs& L, const void* r_in, const void* q, const void* p,
                              void* x, void* r_out, void* bc, const double* scal, int first,
                              int do_update, double* prr, double* pcs, hipStream_t s) {
    const bool R = L.nagg > 0;
    const int g = grid_units(R ? L.nagg : L.n, RG);
    if (!g) return;
    if (do_update && R)
      hipLaunchKernelGGL((k_update_restrict<T, W, true, true>), dim3(g), dim3(kBlock), 0, s, L,
                         (const T*)r_in, (const T*)q, (const T*)p, (T*)x, (T*)r_out, (T*)bc, scal,
                         first, prr, pcs);
    else if (do_update)
      hipLaunchKernelGGL((k_update_restrict<T, W, true, false>), dim3(g), dim3(kBlock), 0, s, L,
                         (const T*)r_in, (const T*)q, (const T*)p, (T*)x, (T*)r_out, (T*)bc, scal,
                         first, prr, pcs);
    else
      hipLaunchKernelGGL((k_update_restrict<T, W, false, true>), dim3(g), dim3(kBlock), 0, s, L,
                         (const T*)r_in, (const T*)q, (const T*)p, (T*)x, (T*)r_out, (T*)bc, scal,
                         first, prr, pcs);
  }
  static void restrict_(const LevelArgs& L, const void* b, void* bc, hipStream_t s) {
    const int g = grid_units(L.nagg, RG);
    if (!g) return;
    hipLaunchKernelGGL((k_update_restrict<T, W, false, true>), dim3(g), dim3(kBlock), 0, s, L,
                       (const T*)b, (const T*)nullptr, (const T*)nullptr, (T*)nullptr,
                       (T*)nullptr, (T*)bc, (const double*)nullptr, 0, (double*)nullptr,
                       (double*)nullptr);
  }
  static void prolong_smooth(const LevelArgs& L, const void* b, const void* xc, void* x,
                             double* part, hipStream_t s) {
    const int g = grid_units(L.n, RG);
    if (!g) return;
    if (part)
      hipLaunchKernelGGL((k_prolong_smooth<T, W, true>), dim3(g), dim3(kBlock), 0, s, L,
                         (const T*)b, (const T*)xc, (T*)x, part);
    else
      hipLaunchKernelGGL((k_prolong_smooth<T, W, false>), dim3(g), dim3(kBlock), 0, s, L,
                         (const T*)b, (const T*)xc, (T*)x, part);
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
    hipLaunchKernelGGL((k_dot<T, W>), dim3(g), dim3(kBlock), 0, s, n, (const T*)a, (const T*)b,
                       part);
  }
  static void residual64(const LevelArgs& L, const double* x64, RhsArgs rhs, void* r_out,
                         double* part, hipStream_t s) {
    const int g = grid_units(L.n, RG);
    if (!g) return;
    hipLaunchKernelGGL((k_residual64<T, W>), dim3(g), dim3(kBlock), 0, s, L, x64, rhs, (T*)r_out,
                       part);
  }
  static void xupdate64(int n, double* x64, const void* d, const double* scal, int first,
                        hipStream_t s) {
    const size_t total = (size_t)n * W;
    int g = (int)std::min<size_t>((total + kBlock - 1) / kBlock, 8192);
    if (!g) return;
    hipLaunchKernelGGL((k_xupdate64<T, W>), dim3(g), dim3(kBlock), 0, s, n, x64, (const T*)d, scal,
                       first);
  }
  static void jl_rhs(const LevelArgs& L, const int* iperm, uint64_t seed, int64_t i0, int64_t k,
                     double* Y, hipStream_t s) {
    const int g = grid_units(L.n, RG);
    if (!g) return;
    hipLaunchKernelGGL((k_jl_rhs<W>), dim3(g), dim3(kBlock), 0, s, L, iperm, seed, i0, k, Y);
  }
  static void jl_rownorm(int n, const double* x64, int ncols, double* N, double* part,
                         hipStream_t s) {
    const int g = grid_units(n, RG);
    if (!g) return;
    hipLaunchKernelGGL((k_jl_rownorm<W>), dim3(g), dim3(kBlock), 0, s, n, x64, ncols, N, part);
  }
  static void jl_rowdot(int n, const double* x64, int ncols, const double* scal, double* Tv,
                        hipStream_t s) {
    const int g = grid_units(n, RG);
    if (!g) return;
    hipLaunchKernelGGL((k_jl_rowdot<W>), dim3(g), dim3(kBlock), 0, s, n, x64, ncols, scal, Tv);
  }
  static void zero(void* p, size_t bytes, hipStream_t s) { zero_fill(p, bytes, s); }

  static KernTable table() {
    KernTable t;
    t.W = W;
    t.esize = sizeof(T);
    t.rg = RG;
    t.spmm_pq = &spmm_pq;
    t.update_restrict = &update_restrict;
    t.restrict_ = &restrict_;
    t.prolong_smooth = &prolong_smooth;
    t.coarse = &coarse;
    t.dot = &dot;
    t.residual64 = &residual64;
    t.xupdate64 = &xupdate64;
    t.jl_rhs = &jl_rhs;
    t.jl_rownorm = &jl_rownorm;
    t.jl_rowdot = &jl_rowdot;
    t.zero = &zero;
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
