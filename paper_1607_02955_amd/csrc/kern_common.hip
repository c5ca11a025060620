// Width-independent kernels (finalize of partial sums, gathers) and the
// per-width table dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "block.hpp"
#include "kern.hpp"

namespace cfc {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

const KernTable* kern_table_1(bool);
const KernTable* kern_table_32(bool);
const KernTable* kern_table_64(bool);
const KernTable* kern_table_128(bool);
const KernTable* kern_table_256(bool);
const KernTable* kern_table_512(bool);

const KernTable* kern_table(int W, bool fp64) {
  switch (W) {
    case 1: return kern_table_1(fp64);
    case 32: return kern_table_32(fp64);
    case 64: return kern_table_64(fp64);
    case 128: return kern_table_128(fp64);
    case 256: return kern_table_256(fp64);
    case 512: return kern_table_512(fp64);
    default: return nullptr;
  }
}

int grid_for(int units, int rg, int cap_scale) {
  // Workgroups per column slice.  Large levels take 1024 (8192 in all at
  // eight slices, four rounds of the 2048 that are resident at once); levels
  // of at most 8192 row tiles take 512, so that each workgroup walks at
  // least a dozen tiles and the partial sums stay small (measured on the
  // level-0 kernels: BA-100k projection +2.4% at 512, R-MAT-20 and
  // road-2048 levels 5-6% slower there).  CFC_GRID_CAP fixes one cap for
  // every level, at most kMaxGrid (the partial-sum buffers' row count).
  // cap_scale > 1 (kernels that slice the columns fewer ways) raises the
  // cap up to that factor, as far as each workgroup still walks 16 tiles
  // (R-MAT-20's FP8 product, 43k tiles: 3.73 against 3.91 ms at twice the
  // cap; BA-100k's, 8k tiles, was slower at twice the cap).
  static const int fixed = [] {
    const char* e = std::getenv("CFC_GRID_CAP");
    return e ? std::max(8, std::min(kMaxGrid, std::atoi(e))) : 0;
  }();
  if (units <= 0) return 0;
  int tiles = (units + rg - 1) / rg;
  int cap = fixed ? fixed : (tiles <= 8192 ? kMaxGrid / 4 : kMaxGrid / 2);
  if (cap_scale > 1) cap = std::min(cap * cap_scale, std::max(cap, tiles / 16));
  cap = std::min(cap, kMaxGrid);
  int g = std::min(tiles, cap);
  if (g >= 64) g &= ~7;
  return g;
}

namespace {

// Sum partial rows g = 0..G-1 of up to three arrays, per column, in a fixed
// order, then apply the scalar update of the PCG / refinement step.  A
// workgroup owns FCH columns; each of its 256/FCH thread groups takes every
// (256/FCH)-th partial row (four loads in flight), and LDS combines the
// groups in order.
constexpr int FCH = 16;

__device__ __forceinline__ double sum_rows(const double* __restrict__ p, int G, int W, int c, int sp,
                                           int S) {
  double s = 0;
  int g = sp;
  for (; g + 3 * S < G; g += 4 * S) {
    const double a0 = p[(size_t)g * W + c], a1 = p[(size_t)(g + S) * W + c];
    const double a2 = p[(size_t)(g + 2 * S) * W + c], a3 = p[(size_t)(g + 3 * S) * W + c];
    s += a0;
    s += a1;
    s += a2;
    s += a3;
  }
  for (; g < G; g += S) s += p[(size_t)g * W + c];
  return s;
}

__global__ __launch_bounds__(256) void k_finalize(int W, int op, int g0, const double* __restrict__ p0,
                                                  int g1, const double* __restrict__ p1, int g2,
                                                  const double* __restrict__ p2,
                                                  double* __restrict__ scal, double* __restrict__ host) {
  const int CH = W < FCH ? W : FCH;
  const int S = 256 / CH;
  const int tid = threadIdx.x;
  const int c = blockIdx.x * CH + tid % CH;
  const int sp = tid / CH;
  __shared__ double red[3][256];
  double s0 = 0, s1 = 0, s2 = 0;
  if (sp < S && c < W) {
    s0 = sum_rows(p0, g0, W, c, sp, S);
    if (p1) s1 = sum_rows(p1, g1, W, c, sp, S);
    if (p2) s2 = sum_rows(p2, g2, W, c, sp, S);
  }
  red[0][tid] = s0;
  red[1][tid] = s1;
  red[2][tid] = s2;
  __syncthreads();
  if (sp != 0 || c >= W) return;
  double t0 = 0, t1 = 0, t2 = 0;
  for (int s = 0; s < S; ++s) {
    t0 += red[0][s * CH + tid];
    t1 += red[1][s * CH + tid];
    t2 += red[2][s * CH + tid];
  }
  switch (op) {
    case F_ALPHA: {
      const double rz = scal[S_RZ * W + c];
      scal[S_PQ * W + c] = t0;
      scal[S_ALPHA * W + c] = (t0 > 0 && rz > 0 && isfinite(rz / t0)) ? rz / t0 : 0.0;
      break;
    }
    case F_RZINIT:
      scal[S_RZ * W + c] = t0;
      scal[S_BETA * W + c] = 0.0;
      break;
    case F_BETA: {
      const double rz = scal[S_RZ * W + c];
      const double beta = (rz > 0 && t0 > 0) ? t0 / rz : 0.0;
      scal[S_BETA * W + c] = isfinite(beta) ? beta : 0.0;
      scal[S_RZ * W + c] = t0;
      scal[S_RR * W + c] = t1;
      scal[S_CS * W + c] = t2;
      if (host) host[S_RR * W + c] = t1;  // read by the host's convergence test
      break;
    }
    case F_R64:
      scal[S_R64 * W + c] = t0;
      if (host) host[S_R64 * W + c] = t0;
      break;
    case F_CS:
      scal[S_CS * W + c] = t0;
      break;
  }
}

__global__ void k_pair_diff(int W, int ncols, const double* __restrict__ x,
                            const int* __restrict__ ps, const int* __restrict__ pt,
                            double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncols) return;
  const int s = ps[j], t = pt[j];
  out[j] = (s >= 0 && t >= 0) ? x[(size_t)s * W + j] - x[(size_t)t * W + j] : 0.0;
}

__global__ void k_pair_acc(int W, int ncols, const float* __restrict__ d, const int* __restrict__ ps,
                           const int* __restrict__ pt, double* __restrict__ out, int first) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncols) return;
  const int s = ps[j], t = pt[j];
  const double v = (s >= 0 && t >= 0) ? double(d[(size_t)s * W + j]) - double(d[(size_t)t * W + j]) : 0.0;
  out[j] = first ? v : out[j] + v;
}

__global__ void k_gather(int q, const double* __restrict__ src, const int* __restrict__ idx,
                         double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < q) out[i] = src[idx[i]];
}

__global__ void k_gather_rc(int64_t q, const double* __restrict__ src, int W,
                            const int* __restrict__ row, const int* __restrict__ col,
                            double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < q) out[i] = src[(size_t)row[i] * W + col[i]];
}

// Compensated (Neumaier) summation step: s + c carries the running sum to
// about one rounding of the exact value.
__device__ inline void neumaier_add(double& s, double& c, double v) {
  const double t = s + v;
  c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
  s = t;
}

// Column-major block (column j of nc at Bc + j n, graph node order) to the
// node-major n x W layout in level-0 row order: rhs[perm[v] W + j]; columns
// nc..W-1 are zero.  32 x 32 tiles staged in LDS so that both the column
// reads (along v) and the row writes (along j) are contiguous.
__global__ __launch_bounds__(256) void k_block_in(int n, int W, int nc, const double* __restrict__ Bc,
                                                  const int* __restrict__ perm,
                                                  double* __restrict__ rhs) {
  __shared__ double tile[32][33];
  const int v0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int k = ty; k < 32; k += 8) {
    const int j = j0 + k, v = v0 + tx;
    tile[k][tx] = (j < nc && v < n) ? Bc[(size_t)j * n + v] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int v = v0 + k, j = j0 + tx;
    if (v < n && j < W) rhs[(size_t)perm[v] * W + j] = tile[tx][k];
  }
}

// The inverse: Xc[j n + v] = x[perm[v] W + j] - cs[j] / n for j < nc (the
// column sums cs of x, so the result is mean-zero).
__global__ __launch_bounds__(256) void k_block_out(int n, int W, int nc, const double* __restrict__ x,
                                                   const int* __restrict__ perm,
                                                   const double* __restrict__ cs,
                                                   double* __restrict__ Xc) {
  __shared__ double tile[32][33];
  const int v0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int k = ty; k < 32; k += 8) {
    const int v = v0 + k, j = j0 + tx;
    tile[k][tx] = (v < n && j < nc) ? x[(size_t)perm[v] * W + j] : 0.0;
  }
  __syncthreads();
  const double inv = 1.0 / double(n);
  for (int k = ty; k < 32; k += 8) {
    const int j = j0 + k, v = v0 + tx;
    if (j < nc && v < n) Xc[(size_t)j * n + v] = tile[tx][k] - cs[j] * inv;
  }
}

// Per-column sum and sum of magnitudes of a node-major n x W block: each
// workgroup adds a contiguous row range in order (partials [blk][2W]), then
// one thread per column adds the partials in order.
__global__ __launch_bounds__(256) void k_colstat_part(int n, int W, const double* __restrict__ x,
                                                      double* __restrict__ part) {
  const int per = (n + gridDim.x - 1) / gridDim.x;
  const int r0 = blockIdx.x * per, r1 = min(n, r0 + per);
  for (int j = threadIdx.x; j < W; j += blockDim.x) {
    double s = 0, c = 0, a = 0;
    for (int r = r0; r < r1; ++r) {
      const double v = x[(size_t)r * W + j];
      neumaier_add(s, c, v);
      a += fabs(v);
    }
    part[(size_t)blockIdx.x * 2 * W + j] = s + c;
    part[(size_t)blockIdx.x * 2 * W + W + j] = a;
  }
}

__global__ void k_colstat_final(int G, int W, const double* __restrict__ part, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= W) return;
  double s = 0, c = 0, a = 0;
  for (int g = 0; g < G; ++g) {
    neumaier_add(s, c, part[(size_t)g * 2 * W + j]);
    a += part[(size_t)g * 2 * W + W + j];
  }
  out[j] = s + c;
  out[W + j] = a;
}

__global__ __launch_bounds__(256) void k_reduce_part(int n, const double* __restrict__ x,
                                                     double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_reduce_final(int g, const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < g; ++i) s += part[i];
    *out = s;
  }
}

__global__ void k_zero(uint32_t* p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void k_zero_cols(int n, int W, double* __restrict__ x, const int* __restrict__ flag) {
  const size_t total = (size_t)n * W;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x)
    if (flag[i % W]) x[i] = 0.0;
}

}  // namespace

void zero_cols(int n, int W, double* x64, const int* flag, hipStream_t s) {
  const size_t total = (size_t)n * W;
  if (!total) return;
  const int g = (int)std::min<size_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(k_zero_cols, dim3(g), dim3(256), 0, s, n, W, x64, flag);
}

// Streaming copy: each lane moves 16 bytes per step with non-temporal loads
// and stores, consecutive lanes on consecutive 16-byte words (every wave
// instruction covers 1 KiB); a grid-stride loop over the 16-byte words,
// then the tail bytes.
__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                     size_t n16, const unsigned char* __restrict__ srcb,
                                                     unsigned char* __restrict__ dstb, size_t tail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < tail) dstb[t] = srcb[t];
}

void stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!bytes) return;
  const size_t n16 = bytes / 16, tail = bytes - n16 * 16;
  const int g = (int)std::max<size_t>(1, std::min<size_t>((n16 + 255) / 256, 16384));
  hipLaunchKernelGGL(k_stream_copy, dim3(g), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, n16,
                     (const unsigned char*)src + n16 * 16, (unsigned char*)dst + n16 * 16, tail);
}

void zero_fill(void* p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  if (!words || !p) return;
  const int g = (int)std::min<size_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero, dim3(g), dim3(256), 0, s, (uint32_t*)p, words);
}

void finalize(int W, int op, int g0, const double* p0, int g1, const double* p1, int g2,
              const double* p2, double* scal, hipStream_t s, double* host) {
  const int CH = W < FCH ? W : FCH;
  hipLaunchKernelGGL(k_finalize, dim3((W + CH - 1) / CH), dim3(256), 0, s, W, op, g0, p0, g1, p1,
                     g2, p2, scal, host);
}

void pair_diff(int W, int ncols, const double* x64, const int* ps, const int* pt, double* out,
               hipStream_t s) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_pair_diff, dim3((ncols + 255) / 256), dim3(256), 0, s, W, ncols, x64, ps, pt,
                     out);
}

void pair_acc(int W, int ncols, const float* d, const int* ps, const int* pt, double* out, int first,
              hipStream_t s) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(k_pair_acc, dim3((ncols + 255) / 256), dim3(256), 0, s, W, ncols, d, ps, pt, out,
                     first);
}

void gather(int q, const double* src, const int* idx, double* out, hipStream_t s) {
  if (q <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3((q + 255) / 256), dim3(256), 0, s, q, src, idx, out);
}

void gather_rc(int64_t q, const double* src, int W, const int* row, const int* col, double* out,
               hipStream_t s) {
  if (q <= 0) return;
  hipLaunchKernelGGL(k_gather_rc, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, q, src, W, row,
                     col, out);
}

void block_in(int n, int W, int nc, const double* Bc, const int* perm, double* rhs, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_block_in, dim3((n + 31) / 32, (W + 31) / 32), dim3(256), 0, s, n, W, nc, Bc, perm,
                     rhs);
}

void block_out(int n, int W, int nc, const double* x, const int* perm, const double* cs, double* Xc,
               hipStream_t s) {
  if (n <= 0 || nc <= 0) return;
  hipLaunchKernelGGL(k_block_out, dim3((n + 31) / 32, (nc + 31) / 32), dim3(256), 0, s, n, W, nc, x,
                     perm, cs, Xc);
}

void col_stats(int n, int W, const double* x, double* part, double* out, hipStream_t s) {
  const int G = kColStatGrid;
  hipLaunchKernelGGL(k_colstat_part, dim3(G), dim3(256), 0, s, n, W, x, part);
  hipLaunchKernelGGL(k_colstat_final, dim3((W + 255) / 256), dim3(256), 0, s, G, W, (const double*)part,
                     out);
}

void reduce_sum(int n, const double* x, double* part, double* out, hipStream_t s) {
  const int g = std::max(1, std::min((n + 255) / 256, 1024));
  hipLaunchKernelGGL(k_reduce_part, dim3(g), dim3(256), 0, s, n, x, part);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, s, g, part, out);
}

}  // namespace cfc
