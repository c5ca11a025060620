// Host-visible interface of the device kernels (one table per block width W
// and element type).  All arrays are node-major: an n x W block stores node
// u's W values contiguously at offset u*W.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace cfc {

constexpr int kBlock = 256;      // threads per workgroup
constexpr int kMaxGrid = 2048;   // workgroups of kernels that emit partial sums
constexpr int kElimDeg = 4;      // neighbour slots of an eliminated row

// Column slices of a W-wide block (see Shape in kern_impl.hpp).
__host__ __device__ constexpr int slices_of(int W) {
  return W >= 512 ? 8 : (W >= 256 ? 4 : (W >= 32 ? W / 32 : 1));
}
// Byte offset of the per-row-slice scales (float[n][KernTable::ns8]) after
// the n x W bytes of an FP8 copy of z.
__host__ __device__ constexpr size_t f8_scale_off(int n, int W) {
  return ((size_t)n * (size_t)W + 255) & ~size_t(255);
}

// One multigrid level as the kernels see it (element type T chosen by table).
struct LevelArgs {
  int n = 0;        // rows
  int nagg = 0;     // aggregates (rows of the next level); 0 on the coarsest
  const int* rowptr = nullptr;
  const int* col = nullptr;
  const void* w = nullptr;    // T[nnz] conductances, nullptr = all ones
  const void* deg = nullptr;  // T[n] D_ii
  const void* sd = nullptr;   // T[n] omega / D_ii (0 for an isolated node)
  const int* agg = nullptr;   // [n] row -> next-level row
  const int* aggptr = nullptr;// [nagg+1] aggregate row ranges
  double omega = 2.0 / 3.0;
  double mu = 1.5;
  int split = 1;    // row groups sharing each row / aggregate: 1, 4 or 16
  // Heavy rows (degree above a threshold) keep no edges in the CSR above;
  // their edges sit in a separate CSR cut into segments that whole
  // workgroups sum in a pre-pass (partials hpart[segment][W]), and the main
  // kernels add a heavy row's segment partials in order.
  int nheavy = 0, nseg = 0;
  const int* heavy = nullptr;  // [n] heavy index of a row, -1 if light
  const int* hseg = nullptr;   // [nheavy+1] segment range of each heavy row
  const int* hptr = nullptr;   // [nheavy+1] edge range of each heavy row
  const int* hcol = nullptr;   // heavy edges: column
  const void* hw = nullptr;    // heavy edges: weight (T), nullptr = all ones
  const int* seg_e = nullptr;  // [nseg+1] edge range of each segment
  const int* seg_row = nullptr;// [nseg] row of each segment
  void* hpart = nullptr;       // [nseg][W] partial sums (element type T)
  // [nheavy][W] (element type T): the segment partials of each heavy row
  // added in segment order by a row-parallel pass after the pre-pass, so
  // the main kernels read one row per heavy row (nullptr: they add the
  // segments themselves)
  void* hsum = nullptr;
  // Elimination level (nC > 0): rows [nC, n) are eliminated; row nC + i has
  // kept neighbours enb[kElimDeg i + j] (j < kElimDeg; the neighbours first,
  // then -1), conductances ew[kElimDeg i + j] and einv[i] = 1 / D_ii
  // (element type T).  enb is 16-byte aligned.
  int nC = 0;
  const int* enb = nullptr;
  const void* ew = nullptr;
  const void* einv = nullptr;
};

// Right-hand side of the FP64 residual kernel.
struct RhsArgs {
  int kind = 0;                  // 0 = dense FP64 n x W, 1 = pairs e_s - e_t, 2 = dense FP32
  const double* dense = nullptr;
  const float* dense32 = nullptr;  // kind 2 (may be residual64's own r_out: each row is read
                                   // before it is overwritten)
  const int* ps = nullptr;       // [W] row of +1 (or -1 = none)
  const int* pt = nullptr;       // [W] row of -1 (or -1 = none)
  double* r64_out = nullptr;     // residual64: also store r in FP64 here (may be dense itself)
  int r0_rows = 0;               // > 0: the first residual (r = b, in the solver's r_a) and
                                 // its partial sums of r^2 (this many rows) are already formed
};

// Scalars kept per column on the device (double[kNScal][W]).
enum Scal { S_RZ = 0, S_ALPHA, S_BETA, S_RR, S_CS, S_PQ, S_R64, S_N };

struct KernTable {
  int W = 0;
  int esize = 0;  // sizeof(T)
  int rg = 0;     // rows (row groups) per workgroup
  // workgroups per column slice (= rows of partial sums) of a kernel over
  // `units` units of the level
  int (*rows_grid)(const LevelArgs&, int units);
  // The FP8 paths (spmm_pq jac = 3, jacobi / update_jacobi zf = 2) slice
  // the columns ns8 ways (half the regular count) with rg8 row groups per
  // workgroup and up to twice the workgroups per slice: their partial sums have
  // rows_grid8 / grid_for(units, rg8, slices_of(W) / ns8) rows, and the
  // scales of an FP8 z are float[n][ns8].
  int rg8 = 0;
  int ns8 = 0;
  int (*rows_grid8)(const LevelArgs&, int units);
  // PCG step: q = L z + beta q, p = z + beta p (first: beta = 0); partial p.q.
  // jac = 1: z is passed as r and formed as S r on the fly; jac = 2: z is
  // its bfloat16 copy (uint16[n][W]); jac = 3: its FP8 copy (uint8[n][W],
  // then float scales[n][slices] at f8_scale_off(n, W)).  x (nullable): also apply the previous
  // iteration's x += alpha p (not on the first iteration).
  void (*spmm_pq)(const LevelArgs&, const void* z, void* p, void* q, void* x, const double* scal,
                  int first, double* part, int jac, hipStream_t);
  // Level-0 update and pre-smooth/residual/restrict:
  //   update: r_out = r_in - alpha q, x = (first ? 0 : x) + alpha p, partials |r_out|^2, sum x
  //   restrict (if nagg > 0): bc[I] = sum_{u in I} (b - L S b)_u with b = r_out, S = omega D^-1
  //   xf = 1: x is left to spmm_pq (x = 0 on the first iteration, p not
  //   read, no sum-x partials)
  void (*update_restrict)(const LevelArgs&, const void* r_in, const void* q, const void* p,
                          void* x, void* r_out, void* bc, const double* scal, int first,
                          int do_update, double* part_rr, double* part_cs, int xf, hipStream_t);
  // Coarse-level pre-smooth/residual/restrict from b (no update).
  void (*restrict_)(const LevelArgs&, const void* b, void* bc, hipStream_t);
  // Prolong + post-smooth: xt = S b + mu xc[agg], x = xt + S (b - L xt); partial b.x if part
  void (*prolong_smooth)(const LevelArgs&, const void* b, const void* xc, void* x,
                         double* part_rz, hipStream_t);
  // x = S b (Jacobi step from zero) on a level; partial b.x if part; zf = 1
  // stores x as bfloat16, zf = 2 as FP8 with per-row-slice scales (both
  // require part)
  void (*jacobi)(const LevelArgs&, const void* b, void* x, double* part, int zf, hipStream_t);
  // Jacobi-PCG update on level 0: r_out = r_in - alpha q, x += alpha p,
  // z = S r_out; partials |r_out|^2, sum x, r_out.z; zf = 1 stores z as
  // bfloat16, zf = 2 as FP8 with per-row-slice scales (z non-null); xf = 1
  // leaves x to spmm_pq (x = 0 on the first iteration, no sum-x partials)
  // and does not read p
  void (*update_jacobi)(const LevelArgs&, const void* r_in, const void* q, const void* p, void* x,
                        void* r_out, void* z, const double* scal, int first, double* prr,
                        double* pcs, double* prz, int zf, int xf, hipStream_t);
  // x += alpha p over n level-0 rows, partial column sums of x (grid
  // grid_for(n, rg)): the last update when spmm_pq carries them
  void (*xfinal)(int n, void* x, const void* p, const double* scal, double* pcs, hipStream_t);
  // Coarsest solve x = Lc^+ b (FP64 arithmetic); Lc^+ is nc_pad x nc_pad.
  void (*coarse)(int nc, int nc_pad, const double* pinv, const void* b, void* x, hipStream_t);
  // Partial dots b.x over n rows (for the single-level case).
  void (*dot)(int n, const void* a, const void* b, double* part, hipStream_t);
  // FP64 residual r = b - L x (x may be null = 0; FP64, or FP32 when
  // x_fp32); r_out of element type T; partial |r|^2.
  void (*residual64)(const LevelArgs& l64, const void* x, int x_fp32, RhsArgs rhs, void* r_out,
                     double* part_rr, hipStream_t);
  // x64 = (first ? 0 : x64) + d - cs/n  (d of element type T; cs from scal)
  void (*xupdate64)(int n, double* x64, const void* d, const double* scal, int first, hipStream_t);
  // Projection right-hand sides (Algorithm 1): Y[u, j] for systems i0 + j < k.
  // r (nullable): also Y in element type T and partial sums of Y^2 into
  // part.  Returns the rows of partial sums (the grid per column slice).
  int (*jl_rhs)(const LevelArgs& l64, const int* iperm, uint64_t seed, int64_t i0, int64_t k,
                double* Y, void* r, double* part, hipStream_t);
  // Per-row |x_u|^2 accumulated into N (double[n]); partial column sums
  // into part_cs when it is non-null.
  void (*jl_rownorm)(int n, const double* x64, int ncols, double* N, double* part_cs, hipStream_t);
  void (*zero)(void* p, size_t bytes, hipStream_t);
  // Elimination level, forward step over the kept rows (lf = the forward
  // operator, lf.n = kept rows): t = r + F r.  jac = 0 writes t to out and,
  // when part_rz is given, partial sums of t . t; jac = 1 writes z = sd1 * t
  // and partial sums of r . z; jac = 2 does the same with z stored as
  // bfloat16.  Partial-sum rows: elim_grid(lf.n).
  void (*elim_fwd)(const LevelArgs& lf, const void* r, void* out, const void* sd1, double* part_rz,
                   int jac, hipStream_t);
  // Elimination level, back substitution z_f = (r_f + sum_c w_fc z_c) / D_ff
  // for the eliminated rows, with partial sums of r . z over the eliminated
  // rows (allrows = 0) or over all rows (allrows = 1); grid = elim_grid.
  // bf = 1: z is held as bfloat16.
  void (*elim_back)(const LevelArgs& l0, const void* r, void* z, double* part_rz, int allrows,
                    int bf, hipStream_t);
  int (*elim_grid)(int units);
  // tp[u] += node throughput of the block's unit flows ps[j] -> pt[j] (rows,
  // -1 = unused column) summed over its first ncols columns; seg_part holds
  // double[nseg] scratch for heavy rows.
  void (*throughput)(const LevelArgs& l64, const double* x64, int ncols, const int* ps,
                     const int* pt, double* seg_part, double* tp, hipStream_t);
  // out[i] += |x_{a_i} - x_{b_i}|^2 over the first ncols columns
  void (*edge_sq)(int ne, const int* a, const int* b, const double* x64, int ncols, double* out,
                  hipStream_t);
};

// Tables for element type float (FP32 inner solver) and double.
const KernTable* kern_table(int W, bool fp64);
int grid_for(int units, int rows_per_block, int cap_scale = 1);

// Sum partials[g][W] over g (fixed order) into scal rows; op selects the
// scalar update (see Finalize in kern_impl.hpp).
enum FinOp { F_ALPHA = 0, F_RZINIT = 1, F_BETA = 2, F_R64 = 3, F_CS = 4 };
// host (nullable): device address of host-mapped memory [S_N][W] that also
// receives the S_RR and S_R64 rows, so the host reads them without a copy.
void finalize(int W, int op, int g0, const double* p0, int g1, const double* p1, int g2,
              const double* p2, double* scal, hipStream_t s, double* host = nullptr);
// out[j] = (first ? 0 : out[j]) + d[s_j, j] - d[t_j, j] for j < ncols (FP32
// d, FP64 sum; 0 where s_j or t_j is -1)
void pair_acc(int W, int ncols, const float* d, const int* ps, const int* pt, double* out, int first,
              hipStream_t s);
// out[j] = x64[s_j, j] - x64[t_j, j] for j < ncols
void pair_diff(int W, int ncols, const double* x64, const int* ps, const int* pt, double* out,
               hipStream_t s);
// out[i] = src[idx[i]] for i < q
void gather(int q, const double* src, const int* idx, double* out, hipStream_t s);
// out[i] = src[row[i] * W + col[i]]
void gather_rc(int64_t q, const double* src, int W, const int* row, const int* col, double* out,
               hipStream_t s);
// x64[u, j] = 0 for every row u and every column j with flag[j] != 0
void zero_cols(int n, int W, double* x64, const int* flag, hipStream_t s);
// plain streaming copy of `bytes` (16-byte non-temporal loads and stores)
void stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// fill with zero bytes by a kernel (graph-capture friendly)
void zero_fill(void* p, size_t bytes, hipStream_t s);
// sum of x[0..n) into *out (two kernels, fixed order)
void reduce_sum(int n, const double* x, double* part, double* out, hipStream_t s);

}  // namespace cfc
