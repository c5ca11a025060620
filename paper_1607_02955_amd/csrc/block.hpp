// Layout kernels for dense right-hand-side blocks handed over in column-major
// order (one graph-node-order column per right-hand side): transposes into
// and out of the node-major n x W solver layout and per-column statistics.
#pragma once
#include <hip/hip_runtime.h>

namespace cfc {

// rhs[perm[v] W + j] = Bc[j n + v] for j < nc, 0 for nc <= j < W
// (perm: graph node -> level-0 row).
void block_in(int n, int W, int nc, const double* Bc, const int* perm, double* rhs, hipStream_t s);
// Xc[j n + v] = x[perm[v] W + j] - cs[j] / n for j < nc.
void block_out(int n, int W, int nc, const double* x, const int* perm, const double* cs, double* Xc,
               hipStream_t s);
// out[j] = sum of column j, out[W + j] = sum of its magnitudes, for a
// node-major n x W FP64 block; part is kColStatGrid x 2W scratch.  The sums
// run in a fixed order, so the result does not depend on timing.
constexpr int kColStatGrid = 256;
void col_stats(int n, int W, const double* x, double* part, double* out, hipStream_t s);

}  // namespace cfc
