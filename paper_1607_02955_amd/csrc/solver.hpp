// Solver declarations.
#pragma once
#include <array>
#include <map>
#include <vector>

#include "internal.hpp"
#include "kern.hpp"

namespace cfc {

enum PartSlot { P_PQ = 0, P_RZ, P_RR, P_CS, P_COUNT };
enum ProfKernel { K_SPMM = 0, K_PROLONG0 = 1, K_RESTRICT0 = 2 };

// Device buffers for solving one block of W columns in one precision.
struct Workspace {
  int W = 0;
  bool fp64 = false;
  int nlev = 0;
  const KernTable* kt = nullptr;
  std::vector<LevelArgs> la;  // per level, element type of the inner solver
  LevelArgs la64;             // level 0 in FP64
  DBuf x, ra, rb, p, q, z;    // level 0, inner element type
  std::vector<DBuf> b, xl;    // levels >= 1: right-hand side and iterate
  std::vector<DBuf> hpart;    // per level: heavy-row segment partials
  std::vector<DBuf> hsum;     // per level: their sums per heavy row
  LevelArgs lf;               // forward operator of an elimination level 0
  DBuf fpart, fsum;           // its heavy-row segment partials and their row sums
  DBuf x64;                   // FP64 solution block
  DBuf rhs;                   // FP64 dense right-hand sides (on demand)
  DBuf r64;                   // FP64 residual kept between refinement steps (on demand)
  DBuf rt;                    // Schur mode: the residual folded onto the kept rows
  DBuf pairs;                 // int32 ps[W], pt[W], segment bounds
  DBuf part;                  // FP64 partial sums [P_COUNT][kMaxGrid][W]
  DBuf scal;                  // FP64 per-column scalars [S_N][W]
  DBuf dvec;                  // FP64 scratch for per-column outputs
  double* pinned = nullptr;   // pinned host staging
  double* mirror = nullptr;   // host-mapped [S_N][W]: S_RR, S_R64 as finalized
  double* mirror_dev = nullptr;  // its device address
  // fewest PCG iterations seen per (V-cycle depth, refinement step, inner
  // tolerance in quarter decades)
  std::map<std::array<int, 3>, int> min_its;
  ~Workspace();
  double* part_ptr(int which) const;
};

Workspace& get_workspace(Graph& g, int W, bool fp64, hipStream_t s, Ctx* mem = nullptr);

struct Solver {
  Graph* g;
  cfc_solve_params params;
  Workspace* ws = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int g_rz = 0, g_rr = 0, g_cs = 0;
  int nuse = 1;  // V-cycle depth
  bool bfz = false;  // Jacobi paths: z = M^-1 r stored as bfloat16 in ws->z
  bool zf8 = false;  // ... or, when the preconditioner is one Jacobi step, as FP8
  int zfmt() const { return bfz ? (zf8 ? 2 : 1) : 0; }
  // bytes per value of the stored z (FP8 adds its per-row-slice scale)
  double zbytes() const { return zf8 ? 1.0 + 4.0 * ws->kt->ns8 / ws->W : 2.0; }
  // Schur mode (level 0 an elimination level, depth two or more): the inner
  // CG runs on level 1, the Schur complement S, preconditioned by one
  // Jacobi step (depth two) or by the V-cycle from level 1; pcg() folds the
  // level-0 residual onto the kept rows first and back-substitutes the
  // eliminated rows of the correction after.
  bool schur = false;
  int base = 0;  // level the inner CG runs on (1 in Schur mode)
  bool jac_top = false;  // the preconditioner is one Jacobi step on level `base`
  void* r0 = nullptr;  // the inner CG's initial residual (ws.ra, or ws.rt in Schur mode)
  // Set by the caller of solve_block for pair right-hand sides: device
  // double[W] that receives x[s_j] - x[t_j] directly (FP32 Schur mode only;
  // pair_used tells whether the last block did so, else x64 holds x).
  double* pair_out = nullptr;
  bool pair_used = false;
  bool pairs_now = false;  // inside solve_block: the current block does
  // the residual buffer the iterations alternate with ws.rb: ws.ra, or in
  // Schur mode ws.rt, so that ws.ra keeps the level-0 residual
  void* r_alt() const { return schur ? ws->rt.p : ws->ra.p; }
  bool xfu = false;  // x updates applied by the product kernel
  bool multi_step = false;  // a block of this solve took more than one refinement step
  // FP32/FP64 blocks streamed by the level-0 CG update (r_in, q, x, p read;
  // x, r_out written; with xfu only r_in, q, r_out, and x = 0 the first time)
  double upd_blocks(bool first) const { return xfu ? (first ? 4 : 3) : (first ? 5 : 6); }
  // statistics
  int64_t columns = 0, converged = 0, inner_iters = 0, refine_steps = 0, blocks = 0;
  double max_rel = 0, bytes = 0;
  // kernel timing with HIP events on the launch stream (CFC_PROFILE=1)
  bool profile = false;
  bool debug = false;
  struct ProfEv {
    int kind;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<ProfEv> prof_ev;
  // Refinement step of the inner solve in progress (-1: unknown); with the
  // workspace's record of the fewest PCG iterations earlier inner solves
  // needed at that step (same depth and inner tolerance), convergence is
  // not tested, and the host not synchronised, before that count less one.
  int cur_step = -1;
  double prof_ms[3] = {0, 0, 0}, prof_bytes[3] = {0, 0, 0};
  int64_t prof_launches[3] = {0, 0, 0};

  // stream_override: launch stream (default: the context's); mem: context
  // whose allocator backs new workspaces (default: the graph's)
  Solver(Graph& g, const cfc_solve_params& p, hipStream_t stream_override = nullptr,
         Ctx* mem = nullptr);
  ~Solver();
  // HIP graphs of one PCG iteration each, r_b -> r_a ([0]) and r_a -> r_b
  // ([1]), built on first use and replayed alternately
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int64_t graph_replays = 0;
  double iter_bytes = 0;
  void iteration(bool first, void* r_in, void* r_out);
  void capture_iterations();
  void vcycle(bool update, bool first_x, const void* r_in, void* r_out);
  void vcycle_elim(bool update, bool first_x, const void* r_in, void* r_out);
  // itol[j]: the reduction of column j's residual norm the inner solve
  // stops at (columns with rr0[j] <= 0 are not tested)
  int pcg(const std::vector<double>& rr0, const std::vector<double>& itol, int max_inner, int check_every);
  int pcg_iterations(const std::vector<double>& rr0, const std::vector<double>& itol, int max_inner,
                     int check_every);
  void solve_block(const RhsArgs& rhs, int ncols, const cfc_solve_params& p, int32_t* status,
                   double* final_rel);
  void read_scal(int which, double* out);
  void prof_begin(int which);
  void prof_end(int which, double bytes);
  void prof_collect();
  void finish(cfc_solve_stats* st);
};

cfc_solve_params default_solve();
// CFC_E_INVALID unless every field of p is in range
void check_params(const cfc_solve_params& p);
// Fill in block width and V-cycle depth left at 0 (autotuner; cached in
// the graph and optionally on disk).
cfc_solve_params tune_params(Graph& g, const cfc_solve_params& p, int64_t ncols);

// Estimators (estimators.cpp)
void solve_dense(Graph& g, int64_t nrhs, const double* B, double* X, const cfc_solve_params& p,
                 cfc_solve_stats* st, int32_t* col_status);
// Solve e_{s_j} - e_{t_j} (graph ids) and return x(s_j) - x(t_j) per column.
void pair_solves(Graph& g, int64_t npairs, const int64_t* s, const int64_t* t, double* out,
                 const cfc_solve_params& p, cfc_solve_stats* st, int32_t* col_status);
void jl_sketch(Graph& g, int64_t k, uint64_t seed, const cfc_solve_params& p, cfc_solve_stats* st);
void jl_farness(Graph& g, int64_t q, const int64_t* nodes, double* far, double* clo,
                Ctx* mem = nullptr, hipStream_t stream = nullptr);

}  // namespace cfc
