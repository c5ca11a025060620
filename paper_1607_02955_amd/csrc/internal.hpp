// Internal declarations of libcfc (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <cstdint>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/cfc.h"

namespace cfc {

// ---- errors -----------------------------------------------------------------
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
void set_last_error(const std::string& msg);
[[noreturn]] void fail(int code, const std::string& msg);

#define CFC_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      ::cfc::fail(CFC_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---- context ------------------------------------------------------------------
struct Ctx {
  int device = -1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  cfc_alloc_fn alloc = nullptr;
  cfc_free_fn free_fn = nullptr;
  void* user = nullptr;
  uint64_t budget = 0;
  std::atomic<uint64_t> in_use{0};
  std::mutex mu;  // serialises allocator callbacks
  bool host_only() const { return device < 0; }
  void* dalloc(size_t bytes);
  void dfree(void* p, size_t bytes);
};

// Device buffer owned through a context's allocator.
struct DBuf {
  Ctx* ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    reset();
    ctx = o.ctx; p = o.p; bytes = o.bytes;
    o.p = nullptr; o.bytes = 0;
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() {
    if (p && ctx) ctx->dfree(p, bytes);
    p = nullptr; bytes = 0;
  }
  void alloc(Ctx* c, size_t b) {
    reset();
    ctx = c;
    bytes = b;
    p = b ? c->dalloc(b) : nullptr;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---- host graph and hierarchy ---------------------------------------------------
struct HostLevel {
  int64_t n = 0;
  std::vector<int32_t> rowptr, col;  // off-diagonal pattern, both directions
  std::vector<double> w;             // conductances
  std::vector<double> deg;           // D_ii
  std::vector<int32_t> agg;          // row -> next-level node (empty on coarsest)
  std::vector<int32_t> aggptr;       // next-level node -> row range
  // Elimination level (nC > 0): rows [0, nC) are kept and are the next
  // level's rows; rows [nC, n) are eliminated.  Forward operator over kept
  // rows: fptr/fcol/fcoef (coefficient w_cf / d_f of eliminated row f);
  // eliminated row f: kept neighbours enb[CFC_ELIM_MAX_DEGREE (f - nC) + i]
  // (ascending, then -1) with conductances ew[...] and einv = 1 / d_f.
  int64_t nC = 0;
  std::vector<int32_t> fptr, fcol, enb;
  std::vector<double> fcoef, ew, einv;
  int64_t nnz() const { return (int64_t)col.size(); }
};

struct Hierarchy {
  std::vector<HostLevel> lv;
  std::vector<int32_t> perm;   // graph node -> level-0 row
  std::vector<int32_t> iperm;  // level-0 row -> graph node
  std::vector<double> cpinv;   // coarsest dense pseudoinverse (row-major)
  double omega = 0.8, mu = 1.5;
  double setup_ms = 0;
};

// Device copy of one level.
struct DevLevel {
  int n = 0, nnz = 0, nagg = 0;
  int nC = 0;  // elimination level: kept rows (see HostLevel)
  int light_nnz = 0, nheavy = 0, nseg = 0;  // heavy rows live in their own CSR
  DBuf rowptr, col, w32, w64, deg32, deg64, sdinv32, sdinv64, agg, aggptr;
  DBuf heavy, hseg, hptr, hcol, hw32, hw64, seg_e, seg_row;
  DBuf enb, ew32, ew64, einv32, einv64;  // eliminated rows
  bool unit = false;
  float omega32 = 0;
  double omega64 = 0;
};

struct DevHierarchy {
  std::vector<DevLevel> lv;
  DevLevel fwd;  // forward operator of an elimination level 0 (rows = kept rows)
  DBuf cpinv;   // n_c x n_c FP64
  DBuf iperm;   // level-0 row -> graph node (int32)
  DBuf perm;    // graph node -> level-0 row (int32)
  DBuf wgraph;  // level-0 original weights FP64 per nnz (for JL RHS), = w64 unless unit
  int nc = 0;
  uint64_t bytes = 0;
};

struct Workspace;  // solver buffers for one (W, precision)
struct JLSketch {
  int64_t k = 0;
  uint64_t seed = 0;
  DBuf N_dev;   // per level-0 row ||Z_.v||^2
  DBuf S2_dev;  // ||Z||_F^2 and reduction scratch
  double S2 = 0;
  bool valid = false;
};

struct Graph {
  Ctx* ctx = nullptr;
  int64_t n = 0, input_n = 0;
  std::vector<int64_t> orig;  // graph node -> input id
  std::vector<int64_t> eu, ev;  // canonical edges (graph ids, lo < hi)
  std::vector<double> ew;
  bool unit = true;
  // level-0 CSR in graph numbering
  std::vector<int32_t> rowptr, col;
  std::vector<double> w, deg;
  int32_t max_degree = 0;
  Hierarchy H;
  bool have_h = false;
  std::unique_ptr<DevHierarchy> D;
  std::vector<std::unique_ptr<Workspace>> ws;
  JLSketch jl;
  // autotuned (precision, requested W or 0, W, depth, one-step refinement)
  std::vector<std::array<int, 5>> tuned;
  std::mutex mu;
  // Server this graph is registered with (null when none).  While it is
  // set, the server's worker thread is the only user of the graph's device
  // state (workspaces, sketch), and direct calls are refused.
  std::atomic<const void*> server{nullptr};
  Graph();
  ~Graph();
};

// graph.cpp
Graph* load_graph(Ctx* ctx, int64_t n, int64_t m, const int64_t* u, const int64_t* v,
                  const double* w, uint32_t flags);
// Device bytes of a width-W workspace's heavy-row partial sums: the segment
// partials and per-row sums of every level and of the forward operator,
// FP64-sized, as the solver allocates them (for memory estimates).
uint64_t heavy_partial_bytes(const Graph& g, int W);
// hierarchy.cpp
void build_hierarchy(Graph& g, const cfc_setup_params& p);
void upload_hierarchy(Graph& g);
cfc_setup_params default_setup();
// noalloc.hip: look up this device's copy of the static staging array of
// cfc_farness_jl_static (the device must be current)
void noalloc_init(int device);
// rng host helpers
void sampling_pivots(uint64_t seed, int64_t node, int64_t n, int64_t k, std::vector<int64_t>& out);

}  // namespace cfc
