// Hierarchy setup shared by the host build (hierarchy.cpp) and the device
// build (setup_dev.hip).
#pragma once
#include <memory>
#include <vector>

#include "internal.hpp"

namespace cfc {

constexpr uint64_t kTagTestVec = 0x5456ull;

struct BLevel {  // a level in build numbering
  int64_t n = 0;
  std::vector<int32_t> rowptr, col;
  std::vector<double> w, deg;
  std::vector<int32_t> agg;  // to next level (build numbering)
  int64_t nagg = 0;
  // elimination level: cidx[u] = u's node on the next level, -1 if eliminated
  std::vector<int32_t> cidx;
  std::vector<int32_t> F;    // eliminated nodes
};

// Affinity of every CSR entry e = (u, col[e]): <X_u, X_v>^2 / (|X_u|^2 |X_v|^2)
// over the relaxed test vectors, times (1 + 1e-12 w_e).
std::vector<double> affinities(const BLevel& L, int level, const cfc_setup_params& p);

// Device copies of the build levels and the setup steps that run on them:
// affinities, Galerkin products and the final renumbering.  Every result is
// bit-identical to the host build (same FP64 operations in the same order,
// no contraction; sums over a coarse edge or row run in the host's order).
class DeviceSetup {
 public:
  explicit DeviceSetup(Ctx* ctx);
  ~DeviceSetup();
  // upload a level's CSR; returns its handle
  int add(const BLevel& L);
  // keep = true: leave them on the device for aggregate() (nothing returned)
  std::vector<double> affinities(int lv, int level, const cfc_setup_params& p, bool keep = false);
  // parallel aggregation of level lv over its kept affinities: handshake
  // matching rounds, every unmatched node joining its strongest matched
  // neighbour's aggregate, then two rounds of handshake matching between
  // aggregates (merged size at most cap); agg (host) numbers the aggregates
  // in the order of their roots.  Returns their number.
  int64_t aggregate(int lv, int cap, std::vector<int32_t>& agg);
  // quotient graph of level lv under agg (host array), downloaded into C and
  // kept on the device; returns its handle
  int galerkin(int lv, const std::vector<int32_t>& agg, int64_t nc, BLevel& C);
  // columns and weights of level lv renumbered by newid, rows in new order
  // and columns ascending within a row
  void renumber(int lv, const std::vector<int32_t>& newid, std::vector<int32_t>& col,
                std::vector<double>& w);
  struct Impl;

 private:
  std::unique_ptr<Impl> d;
};

}  // namespace cfc
