// Graph ingest: validation, canonical edge list, connectivity, CSR.
// The graph is undirected with conductance weights (Sec. 2); self-loops are
// ignored and, for disconnected input, the largest connected component is
// kept on request (Sec. 2 treats components separately; Sec. 6.3 uses LCCs).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.hpp"

namespace cfc {

namespace {
struct DSU {
  std::vector<int64_t> p;
  explicit DSU(int64_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
  int64_t find(int64_t x) {
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
    return x;
  }
  void unite(int64_t a, int64_t b) {
    a = find(a); b = find(b);
    if (a != b) p[std::max(a, b)] = std::min(a, b);
  }
};
}  // namespace

Graph* load_graph(Ctx* ctx, int64_t n, int64_t m, const int64_t* u, const int64_t* v,
                  const double* w, uint32_t flags) {
  if (n <= 0) fail(CFC_E_INVALID, "graph must have at least one node");
  if (n >= (int64_t(1) << 31) - 1) fail(CFC_E_INVALID, "more than 2^31-2 nodes");
  if (m < 0 || (m > 0 && (!u || !v))) fail(CFC_E_INVALID, "bad edge arrays");
  // canonical (lo, hi, w), self-loops dropped
  std::vector<std::pair<uint64_t, double>> e;
  e.reserve(m);
  for (int64_t i = 0; i < m; ++i) {
    int64_t a = u[i], b = v[i];
    if (a < 0 || a >= n || b < 0 || b >= n)
      fail(CFC_E_INVALID, "edge " + std::to_string(i) + " has an endpoint outside [0, n)");
    double wi = w ? w[i] : 1.0;
    if (!(std::isfinite(wi) && wi > 0))
      fail(CFC_E_INVALID, "edge " + std::to_string(i) + " has a weight that is not finite and > 0");
    if (a == b) continue;
    int64_t lo = std::min(a, b), hi = std::max(a, b);
    e.emplace_back((uint64_t(lo) << 32) | uint64_t(hi), wi);
  }
  std::sort(e.begin(), e.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  std::vector<std::pair<uint64_t, double>> c;
  c.reserve(e.size());
  for (auto& x : e) {
    if (!c.empty() && c.back().first == x.first) {
      if (flags & CFC_REJECT_PARALLEL) fail(CFC_E_INVALID, "repeated edge and CFC_REJECT_PARALLEL set");
      c.back().second += x.second;  // parallel conductances add
    } else {
      c.push_back(x);
    }
  }
  e.clear();
  e.shrink_to_fit();
  // components
  DSU d(n);
  for (auto& x : c) d.unite(int64_t(x.first >> 32), int64_t(x.first & 0xffffffffu));
  std::vector<int64_t> size(n, 0);
  for (int64_t i = 0; i < n; ++i) size[d.find(i)]++;
  int64_t best = 0;
  for (int64_t i = 0; i < n; ++i)
    if (size[i] > size[best]) best = i;
  auto g = std::make_unique<Graph>();
  g->ctx = ctx;
  g->input_n = n;
  std::vector<int64_t> newid(n, -1);
  if (size[best] != n) {
    if (!(flags & CFC_LCC_ONLY))
      fail(CFC_E_DISCONNECTED, "graph is not connected (" + std::to_string(size[best]) + " of " +
                                   std::to_string(n) + " nodes in the largest component); "
                                   "pass CFC_LCC_ONLY to keep it");
    for (int64_t i = 0; i < n; ++i)
      if (d.find(i) == best) { newid[i] = (int64_t)g->orig.size(); g->orig.push_back(i); }
  } else {
    g->orig.resize(n);
    std::iota(g->orig.begin(), g->orig.end(), 0);
    std::iota(newid.begin(), newid.end(), 0);
  }
  g->n = (int64_t)g->orig.size();
  for (auto& x : c) {
    int64_t a = newid[int64_t(x.first >> 32)], b = newid[int64_t(x.first & 0xffffffffu)];
    if (a < 0) continue;
    g->eu.push_back(a);
    g->ev.push_back(b);
    g->ew.push_back(x.second);
    if (x.second != 1.0) g->unit = false;
  }
  int64_t me = (int64_t)g->eu.size();
  if (2 * me >= (int64_t(1) << 31)) fail(CFC_E_INVALID, "more than 2^30 edges");
  // CSR, both directions, columns ascending within a row
  g->rowptr.assign(g->n + 1, 0);
  for (int64_t i = 0; i < me; ++i) { g->rowptr[g->eu[i] + 1]++; g->rowptr[g->ev[i] + 1]++; }
  for (int64_t i = 0; i < g->n; ++i) g->rowptr[i + 1] += g->rowptr[i];
  g->col.resize(2 * me);
  g->w.resize(2 * me);
  g->deg.assign(g->n, 0.0);
  std::vector<int32_t> pos(g->rowptr.begin(), g->rowptr.end() - 1);
  // edges are sorted by (lo, hi): emitting lo->hi in order keeps rows sorted
  // for the "hi" neighbours; the "lo" neighbours of row hi arrive in ascending
  // lo order as well because the list is sorted by lo first.
  for (int64_t i = 0; i < me; ++i) {
    int32_t a = (int32_t)g->eu[i], b = (int32_t)g->ev[i];
    g->col[pos[b]] = a; g->w[pos[b]++] = g->ew[i];
  }
  for (int64_t i = 0; i < me; ++i) {
    int32_t a = (int32_t)g->eu[i], b = (int32_t)g->ev[i];
    g->col[pos[a]] = b; g->w[pos[a]++] = g->ew[i];
  }
  for (int64_t r = 0; r < g->n; ++r) {
    double s = 0;
    for (int32_t k = g->rowptr[r]; k < g->rowptr[r + 1]; ++k) s += g->w[k];
    g->deg[r] = s;
    g->max_degree = std::max<int32_t>(g->max_degree, g->rowptr[r + 1] - g->rowptr[r]);
  }
  return g.release();
}

uint64_t heavy_partial_bytes(const Graph& g, int W) {
  uint64_t rows = 0;
  for (const DevLevel& d : g.D->lv) rows += (uint64_t)d.nseg + d.nheavy;
  if (g.D->lv[0].nC > 0) rows += (uint64_t)g.D->fwd.nseg + g.D->fwd.nheavy;
  return rows * W * 8;
}

}  // namespace cfc
