// Multigrid hierarchy setup (host).
//
// The paper's solver builds coarser systems by aggregating nodes according to
// an affinity measure (Sec. 3.1); its details are not given there, so the
// design here is this library's own:
//   * affinity of an edge {u,v}: c_uv = <X_u, X_v>^2 / (|X_u|^2 |X_v|^2) over
//     K test vectors relaxed toward the near-null space of L;
//   * greedy aggregation in ascending-degree order: each free node joins its
//     strongest neighbour's aggregate (or founds one with a free neighbour)
//     while the aggregate has fewer than `agg_cap` nodes; a node whose
//     neighbours all sit in full aggregates joins an overflow aggregate keyed
//     by its strongest neighbour's aggregate;
//   * piecewise-constant interpolation P(u, I) = 1 iff u is in I and the
//     Galerkin operator P^T L P, which is again a graph Laplacian: the quotient
//     graph with W_IJ = sum of w_uv over u in I, v in J;
//   * a nested renumbering that makes every aggregate a contiguous row range
//     on every level (restriction and prolongation then need no atomics),
//     ordered along a Cuthill-McKee sweep of the fine graph so that
//     neighbouring rows stay close in memory;
//   * optionally first an elimination level (LAMG alternates elimination and
//     aggregation, Sec. 3.1): an independent set F of degree-1 and degree-2
//     nodes is removed exactly.  Ordering the kept nodes C first,
//     L = [L_CC L_CF; L_FC D_F] with D_F diagonal, and the Schur complement
//     L_CC - L_CF D_F^-1 L_FC is again a graph Laplacian on C: a degree-1 node
//     takes its edge with it, a degree-2 node with neighbours a, b is replaced
//     by the series edge {a, b} of conductance w_a w_b / (w_a + w_b);
//   * the coarsest level's dense pseudoinverse L_c^+ = Pi G Pi, with G the
//     inverse of L_c grounded at node 0 (Sec. 4, last paragraph) padded with
//     a zero row and column, and Pi = I - 11^T / n_c.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>

#include "internal.hpp"
#include "rng.hpp"
#include "setup.hpp"

namespace cfc {

// An aggregation level whose nnz + n exceeds this share of the level it
// coarsens is not given to the solver (the quotient graph keeps almost every
// edge: a cycle through it costs nearly a fine-level product and adds little).
constexpr double kMaxLevelRatio = 0.8;

cfc_setup_params default_setup() {
  cfc_setup_params p;
  p.coarsest_max = 512;
  p.agg_cap = 8;
  p.test_vectors = 8;
  p.relax_sweeps = 8;
  p.omega = 0.8;
  p.mu = 1.5;
  p.seed = 1;
  p.eliminate = 1;
  p.device = 1;
  p.order = 0;
  p.max_complexity_pct = 0;
  p.elim_degree = 0;
  p.nest = 0;
  return p;
}

namespace {

// Choose an independent set of low-degree nodes, degree 1 first, then 2, up
// to dmax (in id order within a degree), and form the Schur complement graph
// on the rest.  Returns false when the mode's threshold is not met (mode 1:
// at least 5% of the nodes).
bool eliminate(BLevel& B, int mode, int dmax, BLevel& R) {
  const int64_t n = B.n;
  if (mode == 0 || n < 3) return false;
  std::vector<char> blocked(n, 0);
  std::vector<int32_t> F;
  for (int d = 1; d <= dmax; ++d)
    for (int64_t u = 0; u < n; ++u) {
      if (blocked[u] || B.rowptr[u + 1] - B.rowptr[u] != d) continue;
      if (n - (int64_t)F.size() <= 2) break;  // keep at least two nodes
      F.push_back((int32_t)u);
      blocked[u] = 1;
      for (int32_t e = B.rowptr[u]; e < B.rowptr[u + 1]; ++e) blocked[B.col[e]] = 1;
    }
  if (F.empty() || (mode == 1 && (double)F.size() < 0.05 * (double)n)) return false;
  std::vector<char> isF(n, 0);
  for (int32_t f : F) isF[f] = 1;
  B.cidx.assign(n, -1);
  int64_t nc = 0;
  for (int64_t u = 0; u < n; ++u)
    if (!isF[u]) B.cidx[u] = (int32_t)nc++;
  R.n = nc;
  R.rowptr.assign(nc + 1, 0);
  R.deg.assign(nc, 0.0);
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t u = 0; u < n; ++u) {
    if (isF[u]) continue;
    row.clear();
    for (int32_t e = B.rowptr[u]; e < B.rowptr[u + 1]; ++e) {
      const int32_t v = B.col[e];
      if (!isF[v]) {
        row.emplace_back(B.cidx[v], B.w[e]);
        continue;
      }
      // eliminated neighbour v (all of its neighbours are kept): the Schur
      // complement joins u to each other neighbour o of v with conductance
      // w_uv w_vo / D_vv (a degree-1 v only lowers u's degree; degree 2 is
      // the series rule)
      for (int32_t o = B.rowptr[v]; o < B.rowptr[v + 1]; ++o)
        if (B.col[o] != u) row.emplace_back(B.cidx[B.col[o]], B.w[e] * B.w[o] / B.deg[v]);
    }
    std::sort(row.begin(), row.end());
    const int64_t c = B.cidx[u];
    for (size_t i = 0; i < row.size(); ++i) {
      if (i && row[i].first == row[i - 1].first) {
        R.w.back() += row[i].second;  // parallel conductances add
        continue;
      }
      R.col.push_back(row[i].first);
      R.w.push_back(row[i].second);
    }
    R.rowptr[c + 1] = (int32_t)R.col.size();
  }
  for (int64_t c = 0; c < nc; ++c) {
    double sacc = 0;
    for (int32_t e = R.rowptr[c]; e < R.rowptr[c + 1]; ++e) sacc += R.w[e];
    R.deg[c] = sacc;
  }
  B.F = std::move(F);
  B.nagg = nc;
  return true;
}

}  // namespace

// Affinity of every CSR entry e = (u, col[e]) of a level, times
// (1 + 1e-12 w_e) so that exact ties go to the heavier edge.  The device
// version (setup_dev.hip) performs the same FP64 operations in the same
// order, without contraction, and returns identical values.
std::vector<double> affinities(const BLevel& L, int level, const cfc_setup_params& p) {
  const int64_t n = L.n;
  const int K = std::max(1, p.test_vectors);
  // test vectors, node-major n x K
  std::vector<double> X(n * K), Y(n * K);
  for (int64_t u = 0; u < n; ++u)
    for (int k = 0; k < K; ++k) {
      uint64_t h = key_hash(p.seed, kTagTestVec, uint64_t(level) * 1024 + k, uint64_t(u));
      X[u * K + k] = double(h >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    }
  const double om = 0.6;
  for (int s = 0; s < p.relax_sweeps; ++s) {
    for (int64_t u = 0; u < n; ++u) {
      double acc[64];
      for (int k = 0; k < K; ++k) acc[k] = L.deg[u] * X[u * K + k];
      for (int32_t e = L.rowptr[u]; e < L.rowptr[u + 1]; ++e) {
        const double we = L.w[e];
        const double* xv = &X[int64_t(L.col[e]) * K];
        for (int k = 0; k < K; ++k) acc[k] -= we * xv[k];
      }
      const double sc = L.deg[u] > 0 ? om / L.deg[u] : 0.0;
      for (int k = 0; k < K; ++k) Y[u * K + k] = X[u * K + k] - sc * acc[k];
    }
    X.swap(Y);
  }
  for (int k = 0; k < K; ++k) {  // remove the constant component
    double s = 0;
    for (int64_t u = 0; u < n; ++u) s += X[u * K + k];
    s /= double(n);
    for (int64_t u = 0; u < n; ++u) X[u * K + k] -= s;
  }
  std::vector<double> nx(n);
  for (int64_t u = 0; u < n; ++u) {
    double s = 0;
    for (int k = 0; k < K; ++k) s += X[u * K + k] * X[u * K + k];
    nx[u] = s;
  }
  auto affinity = [&](int64_t u, int64_t v) {
    double s = 0;
    for (int k = 0; k < K; ++k) s += X[u * K + k] * X[v * K + k];
    double den = nx[u] * nx[v];
    return den > 0 ? s * s / den : 0.0;
  };
  std::vector<double> aff(L.col.size());
  for (int64_t u = 0; u < n; ++u)
    for (int32_t e = L.rowptr[u]; e < L.rowptr[u + 1]; ++e)
      aff[e] = affinity(u, L.col[e]) * (1.0 + 1e-12 * L.w[e]);
  return aff;
}

namespace {

// Greedy aggregation in ascending-degree order over precomputed affinities.
// Returns the number of aggregates.
int64_t aggregate(const BLevel& L, const std::vector<double>& aff, const cfc_setup_params& p,
                  std::vector<int32_t>& agg) {
  const int64_t n = L.n;
  std::vector<int64_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return (L.rowptr[a + 1] - L.rowptr[a]) < (L.rowptr[b + 1] - L.rowptr[b]);
  });
  agg.assign(n, -1);
  std::vector<int32_t> size;
  std::vector<int32_t> overflow;  // aggregate -> its open overflow aggregate (-1)
  const int cap = std::max(2, p.agg_cap);
  for (int64_t u : order) {
    if (agg[u] >= 0) continue;
    int64_t best = -1, strongest = -1;
    double bv = -1, sv = -1;
    for (int32_t e = L.rowptr[u]; e < L.rowptr[u + 1]; ++e) {
      int64_t v = L.col[e];
      const double a = aff[e];
      if (a > sv) { sv = a; strongest = v; }
      if (agg[v] >= 0 && size[agg[v]] >= cap) continue;
      if (a > bv) { bv = a; best = v; }
    }
    if (best >= 0) {
      if (agg[best] < 0) {
        int32_t id = (int32_t)size.size();
        size.push_back(2);
        overflow.push_back(-1);
        agg[u] = agg[best] = id;
      } else {
        agg[u] = agg[best];
        size[agg[best]]++;
      }
    } else if (strongest >= 0) {
      int32_t A = agg[strongest];
      int32_t o = overflow[A];
      if (o >= 0 && size[o] < cap) {
        agg[u] = o;
        size[o]++;
      } else {
        int32_t id = (int32_t)size.size();
        size.push_back(1);
        overflow.push_back(-1);
        overflow[A] = id;
        agg[u] = id;
      }
    } else {  // isolated node (only when n == 1)
      int32_t id = (int32_t)size.size();
      size.push_back(1);
      overflow.push_back(-1);
      agg[u] = id;
    }
  }
  return (int64_t)size.size();
}

// Galerkin quotient graph P^T L P for piecewise-constant P.
BLevel galerkin(const BLevel& F, const std::vector<int32_t>& agg, int64_t nc) {
  BLevel C;
  C.n = nc;
  std::vector<int32_t> start(nc + 1, 0), members(F.n);
  for (int64_t u = 0; u < F.n; ++u) start[agg[u] + 1]++;
  for (int64_t i = 0; i < nc; ++i) start[i + 1] += start[i];
  {
    std::vector<int32_t> pos(start.begin(), start.end() - 1);
    for (int64_t u = 0; u < F.n; ++u) members[pos[agg[u]]++] = (int32_t)u;
  }
  std::vector<int32_t> mark(nc, -1);
  std::vector<double> acc;
  std::vector<int32_t> cols;
  C.rowptr.assign(nc + 1, 0);
  for (int64_t I = 0; I < nc; ++I) {
    cols.clear();
    acc.clear();
    for (int32_t mi = start[I]; mi < start[I + 1]; ++mi) {
      int64_t u = members[mi];
      for (int32_t e = F.rowptr[u]; e < F.rowptr[u + 1]; ++e) {
        int32_t J = agg[F.col[e]];
        if (J == I) continue;
        if (mark[J] < 0) {
          mark[J] = (int32_t)cols.size();
          cols.push_back(J);
          acc.push_back(0.0);
        }
        acc[mark[J]] += F.w[e];
      }
    }
    std::vector<int32_t> idx(cols.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return cols[a] < cols[b]; });
    double d = 0;
    for (int i : idx) {
      C.col.push_back(cols[i]);
      C.w.push_back(acc[i]);
      d += acc[i];
    }
    C.deg.push_back(d);
    for (int32_t J : cols) mark[J] = -1;
    C.rowptr[I + 1] = (int32_t)C.col.size();
  }
  return C;
}

// Dense pseudoinverse of a connected graph Laplacian via the grounded inverse.
std::vector<double> laplacian_pinv(const BLevel& L) {
  const int64_t n = L.n;
  std::vector<double> out(n * n, 0.0);
  if (n <= 1) return out;
  const int64_t m = n - 1;  // ground node 0
  std::vector<double> A(m * m, 0.0);
  for (int64_t u = 1; u < n; ++u) {
    A[(u - 1) * m + (u - 1)] = L.deg[u];
    for (int32_t e = L.rowptr[u]; e < L.rowptr[u + 1]; ++e) {
      int64_t v = L.col[e];
      if (v >= 1) A[(u - 1) * m + (v - 1)] -= L.w[e];
    }
  }
  // Cholesky A = C C^T (lower), in place
  for (int64_t j = 0; j < m; ++j) {
    double s = A[j * m + j];
    for (int64_t k = 0; k < j; ++k) s -= A[j * m + k] * A[j * m + k];
    if (!(s > 0)) fail(CFC_E_INTERNAL, "coarsest grounded Laplacian is not positive definite");
    const double cjj = std::sqrt(s);
    A[j * m + j] = cjj;
    for (int64_t i = j + 1; i < m; ++i) {
      double t = A[i * m + j];
      for (int64_t k = 0; k < j; ++k) t -= A[i * m + k] * A[j * m + k];
      A[i * m + j] = t / cjj;
    }
  }
  // G = A^-1 = C^-T C^-1: invert C (lower) then form Cinv^T Cinv
  std::vector<double> Ci(m * m, 0.0);
  for (int64_t j = 0; j < m; ++j) {
    Ci[j * m + j] = 1.0 / A[j * m + j];
    for (int64_t i = j + 1; i < m; ++i) {
      double t = 0;
      for (int64_t k = j; k < i; ++k) t -= A[i * m + k] * Ci[k * m + j];
      Ci[i * m + j] = t / A[i * m + i];
    }
  }
  std::vector<double> G(n * n, 0.0);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      double t = 0;
      for (int64_t k = i; k < m; ++k) t += Ci[k * m + i] * Ci[k * m + j];
      G[(i + 1) * n + (j + 1)] = t;
      G[(j + 1) * n + (i + 1)] = t;
    }
  // L^+ = Pi G Pi
  std::vector<double> rs(n, 0.0);
  double tot = 0;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0;
    for (int64_t j = 0; j < n; ++j) s += G[i * n + j];
    rs[i] = s;
    tot += s;
  }
  const double inv = 1.0 / double(n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j)
      out[i * n + j] = G[i * n + j] - rs[i] * inv - rs[j] * inv + tot * inv * inv;
  return out;
}

// Cuthill-McKee sweep: breadth-first from a pseudo-peripheral node (the end
// of a few repeated BFS passes), neighbours visited in ascending degree.
// Returns the visit position of every node (every component is swept).
std::vector<int64_t> bfs_keys(const BLevel& L) {
  const int64_t n = L.n;
  std::vector<int64_t> key(n, -1), q;
  q.reserve(n);
  auto deg = [&](int64_t u) { return L.rowptr[u + 1] - L.rowptr[u]; };
  auto bfs = [&](int64_t root, std::vector<int64_t>& dist) {
    dist.assign(n, -1);
    std::vector<int64_t> qq{root};
    dist[root] = 0;
    int64_t last = root;
    for (size_t h = 0; h < qq.size(); ++h) {
      const int64_t u = qq[h];
      last = u;
      for (int32_t e = L.rowptr[u]; e < L.rowptr[u + 1]; ++e)
        if (dist[L.col[e]] < 0) {
          dist[L.col[e]] = dist[u] + 1;
          qq.push_back(L.col[e]);
        }
    }
    return last;
  };
  int64_t next = 0;
  std::vector<int64_t> dist, nb;
  for (int64_t start = 0; start < n; ++start) {
    if (key[start] >= 0) continue;
    int64_t root = start;
    for (int it = 0; it < 3; ++it) root = bfs(root, dist);  // pseudo-peripheral
    const size_t q0 = q.size();
    q.push_back(root);
    key[root] = next++;
    for (size_t h = q0; h < q.size(); ++h) {
      const int64_t u = q[h];
      nb.clear();
      for (int32_t e = L.rowptr[u]; e < L.rowptr[u + 1]; ++e)
        if (key[L.col[e]] < 0) nb.push_back(L.col[e]);
      std::sort(nb.begin(), nb.end(), [&](int64_t a, int64_t b) {
        return deg(a) != deg(b) ? deg(a) < deg(b) : a < b;
      });
      for (int64_t v : nb)
        if (key[v] < 0) {
          key[v] = next++;
          q.push_back(v);
        }
    }
  }
  return key;
}

}  // namespace

namespace {
void build_hierarchy_impl(Graph& g, const cfc_setup_params& p, bool on_device);
}

void build_hierarchy(Graph& g, const cfc_setup_params& p) {
  const bool on_device = p.device >= 1 && !g.ctx->host_only();
  try {
    build_hierarchy_impl(g, p, on_device);
  } catch (const Error& e) {
    // a device build that runs out of device memory falls back to the host
    // build (same hierarchy); anything else is reported
    if (!on_device || e.code != CFC_E_NOMEM) throw;
    build_hierarchy_impl(g, p, false);
  }
}

namespace {
void build_hierarchy_impl(Graph& g, const cfc_setup_params& p, bool on_device) {
  auto t0 = std::chrono::steady_clock::now();
  if (p.coarsest_max < 1 || p.coarsest_max > 4096) fail(CFC_E_INVALID, "coarsest_max must be in [1, 4096]");
  if (p.agg_cap < 2 || p.agg_cap > 64) fail(CFC_E_INVALID, "agg_cap must be in [2, 64]");
  if (p.test_vectors < 1 || p.test_vectors > 64) fail(CFC_E_INVALID, "test_vectors must be in [1, 64]");
  if (p.relax_sweeps < 0 || p.relax_sweeps > 100) fail(CFC_E_INVALID, "relax_sweeps must be in [0, 100]");
  if (!(p.omega > 0 && p.omega < 1)) fail(CFC_E_INVALID, "omega must be in (0, 1)");
  if (!(p.mu > 0 && p.mu < 2)) fail(CFC_E_INVALID, "mu must be in (0, 2)");
  if (p.eliminate < 0 || p.eliminate > 2) fail(CFC_E_INVALID, "eliminate must be 0, 1 or 2");
  if (p.nest < 0 || p.nest > 2) fail(CFC_E_INVALID, "nest must be 0, 1 or 2");
  if (p.elim_degree < 0 || p.elim_degree > CFC_ELIM_MAX_DEGREE)
    fail(CFC_E_INVALID, "elim_degree must be in [0, " + std::to_string(CFC_ELIM_MAX_DEGREE) + "]");
  const int elim_degree = p.elim_degree == 0 ? 4 : p.elim_degree;
  if (p.max_complexity_pct < -1 || (p.max_complexity_pct > 0 && p.max_complexity_pct < 100))
    fail(CFC_E_INVALID, "max_complexity_pct must be -1, 0 or at least 100");
  const double budget = p.max_complexity_pct < 0 ? 1e300 : (p.max_complexity_pct == 0 ? 2.0 : p.max_complexity_pct / 100.0);
  std::vector<BLevel> B(1);
  B[0].n = g.n;
  B[0].rowptr = g.rowptr;
  B[0].col = g.col;
  B[0].w = g.w;
  B[0].deg = g.deg;
  {
    BLevel R;
    if (B[0].n > p.coarsest_max && eliminate(B[0], p.eliminate, elim_degree, R)) B.push_back(std::move(R));
  }
  if (p.device < 0 || p.device > 2) fail(CFC_E_INVALID, "device must be 0, 1 or 2");
  if (p.order < 0 || p.order > 3) fail(CFC_E_INVALID, "order must be 0, 1, 2 or 3");
  std::unique_ptr<DeviceSetup> dev;
  std::vector<int> dh;  // device handle of each build level
  if (on_device) {
    dev = std::make_unique<DeviceSetup>(g.ctx);
    for (const BLevel& b : B) dh.push_back(dev->add(b));
  }
  const bool trace = std::getenv("CFC_DEBUG") != nullptr;
  auto ms_since = [](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
  };
  // operator complexity of the aggregation levels, in units of nnz + n of
  // the first level that is aggregated: behind an elimination level that is
  // the Schur complement graph, on which the solver iterates (a cycle over
  // the elimination level costs a fold and a back substitution, no product)
  const double unit0 = (double)B.back().col.size() + (double)B.back().n;
  double oc = 1.0;
  // Levels past the budget are not given to the solver (L_keep), but
  // aggregation may go on to coarsest_max anyway: the numbering then nests
  // aggregates of every level, a recursive clustering that keeps neighbours
  // close (BA-100k: 369 us per operator product with it, 497 us with the
  // numbering of the two levels the budget keeps; with its degree-4 nodes
  // eliminated, 69,754 against 63,321 solved columns/s).  On hub-dominated
  // graphs, whose rows above 256 entries hold a third or more of the
  // entries, the numbering of the kept levels alone is the faster one
  // (R-MAT-20 Sampling: 6,293 against 5,526 columns/s with every level).
  bool order_all = p.nest == 1;
  if (p.nest == 0) {
    int64_t hub_nnz = 0;
    for (int64_t u = 0; u < g.n; ++u) {
      const int64_t d = g.rowptr[u + 1] - g.rowptr[u];
      if (d > 256) hub_nnz += d;
    }
    order_all = 3 * hub_nnz < (int64_t)g.col.size();
  }
  // an aggregation level must shrink nnz + n by a fifth (no limit without a budget)
  const double ratio_cap = p.max_complexity_pct < 0 ? 1e300 : kMaxLevelRatio;
  int L_keep = 0;
  while (B.back().n > p.coarsest_max && (int)B.size() < CFC_MAX_LEVELS) {
    BLevel& F = B.back();
    std::vector<int32_t> agg;
    auto ta = std::chrono::steady_clock::now();
    const int lvl = (int)B.size() - 1;
    int64_t nc;
    if (dev && p.device == 2) {  // aggregation on the device too
      dev->affinities(dh[lvl], lvl, p, true);
      nc = dev->aggregate(dh[lvl], std::max(2, p.agg_cap), agg);
    } else {
      const std::vector<double> aff = dev ? dev->affinities(dh[lvl], lvl, p) : affinities(F, lvl, p);
      nc = aggregate(F, aff, p, agg);
    }
    const double t_agg = ms_since(ta);
    if (nc >= F.n) break;  // no progress (cannot happen on a connected graph with n >= 2)
    ta = std::chrono::steady_clock::now();
    BLevel C;
    int hc = -1;
    if (dev)
      hc = dev->galerkin(dh[lvl], agg, nc, C);
    else
      C = galerkin(F, agg, nc);
    if (trace)
      std::fprintf(stderr, "[cfc] setup level %d: n %lld nnz %zu -> %lld: aggregate %.0f ms, galerkin %.0f ms\n",
                   (int)B.size() - 1, (long long)F.n, F.col.size(), (long long)nc, t_agg, ms_since(ta));
    const double add = ((double)C.col.size() + (double)C.n) / unit0;
    const double ratio = ((double)C.col.size() + (double)C.n) / ((double)F.col.size() + (double)F.n);
    if (!L_keep && (oc + add > budget || ratio > ratio_cap)) {  // the level would cost more than the budget allows
      L_keep = (int)B.size();
      if (!order_all) break;
    }
    oc += add;
    if (dev) dh.push_back(hc);
    F.agg = std::move(agg);
    F.nagg = nc;
    B.push_back(std::move(C));
  }
  if (B.back().n > 4096 && !L_keep) fail(CFC_E_INTERNAL, "coarsening stalled above 4096 nodes");
  const int L = (int)B.size();             // levels that define the numbering
  const int LH = L_keep ? L_keep : L;      // levels the solver gets
  // Locality keys: level-0 nodes get their position in a Cuthill-McKee
  // (breadth-first, ascending degree) sweep from a pseudo-peripheral node; a
  // coarse node gets the smallest key of its aggregate.
  auto tk = std::chrono::steady_clock::now();
  std::vector<std::vector<int64_t>> key(L);
  int key_order = p.order;
  if (key_order == 0) {
    int64_t maxd = 0;
    for (int64_t u = 0; u < B[0].n; ++u) maxd = std::max<int64_t>(maxd, B[0].rowptr[u + 1] - B[0].rowptr[u]);
    const double mean = B[0].n ? (double)B[0].col.size() / (double)B[0].n : 0.0;
    key_order = (double)maxd > 32.0 * mean ? 3 : 1;
  }
  if (key_order == 1) {
    key[0] = bfs_keys(B[0]);
  } else {
    key[0].resize(B[0].n);
    for (int64_t u = 0; u < B[0].n; ++u)
      key[0][u] = key_order == 2 ? u : -(int64_t)(B[0].rowptr[u + 1] - B[0].rowptr[u]) * B[0].n + u;
  }
  for (int l = 0; l + 1 < L; ++l) {
    key[l + 1].assign(B[l + 1].n, INT64_MAX);
    for (int64_t u = 0; u < B[l].n; ++u) {
      const int32_t to = B[l].cidx.empty() ? B[l].agg[u] : B[l].cidx[u];
      if (to < 0) continue;
      int64_t& k = key[l + 1][to];
      k = std::min(k, key[l][u]);
    }
  }
  // nested renumbering, coarsest first: coarse nodes and the members of each
  // aggregate in key order, so every aggregate is a contiguous row range and
  // the numbering follows the sweep on every level
  std::vector<std::vector<int32_t>> order(L), newid(L);
  order[L - 1].resize(B[L - 1].n);
  std::iota(order[L - 1].begin(), order[L - 1].end(), 0);
  std::stable_sort(order[L - 1].begin(), order[L - 1].end(),
                   [&](int32_t a, int32_t b) { return key[L - 1][a] < key[L - 1][b]; });
  for (int l = L - 2; l >= 0; --l) {
    const BLevel& F = B[l];
    if (!F.cidx.empty()) {
      // elimination level: kept nodes in the next level's order, then the
      // eliminated ones next to their first neighbour
      std::vector<int32_t> cnode(B[l + 1].n);
      for (int64_t u = 0; u < F.n; ++u)
        if (F.cidx[u] >= 0) cnode[F.cidx[u]] = (int32_t)u;
      std::vector<int32_t> rowc(B[l + 1].n);
      for (int64_t i = 0; i < B[l + 1].n; ++i) rowc[order[l + 1][i]] = (int32_t)i;
      order[l].reserve(F.n);
      for (int32_t c : order[l + 1]) order[l].push_back(cnode[c]);
      std::vector<std::pair<int64_t, int32_t>> fk;
      for (int32_t f : F.F) fk.emplace_back((int64_t)rowc[F.cidx[F.col[F.rowptr[f]]]] * F.n + f, f);
      std::sort(fk.begin(), fk.end());
      for (auto& x : fk) order[l].push_back(x.second);
      continue;
    }
    std::vector<int32_t> start(F.nagg + 1, 0), mem(F.n);
    for (int64_t u = 0; u < F.n; ++u) start[F.agg[u] + 1]++;
    for (int64_t i = 0; i < F.nagg; ++i) start[i + 1] += start[i];
    std::vector<int32_t> pos(start.begin(), start.end() - 1);
    for (int64_t u = 0; u < F.n; ++u) mem[pos[F.agg[u]]++] = (int32_t)u;
    for (int64_t I = 0; I < F.nagg; ++I)
      std::stable_sort(mem.begin() + start[I], mem.begin() + start[I + 1],
                       [&](int32_t a, int32_t b) { return key[l][a] < key[l][b]; });
    order[l].reserve(F.n);
    for (int32_t I : order[l + 1])
      for (int32_t k = start[I]; k < start[I + 1]; ++k) order[l].push_back(mem[k]);
  }
  for (int l = 0; l < L; ++l) {
    newid[l].assign(B[l].n, -1);
    for (int64_t i = 0; i < B[l].n; ++i) newid[l][order[l][i]] = (int32_t)i;
  }
  Hierarchy H;
  H.omega = p.omega;
  H.mu = p.mu;
  H.lv.resize(LH);
  for (int l = 0; l < LH; ++l) {
    const BLevel& F = B[l];
    HostLevel& O = H.lv[l];
    O.n = F.n;
    O.rowptr.assign(F.n + 1, 0);
    O.col.reserve(F.col.size());
    O.w.reserve(F.w.size());
    O.deg.resize(F.n);
    if (dev) {
      dev->renumber(dh[l], newid[l], O.col, O.w);
      for (int64_t r = 0; r < F.n; ++r) {
        const int32_t old = order[l][r];
        O.rowptr[r + 1] = O.rowptr[r] + (F.rowptr[old + 1] - F.rowptr[old]);
        O.deg[r] = F.deg[old];
      }
    } else {
      std::vector<std::pair<int32_t, double>> row;
      for (int64_t r = 0; r < F.n; ++r) {
        int32_t old = order[l][r];
        row.clear();
        for (int32_t e = F.rowptr[old]; e < F.rowptr[old + 1]; ++e) row.emplace_back(newid[l][F.col[e]], F.w[e]);
        std::sort(row.begin(), row.end());
        for (auto& x : row) { O.col.push_back(x.first); O.w.push_back(x.second); }
        O.rowptr[r + 1] = (int32_t)O.col.size();
        O.deg[r] = F.deg[old];
      }
    }
    if (!F.cidx.empty()) {
      // forward operator over kept rows and the eliminated rows' neighbours
      const int64_t nc = F.nagg;
      O.nC = nc;
      O.fptr.assign(nc + 1, 0);
      O.enb.assign(CFC_ELIM_MAX_DEGREE * (F.n - nc), -1);
      O.ew.assign(CFC_ELIM_MAX_DEGREE * (F.n - nc), 0.0);
      O.einv.assign(F.n - nc, 0.0);
      std::vector<std::pair<int32_t, double>> fr;
      for (int64_t r = 0; r < F.n; ++r) {
        const int32_t old = order[l][r];
        if (r < nc) {
          fr.clear();
          for (int32_t e = F.rowptr[old]; e < F.rowptr[old + 1]; ++e) {
            const int32_t v = F.col[e];
            if (F.cidx[v] < 0) fr.emplace_back(newid[l][v], F.w[e] / F.deg[v]);
          }
          std::sort(fr.begin(), fr.end());
          for (auto& x : fr) { O.fcol.push_back(x.first); O.fcoef.push_back(x.second); }
          O.fptr[r + 1] = (int32_t)O.fcol.size();
        } else {
          const int64_t i = r - nc;
          fr.clear();
          for (int32_t e = F.rowptr[old]; e < F.rowptr[old + 1]; ++e)
            fr.emplace_back(newid[l][F.col[e]], F.w[e]);
          std::sort(fr.begin(), fr.end());
          for (size_t k = 0; k < fr.size(); ++k) {
            O.enb[CFC_ELIM_MAX_DEGREE * i + k] = fr[k].first;
            O.ew[CFC_ELIM_MAX_DEGREE * i + k] = fr[k].second;
          }
          O.einv[i] = 1.0 / F.deg[old];
        }
      }
      for (int64_t r = 0; r < nc; ++r)
        if (F.cidx[order[l][r]] < 0 || newid[l + 1][F.cidx[order[l][r]]] != r)
          fail(CFC_E_INTERNAL, "kept rows are not the next level's rows");
    } else if (l + 1 < LH) {
      O.agg.resize(F.n);
      for (int64_t r = 0; r < F.n; ++r) O.agg[r] = newid[l + 1][F.agg[order[l][r]]];
      O.aggptr.assign(F.nagg + 1, 0);
      for (int64_t r = 0; r < F.n; ++r) O.aggptr[O.agg[r] + 1]++;
      for (int64_t i = 0; i < F.nagg; ++i) O.aggptr[i + 1] += O.aggptr[i];
      for (int64_t r = 1; r < F.n; ++r)
        if (O.agg[r] < O.agg[r - 1]) fail(CFC_E_INTERNAL, "aggregates are not contiguous");
    }
  }
  if (trace) std::fprintf(stderr, "[cfc] setup ordering + level copies %.0f ms\n", ms_since(tk));
  // coarsest pseudoinverse in final numbering (none when the budget left
  // the deepest level above 4096 nodes: cycles end there with a Jacobi step)
  if (H.lv[LH - 1].n <= 4096) {
    BLevel C;
    C.n = H.lv[LH - 1].n;
    C.rowptr = H.lv[LH - 1].rowptr;
    C.col = H.lv[LH - 1].col;
    C.w = H.lv[LH - 1].w;
    C.deg = H.lv[LH - 1].deg;
    H.cpinv = laplacian_pinv(C);
  }
  H.perm = newid[0];
  H.iperm = order[0];
  H.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  g.H = std::move(H);
  g.have_h = true;
}
}  // namespace

}  // namespace cfc
