// Further uses of the batched Laplacian solve:
//   shared-pivot Sampling -- one pivot set for every query node (Sec. 5.1
//                            read literally), k + q solves instead of k q;
//   spanning-edge centrality -- w_e d_ER(u, v) (Sec. 3.2), exact or from the
//                            projection sketch of Sec. 5.2;
//   current-flow betweenness -- node throughput of unit s-t currents (Sec. 3.2,
//                            electrical networks), summed over pairs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "centrality.hpp"
#include "kern.hpp"
#include "rng.hpp"
#include "solver.hpp"

namespace cfc {

namespace {

// Lemire's bounded integer from the words H(seed, tag, a, c), c = 0, 1, ...
struct Words {
  uint64_t seed, tag, a, c = 0;
  uint64_t next() { return key_hash(seed, tag, a, c++); }
  uint64_t bounded(uint64_t bound) {
    unsigned __int128 m = (unsigned __int128)next() * bound;
    uint64_t low = (uint64_t)m;
    if (low < bound) {
      const uint64_t t = (0 - bound) % bound;
      while (low < t) {
        m = (unsigned __int128)next() * bound;
        low = (uint64_t)m;
      }
    }
    return (uint64_t)(m >> 64);
  }
};

void check_nodes(const Graph& g, int64_t q, const int64_t* nodes) {
  if (q < 0 || (q > 0 && !nodes)) fail(CFC_E_INVALID, "bad node list");
  for (int64_t i = 0; i < q; ++i)
    if (nodes[i] < 0 || nodes[i] >= g.n) fail(CFC_E_INVALID, "node id out of range");
}

void require_converged(const std::vector<int32_t>& stat, int nc) {
  for (int j = 0; j < nc; ++j)
    if (stat[j] != CFC_COL_OK && stat[j] != CFC_COL_SKIPPED)
      fail(CFC_E_NOT_CONVERGED, "some solves missed the tolerance");
}

}  // namespace

void floyd_subset(uint64_t seed, uint64_t tag, uint64_t a, int64_t n, int64_t k,
                  std::vector<int64_t>& out) {
  k = std::min(k, n);
  Words wd{seed, tag, a};
  std::vector<int64_t> chosen;
  chosen.reserve(k);
  std::vector<char> in(k > 0 ? (size_t)n : 0, 0);
  for (int64_t j = n - k; j < n; ++j) {
    const int64_t t = (int64_t)wd.bounded(uint64_t(j) + 1);
    const int64_t pick = in[t] ? j : t;
    in[pick] = 1;
    chosen.push_back(pick);
  }
  std::sort(chosen.begin(), chosen.end());
  out = std::move(chosen);
}

void random_pairs(uint64_t seed, int64_t n, int64_t count, int64_t* s, int64_t* t) {
  for (int64_t i = 0; i < count; ++i) {
    Words wd{seed, kTagPairs, uint64_t(i)};
    const int64_t a = (int64_t)wd.bounded(uint64_t(n));
    const int64_t b = (int64_t)wd.bounded(uint64_t(n - 1));
    s[i] = a;
    t[i] = b + (b >= a ? 1 : 0);
  }
}

double edge_weight(const Graph& g, int64_t u, int64_t v, int64_t hint) {
  if (u < 0 || u >= g.n || v < 0 || v >= g.n || u == v) fail(CFC_E_INVALID, "not an edge of the graph");
  // edge lists passed in the graph's own canonical order hit directly
  if (hint >= 0 && hint < (int64_t)g.eu.size() &&
      ((g.eu[hint] == u && g.ev[hint] == v) || (g.eu[hint] == v && g.ev[hint] == u)))
    return g.ew[hint];
  // search the shorter of the two sorted rows
  if (g.rowptr[u + 1] - g.rowptr[u] > g.rowptr[v + 1] - g.rowptr[v]) std::swap(u, v);
  const int32_t* b = g.col.data() + g.rowptr[u];
  const int32_t* e = g.col.data() + g.rowptr[u + 1];
  const int32_t* it = std::lower_bound(b, e, (int32_t)v);
  if (it == e || *it != (int32_t)v) fail(CFC_E_INVALID, "not an edge of the graph");
  return g.w[it - g.col.data()];
}

// ---------------------------------------------------------------------------
// Shared-pivot Sampling.  With y_a = L^+ (e_a - e_r) for a fixed node r
// (the smallest pivot), d_ER(v, s) = (e_v - e_s)^T (y_v - y_s)
//   = y_v[v] - y_v[s] - y_s[v] + y_s[s],
// so sum_{s in S} d_ER(v, s) = k y_v[v] - sum_S y_v[s] - sum_S y_s[v] + sum_S y_s[s]
// needs one solve per node of S and Q (y_r = 0 needs none).

void shared_sampling(Graph& g, int64_t q, const int64_t* nodes, int64_t k, uint64_t seed, double* far,
                     double* clo, const cfc_solve_params& p0, cfc_solve_stats* st) {
  check_params(p0);
  check_nodes(g, q, nodes);
  if (k < 1) fail(CFC_E_INVALID, "k must be >= 1");
  if (q > 0 && !far) fail(CFC_E_INVALID, "far is NULL");
  const int64_t n = g.n;
  std::vector<int64_t> S;
  floyd_subset(seed, kTagShared, 0, n, k, S);
  const int64_t kk = (int64_t)S.size();
  const int64_t ref = S[0];
  std::vector<int64_t> cols;
  std::unordered_map<int64_t, int64_t> colof;
  auto add = [&](int64_t a) {
    if (a != ref && !colof.count(a)) {
      colof.emplace(a, (int64_t)cols.size());
      cols.push_back(a);
    }
  };
  for (int64_t s : S) add(s);
  for (int64_t i = 0; i < q; ++i) add(nodes[i]);
  std::unordered_map<int64_t, std::vector<int64_t>> qidx;  // node -> query positions
  for (int64_t i = 0; i < q; ++i) qidx[nodes[i]].push_back(i);

  std::vector<double> A(q, 0.0), B(q, 0.0), C(q, 0.0);
  double sumSS = 0;
  const int64_t ncols = (int64_t)cols.size();
  cfc_solve_params p = tune_params(g, p0, std::max<int64_t>(ncols, 1));
  Solver Sv(g, p);
  Workspace& w = *Sv.ws;
  const int W = w.W;
  int* ps = w.pairs.as<int>();
  int* pt = ps + W;
  std::vector<int> hp(2 * W);
  std::vector<int32_t> stat(W);
  // gathers of one block: (row, column) into x64 and where each value goes
  enum Dest { D_SS = 0, D_A, D_B, D_C };
  std::vector<int32_t> grow, gcol;
  std::vector<std::pair<int, int64_t>> dest;
  DBuf drow, dcol, dval;
  std::vector<double> val;
  const int rref = g.H.perm[ref];
  for (int64_t c0 = 0; c0 < ncols; c0 += W) {
    const int nc = (int)std::min<int64_t>(W, ncols - c0);
    for (int j = 0; j < W; ++j) {
      hp[j] = j < nc ? g.H.perm[cols[c0 + j]] : -1;
      hp[W + j] = j < nc ? rref : -1;
    }
    CFC_HIP(hipMemcpyAsync(ps, hp.data(), 2 * W * sizeof(int), hipMemcpyHostToDevice, Sv.stream));
    RhsArgs r;
    r.kind = 1;
    r.ps = ps;
    r.pt = pt;
    Sv.solve_block(r, nc, p, stat.data(), nullptr);
    require_converged(stat, nc);
    grow.clear();
    gcol.clear();
    dest.clear();
    auto want = [&](int64_t node, int j, int d, int64_t i) {
      grow.push_back(g.H.perm[node]);
      gcol.push_back(j);
      dest.emplace_back(d, i);
    };
    for (int j = 0; j < nc; ++j) {
      const int64_t a = cols[c0 + j];
      if (std::binary_search(S.begin(), S.end(), a)) {
        want(a, j, D_SS, 0);
        for (int64_t i = 0; i < q; ++i) want(nodes[i], j, D_C, i);
      }
      auto it = qidx.find(a);
      if (it != qidx.end())
        for (int64_t i : it->second) {
          want(a, j, D_A, i);
          for (int64_t s : S) want(s, j, D_B, i);
        }
    }
    const size_t ng = grow.size();
    if (!ng) continue;
    if (drow.bytes < ng * 4) {
      drow.alloc(g.ctx, ng * 4);
      dcol.alloc(g.ctx, ng * 4);
      dval.alloc(g.ctx, ng * 8);
    }
    CFC_HIP(hipMemcpyAsync(drow.p, grow.data(), ng * 4, hipMemcpyHostToDevice, Sv.stream));
    CFC_HIP(hipMemcpyAsync(dcol.p, gcol.data(), ng * 4, hipMemcpyHostToDevice, Sv.stream));
    gather_rc((int64_t)ng, w.x64.as<double>(), W, drow.as<int>(), dcol.as<int>(), dval.as<double>(),
              Sv.stream);
    val.resize(ng);
    CFC_HIP(hipMemcpyAsync(val.data(), dval.p, ng * 8, hipMemcpyDeviceToHost, Sv.stream));
    CFC_HIP(hipStreamSynchronize(Sv.stream));
    for (size_t i = 0; i < ng; ++i) {
      const double x = val[i];
      switch (dest[i].first) {
        case D_SS: sumSS += x; break;
        case D_A: A[dest[i].second] += x; break;
        case D_B: B[dest[i].second] += x; break;
        default: C[dest[i].second] += x; break;
      }
    }
  }
  Sv.finish(st);
  for (int64_t i = 0; i < q; ++i) {
    const double tot = double(kk) * A[i] - B[i] - C[i] + sumSS;
    far[i] = double(n) / double(kk) * tot;
    if (clo) clo[i] = tot > 0 ? (double(kk) / double(n)) * double(n - 1) / tot : INFINITY;
  }
}

// ---------------------------------------------------------------------------
// Spanning-edge centrality w_e d_ER(u, v)

void spanning_edge(Graph& g, int64_t ne, const int64_t* u, const int64_t* v, double* c,
                   const cfc_solve_params& p, cfc_solve_stats* st) {
  if (ne < 0 || (ne > 0 && (!u || !v || !c))) fail(CFC_E_INVALID, "bad edge list");
  std::vector<double> we(ne);
  for (int64_t i = 0; i < ne; ++i) we[i] = edge_weight(g, u[i], v[i], i);
  std::vector<int32_t> status(ne);
  pair_solves(g, ne, u, v, c, p, st, status.data());
  require_converged(status, (int)std::min<int64_t>(ne, INT32_MAX));
  for (int64_t i = 0; i < ne; ++i) c[i] *= we[i];
}

void spanning_edge_jl(Graph& g, int64_t ne, const int64_t* u, const int64_t* v, int64_t k,
                      uint64_t seed, double* c, const cfc_solve_params& p0, cfc_solve_stats* st) {
  check_params(p0);
  if (k < 1) fail(CFC_E_INVALID, "k must be >= 1");
  if (ne < 0 || (ne > 0 && (!u || !v || !c))) fail(CFC_E_INVALID, "bad edge list");
  if (ne > INT32_MAX) fail(CFC_E_INVALID, "too many edges");
  std::vector<double> we(ne);
  std::vector<int32_t> ea(ne), eb(ne);
  for (int64_t i = 0; i < ne; ++i) {
    we[i] = edge_weight(g, u[i], v[i], i);
    ea[i] = g.H.perm[u[i]];
    eb[i] = g.H.perm[v[i]];
  }
  cfc_solve_params p = tune_params(g, p0, k);
  const int n0 = g.D->lv[0].n;
  Solver S(g, p);
  Workspace& w = *S.ws;
  const int W = w.W;
  if (!w.rhs.p) w.rhs.alloc(g.ctx, (size_t)n0 * W * sizeof(double));
  DBuf da, db, dout;
  const size_t nb = (size_t)std::max<int64_t>(ne, 1);
  da.alloc(g.ctx, nb * 4);
  db.alloc(g.ctx, nb * 4);
  dout.alloc(g.ctx, nb * 8);
  if (ne) {
    CFC_HIP(hipMemcpyAsync(da.p, ea.data(), ne * 4, hipMemcpyHostToDevice, S.stream));
    CFC_HIP(hipMemcpyAsync(db.p, eb.data(), ne * 4, hipMemcpyHostToDevice, S.stream));
  }
  w.kt->zero(dout.p, nb * 8, S.stream);
  std::vector<int32_t> stat(W);
  for (int64_t i0 = 0; i0 < k; i0 += W) {
    const int nc = (int)std::min<int64_t>(W, k - i0);
    const int rows = w.kt->jl_rhs(w.la64, g.D->iperm.as<int>(), seed, i0, k, w.rhs.as<double>(), w.ra.p,
                                  w.part_ptr(P_PQ), S.stream);
    RhsArgs r;
    r.kind = 0;
    r.dense = w.rhs.as<double>();
    r.r0_rows = rows;
    S.solve_block(r, nc, p, stat.data(), nullptr);
    require_converged(stat, nc);
    w.kt->edge_sq((int)ne, da.as<int>(), db.as<int>(), w.x64.as<double>(), nc, dout.as<double>(),
                  S.stream);
    S.bytes += 2.0 * ne * W * 8 + 16.0 * ne;
  }
  if (ne) CFC_HIP(hipMemcpyAsync(c, dout.p, ne * 8, hipMemcpyDeviceToHost, S.stream));
  CFC_HIP(hipStreamSynchronize(S.stream));
  S.finish(st);
  for (int64_t i = 0; i < ne; ++i) c[i] *= we[i];
}

// ---------------------------------------------------------------------------
// Node throughput of unit currents: tau[v] = sum over pairs j with
// v not in {s_j, t_j} of 1/2 sum_{x in N(v)} w_vx |p_j(v) - p_j(x)|.

void current_throughput(Graph& g, int64_t npairs, const PairSource& pairs, double* tau,
                        const cfc_solve_params& p0, cfc_solve_stats* st) {
  check_params(p0);
  if (npairs < 0 || !tau) fail(CFC_E_INVALID, "bad arguments");
  cfc_solve_params p = tune_params(g, p0, std::max<int64_t>(npairs, 1));
  const int n0 = g.D->lv[0].n;
  Solver S(g, p);
  Workspace& w = *S.ws;
  const int W = w.W;
  int* ps = w.pairs.as<int>();
  int* pt = ps + W;
  DBuf tp, segp;
  tp.alloc(g.ctx, (size_t)n0 * 8);
  const int nseg = g.D->lv[0].nseg;
  if (nseg) segp.alloc(g.ctx, (size_t)nseg * 8);
  w.kt->zero(tp.p, (size_t)n0 * 8, S.stream);
  std::vector<int> hp(2 * W);
  std::vector<int32_t> stat(W);
  const int64_t n = g.n;
  for (int64_t c0 = 0; c0 < npairs; c0 += W) {
    const int nc = (int)std::min<int64_t>(W, npairs - c0);
    for (int j = 0; j < W; ++j) {
      hp[j] = hp[W + j] = -1;
      if (j >= nc) continue;
      int64_t s = 0, t = 0;
      pairs(c0 + j, s, t);
      if (s < 0 || s >= n || t < 0 || t >= n) fail(CFC_E_INVALID, "node id out of range");
      if (s == t) continue;  // no current
      hp[j] = g.H.perm[s];
      hp[W + j] = g.H.perm[t];
    }
    CFC_HIP(hipMemcpyAsync(ps, hp.data(), 2 * W * sizeof(int), hipMemcpyHostToDevice, S.stream));
    RhsArgs r;
    r.kind = 1;
    r.ps = ps;
    r.pt = pt;
    S.solve_block(r, nc, p, stat.data(), nullptr);
    require_converged(stat, nc);
    w.kt->throughput(w.la64, w.x64.as<double>(), nc, ps, pt, segp.as<double>(), tp.as<double>(),
                     S.stream);
    const DevLevel& d0 = g.D->lv[0];
    S.bytes += (double)n0 * W * 8 + 8.0 * d0.nnz * W + 12.0 * d0.nnz + 16.0 * n0;
  }
  std::vector<double> h(n0);
  CFC_HIP(hipMemcpyAsync(h.data(), tp.p, (size_t)n0 * 8, hipMemcpyDeviceToHost, S.stream));
  CFC_HIP(hipStreamSynchronize(S.stream));
  S.finish(st);
  for (int64_t x = 0; x < n; ++x) tau[x] = h[g.H.perm[x]];
}

}  // namespace cfc
