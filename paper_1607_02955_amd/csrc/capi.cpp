// extern "C" entry points of libcfc (declared in include/cfc.h).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"
#include "kern.hpp"
#include "rng.hpp"
#include "centrality.hpp"
#include "solver.hpp"

namespace cfc {

static thread_local std::string g_last_error;

void set_last_error(const std::string& m) { g_last_error = m; }
void fail(int code, const std::string& msg) { throw Error(code, msg); }

void* Ctx::dalloc(size_t bytes) {
  if (budget && in_use + bytes > budget)
    fail(CFC_E_NOMEM, "device budget exceeded (" + std::to_string(in_use + bytes) + " > " +
                          std::to_string(budget) + " bytes)");
  void* p = nullptr;
  if (alloc) {
    std::lock_guard<std::mutex> lk(mu);
    p = alloc(bytes, user);
    if (!p) fail(CFC_E_NOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(CFC_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  in_use += bytes;
  return p;
}

void Ctx::dfree(void* p, size_t bytes) {
  if (!p) return;
  if (free_fn) {
    std::lock_guard<std::mutex> lk(mu);
    free_fn(p, user);
  } else {
    (void)hipFree(p);
  }
  in_use -= bytes;
}

Graph::Graph() = default;

Graph::~Graph() {
  if (ctx && !ctx->host_only()) {
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  }
  ws.clear();
  jl = JLSketch();
  D.reset();
}

void sampling_pivots(uint64_t seed, int64_t node, int64_t n, int64_t k, std::vector<int64_t>& out) {
  floyd_subset(seed, kTagSample, uint64_t(node), n, k, out);
}

}  // namespace cfc

using namespace cfc;

#define CFC_TRY try {
#define CFC_CATCH                                                      \
  }                                                                    \
  catch (const Error& e) {                                             \
    set_last_error(e.what());                                          \
    return e.code;                                                     \
  }                                                                    \
  catch (const std::bad_alloc&) {                                      \
    set_last_error("host allocation failed");                          \
    return CFC_E_NOMEM;                                                \
  }                                                                    \
  catch (const std::exception& e) {                                    \
    set_last_error(e.what());                                          \
    return CFC_E_INTERNAL;                                             \
  }                                                                    \
  catch (...) {                                                        \
    set_last_error("unknown failure");                                 \
    return CFC_E_INTERNAL;                                             \
  }

// cfc_ctx is a real subclass of Ctx; cfc_graph stays an opaque handle to a Graph.
struct cfc_ctx : Ctx {};

static Graph* G(cfc_graph* g) { return reinterpret_cast<Graph*>(g); }
static const Graph* G(const cfc_graph* g) { return reinterpret_cast<const Graph*>(g); }

// A graph registered with a server is served by that server's worker
// thread alone until the server is destroyed.
static void not_served(const Graph* g) {
  if (g->server.load()) fail(CFC_E_STATE, "graph is registered with a server (destroy the server first)");
}

static void need_device(Graph* g) {
  not_served(g);
  if (g->ctx->host_only()) fail(CFC_E_STATE, "context has no device");
  if (!g->D) fail(CFC_E_STATE, "hierarchy not built (call cfc_hierarchy_build)");
  CFC_HIP(hipSetDevice(g->ctx->device));
}

extern "C" {

const char* cfc_last_error(void) { return g_last_error.c_str(); }
const char* cfc_version(void) { return "cfc 0.1.0 (gfx950)"; }

int cfc_ctx_create(const cfc_ctx_opts* o, cfc_ctx** out) {
  CFC_TRY
  if (!out) fail(CFC_E_INVALID, "out is NULL");
  *out = nullptr;
  auto c = std::make_unique<cfc_ctx>();
  if (o) {
    c->device = o->device;
    c->alloc = o->alloc;
    c->free_fn = o->free;
    c->user = o->user;
    c->budget = o->hbm_budget;
    if ((o->alloc == nullptr) != (o->free == nullptr)) fail(CFC_E_INVALID, "alloc and free must both be set");
  } else {
    c->device = 0;
  }
  if (c->device >= 0) {
    int nd = 0;
    CFC_HIP(hipGetDeviceCount(&nd));
    if (c->device >= nd) fail(CFC_E_INVALID, "no such device");
    CFC_HIP(hipSetDevice(c->device));
    noalloc_init(c->device);
    if (o && o->stream) {
      c->stream = static_cast<hipStream_t>(o->stream);
    } else {
      CFC_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
  }
  *out = c.release();
  return CFC_OK;
  CFC_CATCH
}

int cfc_device_copy(cfc_ctx* c, void* dst, const void* src, size_t bytes) {
  CFC_TRY
  if (!c || ((!dst || !src) && bytes)) fail(CFC_E_INVALID, "NULL argument");
  if (c->host_only()) fail(CFC_E_INVALID, "context has no device");
  CFC_HIP(hipSetDevice(c->device));
  stream_copy(dst, src, bytes, c->stream);
  CFC_HIP(hipGetLastError());
  CFC_HIP(hipStreamSynchronize(c->stream));
  return CFC_OK;
  CFC_CATCH
}

void cfc_ctx_destroy(cfc_ctx* c) {
  if (!c) return;
  if (c->own_stream && c->stream) {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

int cfc_graph_load(cfc_ctx* ctx, int64_t n, int64_t m, const int64_t* u, const int64_t* v,
                   const double* w, uint32_t flags, cfc_graph** out) {
  CFC_TRY
  if (!ctx || !out) fail(CFC_E_INVALID, "ctx/out is NULL");
  *out = nullptr;
  if (flags & ~(CFC_LCC_ONLY | CFC_REJECT_PARALLEL)) fail(CFC_E_INVALID, "unknown flags");
  Graph* g = load_graph(ctx, n, m, u, v, w, flags);
  *out = reinterpret_cast<cfc_graph*>(g);
  return CFC_OK;
  CFC_CATCH
}

int cfc_graph_get_info(const cfc_graph* gg, cfc_graph_info* out) {
  CFC_TRY
  if (!gg || !out) fail(CFC_E_INVALID, "NULL argument");
  const Graph* g = G(gg);
  std::memset(out, 0, sizeof(*out));
  out->n = g->n;
  out->m = (int64_t)g->eu.size();
  out->input_n = g->input_n;
  out->unit_weights = g->unit ? 1 : 0;
  out->max_degree = g->max_degree;
  if (g->have_h && g->H.lv[0].nC > 0) out->eliminated = (int32_t)(g->H.lv[0].n - g->H.lv[0].nC);
  if (g->have_h) {
    out->levels = (int32_t)g->H.lv.size();
    double num = 0, den = 0;
    for (size_t l = 0; l < g->H.lv.size(); ++l) {
      out->level_n[l] = g->H.lv[l].n;
      out->level_nnz[l] = g->H.lv[l].nnz();
      num += (double)g->H.lv[l].nnz() + (double)g->H.lv[l].n;
    }
    den = (double)g->H.lv[0].nnz() + (double)g->H.lv[0].n;
    out->operator_complexity = den > 0 ? num / den : 1.0;
    const size_t a = g->H.lv[0].nC > 0 ? 1 : 0;
    double cnum = 0;
    for (size_t l = a; l < g->H.lv.size(); ++l) cnum += (double)g->H.lv[l].nnz() + (double)g->H.lv[l].n;
    const double cden = (double)g->H.lv[a].nnz() + (double)g->H.lv[a].n;
    out->cycle_complexity = cden > 0 ? cnum / cden : 1.0;
    out->setup_ms = g->H.setup_ms;
  }
  if (g->D) out->device_bytes = g->D->bytes;
  for (auto& w : g->ws)
    for (const DBuf* b : {&w->x, &w->ra, &w->rb, &w->p, &w->q, &w->z, &w->x64, &w->rhs, &w->part})
      out->device_bytes += b->bytes;
  return CFC_OK;
  CFC_CATCH
}

int cfc_graph_node_map(const cfc_graph* gg, int64_t* orig) {
  CFC_TRY
  if (!gg || !orig) fail(CFC_E_INVALID, "NULL argument");
  const Graph* g = G(gg);
  std::copy(g->orig.begin(), g->orig.end(), orig);
  return CFC_OK;
  CFC_CATCH
}

void cfc_graph_destroy(cfc_graph* g) { delete G(g); }

int cfc_hierarchy_build(cfc_graph* gg, const cfc_setup_params* p) {
  CFC_TRY
  if (!gg) fail(CFC_E_INVALID, "graph is NULL");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  not_served(g);
  build_hierarchy(*g, p ? *p : default_setup());
  g->tuned.clear();
  if (!g->ctx->host_only()) upload_hierarchy(*g);
  return CFC_OK;
  CFC_CATCH
}

int cfc_hierarchy_level(const cfc_graph* gg, int32_t level, cfc_level_view* out) {
  CFC_TRY
  if (!gg || !out) fail(CFC_E_INVALID, "NULL argument");
  const Graph* g = G(gg);
  if (!g->have_h) fail(CFC_E_STATE, "hierarchy not built");
  if (level < 0 || level >= (int32_t)g->H.lv.size()) fail(CFC_E_INVALID, "level out of range");
  const HostLevel& h = g->H.lv[level];
  std::memset(out, 0, sizeof(*out));
  out->n = h.n;
  out->nnz = h.nnz();
  out->n_coarse = h.nC > 0 ? h.nC : (h.aggptr.empty() ? 0 : (int64_t)h.aggptr.size() - 1);
  out->elimination = h.nC > 0 ? 1 : 0;
  out->elim_nb = h.nC > 0 ? h.enb.data() : nullptr;
  out->row_ptr = h.rowptr.data();
  out->col = h.col.data();
  out->w = h.w.data();
  out->deg = h.deg.data();
  out->agg = h.agg.empty() ? nullptr : h.agg.data();
  out->agg_ptr = h.aggptr.empty() ? nullptr : h.aggptr.data();
  out->perm = level == 0 ? g->H.perm.data() : nullptr;
  out->coarse_pinv = (level + 1 == (int32_t)g->H.lv.size() && !g->H.cpinv.empty()) ? g->H.cpinv.data() : nullptr;
  return CFC_OK;
  CFC_CATCH
}

static cfc_solve_params params_or_default(const cfc_solve_params* p) {
  return p ? *p : default_solve();
}

int cfc_solve(cfc_graph* gg, int64_t nrhs, const double* B, double* X, const cfc_solve_params* p,
              cfc_solve_stats* st, int32_t* col_status) {
  CFC_TRY
  if (!gg) fail(CFC_E_INVALID, "graph is NULL");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (st) std::memset(st, 0, sizeof(*st));
  solve_dense(*g, nrhs, B, X, params_or_default(p), st, col_status);
  return CFC_OK;
  CFC_CATCH
}

int cfc_resistance(cfc_graph* gg, int64_t npairs, const int64_t* s, const int64_t* t, double* r,
                   const cfc_solve_params* p, cfc_solve_stats* st) {
  CFC_TRY
  if (!gg || npairs < 0 || (npairs > 0 && (!s || !t || !r))) fail(CFC_E_INVALID, "bad arguments");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (st) std::memset(st, 0, sizeof(*st));
  std::vector<int32_t> status(npairs);
  pair_solves(*g, npairs, s, t, r, params_or_default(p), st, status.data());
  for (auto x : status)
    if (x != CFC_COL_OK && x != CFC_COL_SKIPPED) fail(CFC_E_NOT_CONVERGED, "some solves missed the tolerance");
  return CFC_OK;
  CFC_CATCH
}

int cfc_farness_exact(cfc_graph* gg, int64_t q, const int64_t* nodes, double* far, double* clo,
                      const cfc_solve_params* p, cfc_solve_stats* st) {
  CFC_TRY
  if (!gg || q < 0 || (q > 0 && (!nodes || !far))) fail(CFC_E_INVALID, "bad arguments");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (st) std::memset(st, 0, sizeof(*st));
  const int64_t n = g->n;
  for (int64_t i = 0; i < q; ++i)
    if (nodes[i] < 0 || nodes[i] >= n) fail(CFC_E_INVALID, "node id out of range");
  std::vector<int64_t> s, t;
  for (int64_t i = 0; i < q; ++i)
    for (int64_t w = 0; w < n; ++w)
      if (w != nodes[i]) { s.push_back(nodes[i]); t.push_back(w); }
  std::vector<double> d(s.size());
  std::vector<int32_t> status(s.size());
  pair_solves(*g, (int64_t)s.size(), s.data(), t.data(), d.data(), params_or_default(p), st, status.data());
  for (auto x : status)
    if (x != CFC_COL_OK && x != CFC_COL_SKIPPED) fail(CFC_E_NOT_CONVERGED, "some solves missed the tolerance");
  for (int64_t i = 0; i < q; ++i) {
    double f = 0;
    for (int64_t j = i * (n - 1); j < (i + 1) * (n - 1); ++j) f += d[j];
    far[i] = f;
    if (clo) clo[i] = f > 0 ? double(n - 1) / f : INFINITY;
  }
  return CFC_OK;
  CFC_CATCH
}

int cfc_farness_sampling(cfc_graph* gg, int64_t q, const int64_t* nodes, int64_t k, uint64_t seed,
                         double* far, double* clo, const cfc_solve_params* p, cfc_solve_stats* st) {
  CFC_TRY
  if (!gg || q < 0 || k < 1 || (q > 0 && (!nodes || !far))) fail(CFC_E_INVALID, "bad arguments");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (st) std::memset(st, 0, sizeof(*st));
  const int64_t n = g->n;
  const int64_t kk = std::min(k, n);
  std::vector<int64_t> s, t, seg(q + 1, 0), piv;
  for (int64_t i = 0; i < q; ++i) {
    if (nodes[i] < 0 || nodes[i] >= n) fail(CFC_E_INVALID, "node id out of range");
    sampling_pivots(seed, nodes[i], n, kk, piv);
    for (int64_t x : piv)
      if (x != nodes[i]) { s.push_back(nodes[i]); t.push_back(x); }
    seg[i + 1] = (int64_t)s.size();
  }
  std::vector<double> d(s.size());
  std::vector<int32_t> status(s.size());
  pair_solves(*g, (int64_t)s.size(), s.data(), t.data(), d.data(), params_or_default(p), st, status.data());
  for (auto x : status)
    if (x != CFC_COL_OK && x != CFC_COL_SKIPPED) fail(CFC_E_NOT_CONVERGED, "some solves missed the tolerance");
  for (int64_t i = 0; i < q; ++i) {
    double sum = 0;
    for (int64_t j = seg[i]; j < seg[i + 1]; ++j) sum += d[j];
    far[i] = double(n) / double(kk) * sum;
    if (clo) clo[i] = sum > 0 ? (double(kk) / double(n)) * double(n - 1) / sum : INFINITY;
  }
  return CFC_OK;
  CFC_CATCH
}

int cfc_jl_sketch(cfc_graph* gg, int64_t k, uint64_t seed, const cfc_solve_params* p,
                  cfc_solve_stats* st) {
  CFC_TRY
  if (!gg) fail(CFC_E_INVALID, "graph is NULL");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (st) std::memset(st, 0, sizeof(*st));
  jl_sketch(*g, k, seed, params_or_default(p), st);
  return CFC_OK;
  CFC_CATCH
}

int cfc_farness_jl(cfc_graph* gg, int64_t q, const int64_t* nodes, double* far, double* clo) {
  CFC_TRY
  if (!gg) fail(CFC_E_INVALID, "graph is NULL");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (!nodes && q == g->n) {
    // every node, in graph-id order
    std::vector<int64_t> all(q);
    for (int64_t i = 0; i < q; ++i) all[i] = i;
    jl_farness(*g, q, all.data(), far, clo);
    return CFC_OK;
  }
  jl_farness(*g, q, nodes, far, clo);
  return CFC_OK;
  CFC_CATCH
}

int cfc_sampling_pivots(uint64_t seed, int64_t node, int64_t n, int64_t k, int64_t* out) {
  CFC_TRY
  if (n < 1 || k < 1 || node < 0 || node >= n || !out) fail(CFC_E_INVALID, "bad arguments");
  std::vector<int64_t> piv;
  sampling_pivots(seed, node, n, k, piv);
  std::copy(piv.begin(), piv.end(), out);
  return CFC_OK;
  CFC_CATCH
}

int cfc_farness_sampling_shared(cfc_graph* gg, int64_t q, const int64_t* nodes, int64_t k,
                                uint64_t seed, double* far, double* clo, const cfc_solve_params* p,
                                cfc_solve_stats* st) {
  CFC_TRY
  if (!gg) fail(CFC_E_INVALID, "graph is NULL");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (st) std::memset(st, 0, sizeof(*st));
  shared_sampling(*g, q, nodes, k, seed, far, clo, params_or_default(p), st);
  return CFC_OK;
  CFC_CATCH
}

int cfc_spanning_edge(cfc_graph* gg, int64_t ne, const int64_t* u, const int64_t* v, double* c,
                      const cfc_solve_params* p, cfc_solve_stats* st) {
  CFC_TRY
  if (!gg) fail(CFC_E_INVALID, "graph is NULL");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (st) std::memset(st, 0, sizeof(*st));
  spanning_edge(*g, ne, u, v, c, params_or_default(p), st);
  return CFC_OK;
  CFC_CATCH
}

int cfc_spanning_edge_jl(cfc_graph* gg, int64_t ne, const int64_t* u, const int64_t* v, int64_t k,
                         uint64_t seed, double* c, const cfc_solve_params* p, cfc_solve_stats* st) {
  CFC_TRY
  if (!gg) fail(CFC_E_INVALID, "graph is NULL");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (st) std::memset(st, 0, sizeof(*st));
  spanning_edge_jl(*g, ne, u, v, k, seed, c, params_or_default(p), st);
  return CFC_OK;
  CFC_CATCH
}

int cfc_current_throughput(cfc_graph* gg, int64_t npairs, const int64_t* s, const int64_t* t,
                           double* tau, const cfc_solve_params* p, cfc_solve_stats* st) {
  CFC_TRY
  if (!gg) fail(CFC_E_INVALID, "graph is NULL");
  if (npairs < 0 || (npairs > 0 && (!s || !t))) fail(CFC_E_INVALID, "bad pair list");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (st) std::memset(st, 0, sizeof(*st));
  current_throughput(*g, npairs, [&](int64_t j, int64_t& a, int64_t& b) { a = s[j]; b = t[j]; }, tau,
                     params_or_default(p), st);
  return CFC_OK;
  CFC_CATCH
}

int cfc_cfb_sampled(cfc_graph* gg, int64_t count, uint64_t seed, double* cb,
                    const cfc_solve_params* p, cfc_solve_stats* st) {
  CFC_TRY
  if (!gg) fail(CFC_E_INVALID, "graph is NULL");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  if (g->n < 3) fail(CFC_E_INVALID, "betweenness needs n >= 3");
  if (count < 1 || !cb) fail(CFC_E_INVALID, "bad arguments");
  if (st) std::memset(st, 0, sizeof(*st));
  std::vector<int64_t> s(count), t(count);
  random_pairs(seed, g->n, count, s.data(), t.data());
  current_throughput(*g, count, [&](int64_t j, int64_t& a, int64_t& b) { a = s[j]; b = t[j]; }, cb,
                     params_or_default(p), st);
  const double n = (double)g->n, scale = n / (n - 2.0) / (double)count;
  for (int64_t v = 0; v < g->n; ++v) cb[v] *= scale;
  return CFC_OK;
  CFC_CATCH
}

int cfc_cfb_exact(cfc_graph* gg, double* cb, const cfc_solve_params* p, cfc_solve_stats* st) {
  CFC_TRY
  if (!gg) fail(CFC_E_INVALID, "graph is NULL");
  Graph* g = G(gg);
  std::lock_guard<std::mutex> lk(g->mu);
  need_device(g);
  const int64_t n = g->n;
  if (n < 3) fail(CFC_E_INVALID, "betweenness needs n >= 3");
  if (!cb) fail(CFC_E_INVALID, "cb is NULL");
  if (st) std::memset(st, 0, sizeof(*st));
  // pair j of the C(n, 2) pairs s < t in row-major order of the upper triangle
  int64_t cs = 0, ct = 1;
  int64_t next = 0;
  current_throughput(*g, n * (n - 1) / 2,
                     [&](int64_t j, int64_t& a, int64_t& b) {
                       if (j != next) fail(CFC_E_INTERNAL, "pairs out of order");
                       a = cs;
                       b = ct;
                       ++next;
                       if (++ct == n) { ++cs; ct = cs + 1; }
                     },
                     cb, params_or_default(p), st);
  const double norm = 2.0 / ((double)(n - 1) * (double)(n - 2));
  for (int64_t v = 0; v < n; ++v) cb[v] *= norm;
  return CFC_OK;
  CFC_CATCH
}

int cfc_shared_pivots(uint64_t seed, int64_t n, int64_t k, int64_t* out) {
  CFC_TRY
  if (n < 1 || k < 1 || !out) fail(CFC_E_INVALID, "bad arguments");
  std::vector<int64_t> piv;
  floyd_subset(seed, kTagShared, 0, n, k, piv);
  std::copy(piv.begin(), piv.end(), out);
  return CFC_OK;
  CFC_CATCH
}

int cfc_random_pairs(uint64_t seed, int64_t n, int64_t count, int64_t* s, int64_t* t) {
  CFC_TRY
  if (n < 2 || count < 0 || (count > 0 && (!s || !t))) fail(CFC_E_INVALID, "bad arguments");
  random_pairs(seed, n, count, s, t);
  return CFC_OK;
  CFC_CATCH
}

uint64_t cfc_jl_sign_word(uint64_t seed, uint64_t word, int64_t lo, int64_t hi) {
  return jl_word(seed, word, uint64_t(lo), uint64_t(hi));
}

}  // extern "C"
