// Serving loop: continuous batching of farness queries over resident graphs.
//
// Each registered graph keeps its hierarchy (and, when asked, a projection
// sketch) resident and gets a worker thread with its own HIP stream, so work
// for different graphs overlaps on the device.  A Sampling query becomes one
// right-hand side e_v - e_s per pivot (Sec. 5.1); its columns queue for the
// W column slots of the graph's solve block.  At every refinement-step
// boundary the worker computes the FP64 residual of all slots, harvests the
// columns that meet the tolerance (d_ER = x(v) - x(s)), frees their slots and
// refills them from the queue, so requests that arrive while others are in
// flight join the running block.  A projection query reads the resident
// sketch.  Slot workspaces are admitted against the server's device-memory
// budget; a graph without admission keeps its queries queued.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "kern.hpp"
#include "solver.hpp"

namespace cfc {

using Clock = std::chrono::steady_clock;

struct QueryState {
  uint64_t ticket = 0;
  int gid = 0, kind = 0;
  std::vector<int64_t> nodes;
  int64_t k = 0;
  uint64_t seed = 0;
  std::vector<double> sums;
  std::vector<int64_t> left;
  int64_t cols_left = 0;
  std::vector<double> far, clo;
  int status = CFC_OK;
  bool done = false;
  Clock::time_point t_arrive, t_done;
};

struct ColTask {
  QueryState* q = nullptr;
  int node = 0;
  int s_row = -1, t_row = -1;
};

struct ServerImpl;

struct GraphWorker {
  ServerImpl* srv = nullptr;
  Graph* g = nullptr;
  int gid = 0;
  int depth = 0;                    // V-cycle depth (autotuned at registration)
  double itol = 1e-4;               // inner tolerance floor (autotuned at registration)
  hipStream_t stream = nullptr;
  std::thread th;
  std::deque<ColTask> pending;      // guarded by srv->mu
  std::deque<QueryState*> jlq;      // guarded by srv->mu
  int64_t active = 0;               // worker-owned
  uint64_t reserved = 0;            // admitted workspace bytes
  void run();
};

struct ServerImpl {
  Ctx* ctx = nullptr;
  // Worker threads allocate slot workspaces through this context: plain
  // hipMalloc on the same device, never the caller's allocator callbacks
  // (which may call back into a host runtime from a foreign thread).
  Ctx wctx;
  cfc_server_opts opts{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_admit;
  std::vector<std::unique_ptr<GraphWorker>> graphs;
  std::unordered_map<uint64_t, std::unique_ptr<QueryState>> queries;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<double> lat;
  int64_t submitted = 0, completed = 0, open_queries = 0;
  Clock::time_point t_first, t_last;
  bool have_first = false;
  uint64_t admitted_bytes = 0;

  void complete(QueryState* q) {  // caller holds mu
    q->done = true;
    q->t_done = Clock::now();
    const double ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_arrive).count();
    lat.push_back(ms);
    completed++;
    open_queries--;
    t_last = q->t_done;
    cv_done.notify_all();
  }
};

static cfc_solve_params serve_params(const cfc_server_opts& o) {
  cfc_solve_params p = default_solve();
  p.tol = o.tol;
  p.block = o.slots;
  return p;
}

static uint64_t workspace_bytes(const Graph& g, int W) {
  uint64_t n = 0;
  for (const auto& l : g.D->lv) n += (uint64_t)l.n;
  const uint64_t n0 = (uint64_t)g.D->lv[0].n;
  return n0 * W * (6 * 4 + 8) + 2 * (n - n0) * W * 4 + (uint64_t)P_COUNT * kMaxGrid * W * 8 +
         heavy_partial_bytes(g, W);
}

void GraphWorker::run() {
  ServerImpl& S = *srv;
  (void)hipSetDevice(S.ctx->device);
  cfc_solve_params p = serve_params(S.opts);
  p.levels = depth;
  p.inner_tol = itol;
  const int W = p.block;
  std::unique_ptr<Solver> sol;
  std::vector<ColTask> slot(W);
  std::vector<char> busy(W, 0);
  std::vector<int> steps(W, 0), hp(2 * W, -1), flag(W, 0);
  std::vector<double> r64(W), dres(W);
  const uint64_t need = workspace_bytes(*g, W);
  for (;;) {
    std::vector<QueryState*> jl_now;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv_work.wait(lk, [&] { return S.stop || !pending.empty() || !jlq.empty() || active > 0; });
      if (S.stop) break;
      jl_now.assign(jlq.begin(), jlq.end());
      jlq.clear();
    }
    // projection queries: gather from the resident sketch
    for (QueryState* q : jl_now) {
      int rc = CFC_OK;
      try {
        q->far.resize(q->nodes.size());
        q->clo.resize(q->nodes.size());
        Graph& G = *g;
        if (S.opts.jl_k <= 0 || !G.jl.valid || G.jl.k != S.opts.jl_k || G.jl.seed != S.opts.seed)
          fail(CFC_E_STATE, "the server keeps no projection sketch for this graph");
        // jl_farness uses the context stream; serialise on it
        jl_farness(G, (int64_t)q->nodes.size(), q->nodes.data(), q->far.data(), q->clo.data(),
                   &S.wctx, stream);
      } catch (const Error& e) {
        rc = e.code;
      } catch (...) {
        rc = CFC_E_INTERNAL;
      }
      std::lock_guard<std::mutex> lk(S.mu);
      q->status = rc;
      S.complete(q);
    }
    bool has_pending;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      has_pending = !pending.empty();
    }
    if (!has_pending && active == 0) {
      if (sol && S.opts.hbm_budget) {  // idle: give the slot workspace back
        sol.reset();
        g->ws.clear();
        std::lock_guard<std::mutex> lk(S.mu);
        S.admitted_bytes -= reserved;
        reserved = 0;
        S.cv_admit.notify_all();
      }
      continue;
    }
    try {
      if (!sol) {
        {
          std::unique_lock<std::mutex> lk(S.mu);
          if (S.opts.hbm_budget) {
            if (need > S.opts.hbm_budget) fail(CFC_E_NOMEM, "slot workspace exceeds the server budget");
            S.cv_admit.wait(lk, [&] { return S.stop || S.admitted_bytes + need <= S.opts.hbm_budget; });
            if (S.stop) break;
          }
          S.admitted_bytes += need;
          reserved = need;
        }
        sol = std::make_unique<Solver>(*g, p, stream, &S.wctx);
        zero_fill(sol->ws->x64.p, sol->ws->x64.bytes, stream);
      }
      Workspace& w = *sol->ws;
      // refill free slots from the queue
      std::fill(flag.begin(), flag.end(), 0);
      bool changed = false;
      {
        std::lock_guard<std::mutex> lk(S.mu);
        for (int j = 0; j < W && !pending.empty(); ++j) {
          if (busy[j]) continue;
          slot[j] = pending.front();
          pending.pop_front();
          busy[j] = 1;
          steps[j] = 0;
          flag[j] = 1;
          active++;
          changed = true;
        }
      }
      for (int j = 0; j < W; ++j) {
        hp[j] = busy[j] ? slot[j].s_row : -1;
        hp[W + j] = busy[j] ? slot[j].t_row : -1;
      }
      int* ps = w.pairs.as<int>();
      int* pt = ps + W;
      int* dflag = pt + W;
      CFC_HIP(hipMemcpyAsync(ps, hp.data(), 2 * W * sizeof(int), hipMemcpyHostToDevice, stream));
      if (changed) {
        CFC_HIP(hipMemcpyAsync(dflag, flag.data(), W * sizeof(int), hipMemcpyHostToDevice, stream));
        zero_cols(w.la64.n, W, w.x64.as<double>(), dflag, stream);
      }
      // FP64 residual of every slot
      RhsArgs rhs;
      rhs.kind = 1;
      rhs.ps = ps;
      rhs.pt = pt;
      w.kt->residual64(w.la64, w.x64.p, 0, rhs, w.ra.p, w.part_ptr(P_PQ), stream);
      finalize(W, F_R64, w.kt->rows_grid(w.la64, w.la64.n), w.part_ptr(P_PQ), 0, nullptr, 0, nullptr,
               w.scal.as<double>(), stream, w.mirror_dev);
      sol->read_scal(S_R64, r64.data());
      // harvest converged (or failed) columns
      std::vector<int> fin;
      std::fill(flag.begin(), flag.end(), 0);
      double cur_max = 0;
      for (int j = 0; j < W; ++j) {
        if (!busy[j]) continue;
        const double rel = std::sqrt(r64[j] / 2.0);
        if (rel <= p.tol || !std::isfinite(rel) || steps[j] >= p.max_refine) fin.push_back(j);
        else cur_max = std::max(cur_max, rel);
      }
      if (!fin.empty()) {
        pair_diff(W, W, w.x64.as<double>(), ps, pt, w.dvec.as<double>(), stream);
        CFC_HIP(hipMemcpyAsync(w.pinned, w.dvec.p, W * sizeof(double), hipMemcpyDeviceToHost, stream));
        CFC_HIP(hipStreamSynchronize(stream));
        std::memcpy(dres.data(), w.pinned, W * sizeof(double));
        std::lock_guard<std::mutex> lk(S.mu);
        for (int j : fin) {
          QueryState* q = slot[j].q;
          const double rel = std::sqrt(r64[j] / 2.0);
          if (!(rel <= p.tol)) q->status = CFC_E_NOT_CONVERGED;
          q->sums[slot[j].node] += dres[j];
          q->cols_left--;
          if (--q->left[slot[j].node] == 0) {
            const double n = (double)g->n, kk = (double)q->k, sum = q->sums[slot[j].node];
            q->far[slot[j].node] = n / kk * sum;
            q->clo[slot[j].node] = sum > 0 ? (kk / n) * (n - 1) / sum : INFINITY;
          }
          if (q->cols_left == 0) S.complete(q);
          busy[j] = 0;
          flag[j] = 1;
          active--;
        }
        // freed slots restart from zero; refill (and a fresh residual) first
        CFC_HIP(hipMemcpyAsync(dflag, flag.data(), W * sizeof(int), hipMemcpyHostToDevice, stream));
        zero_cols(w.la64.n, W, w.x64.as<double>(), dflag, stream);
        for (int j : fin) hp[j] = hp[W + j] = -1;
        continue;
      }
      // one refinement step for every live slot, each aiming at its own
      // remaining reduction to tol
      const double aim = (p.precision == CFC_PREC_FP64 || p.inner_tol < 1e-6) ? 0.9 : 0.5;
      std::vector<double> itol(W, 0.5);
      for (int j = 0; j < W; ++j) {
        const double rel = std::sqrt(r64[j] / 2.0);
        const double relj = (busy[j] && rel > 0 && std::isfinite(rel)) ? rel : std::max(cur_max, 1e-300);
        itol[j] = std::min(0.5, std::max(p.inner_tol, aim * p.tol / relj));
      }
      sol->pcg(r64, itol, p.max_inner, 1);
      w.kt->xupdate64(w.la64.n, w.x64.as<double>(), w.x.p, w.scal.as<double>(), 0, stream);
      for (int j = 0; j < W; ++j)
        if (busy[j]) steps[j]++;
    } catch (const std::exception& ex) {
      // fail every query that has columns here
      const Error* ce = dynamic_cast<const Error*>(&ex);
      const int code = ce ? ce->code : CFC_E_INTERNAL;
      std::lock_guard<std::mutex> lk(S.mu);
      auto fail_q = [&](QueryState* q) {
        if (q->done) return;
        q->status = code;
        S.complete(q);
      };
      for (int j = 0; j < W; ++j)
        if (busy[j]) { fail_q(slot[j].q); busy[j] = 0; }
      active = 0;
      for (auto& t : pending) fail_q(t.q);
      pending.clear();
    }
  }
  (void)hipStreamSynchronize(stream);
  sol.reset();
  g->ws.clear();  // these were allocated through the server's context
}

}  // namespace cfc

using namespace cfc;

struct cfc_server : ServerImpl {};

static Graph* GG(cfc_graph* g) { return reinterpret_cast<Graph*>(g); }

extern "C" {

int cfc_server_create(cfc_ctx* ctx, const cfc_server_opts* o, cfc_server** out) {
  try {
    if (!ctx || !out) fail(CFC_E_INVALID, "NULL argument");
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (c->host_only()) fail(CFC_E_STATE, "server needs a device context");
    auto s = std::make_unique<cfc_server>();
    s->ctx = c;
    s->wctx.device = c->device;
    s->wctx.stream = c->stream;
    cfc_server_opts d{256, 4096, 256, 200, 1, 1e-6, 0};
    s->opts = o ? *o : d;
    if (!kern_table(s->opts.slots, false) || s->opts.slots < 32)
      fail(CFC_E_INVALID, "slots must be 32, 64, 128, 256 or 512");
    if (s->opts.max_queue < 1) fail(CFC_E_INVALID, "max_queue must be >= 1");
    if (!(s->opts.tol > 0 && s->opts.tol < 1)) fail(CFC_E_INVALID, "tol must be in (0, 1)");
    if (s->opts.sampling_k < 1) s->opts.sampling_k = 200;
    *out = s.release();
    return CFC_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return CFC_E_INTERNAL;
  }
}

int cfc_server_add_graph(cfc_server* s, cfc_graph* gh, int32_t* gid) {
  try {
    if (!s || !gh) fail(CFC_E_INVALID, "NULL argument");
    Graph* g = GG(gh);
    // direct calls on the graph hold g->mu; once the server is recorded they
    // are refused, so from here on only this call and then the worker
    // thread touch the graph's device state
    std::lock_guard<std::mutex> glk(g->mu);
    if (!g->D) fail(CFC_E_STATE, "hierarchy not built");
    if (g->ctx != s->ctx) fail(CFC_E_INVALID, "graph belongs to another context");
    const void* none = nullptr;
    if (!g->server.compare_exchange_strong(none, static_cast<const void*>(s)))
      fail(CFC_E_STATE, "graph is already registered with a server");
    struct Release {  // undo the claim if registration fails below
      Graph* g;
      bool keep = false;
      ~Release() { if (!keep) g->server.store(nullptr); }
    } rel{g};
    CFC_HIP(hipSetDevice(s->ctx->device));
    if (s->opts.jl_k > 0 && !(g->jl.valid && g->jl.k == s->opts.jl_k && g->jl.seed == s->opts.seed)) {
      cfc_solve_params p = default_solve();
      p.tol = s->opts.tol;
      jl_sketch(*g, s->opts.jl_k, s->opts.seed, p, nullptr);
    }
    auto w = std::make_unique<GraphWorker>();
    w->srv = s;
    w->g = g;
    {
      const cfc_solve_params tp = tune_params(*g, serve_params(s->opts), s->opts.slots);
      w->depth = tp.levels;
      w->itol = tp.inner_tol;
    }
    // workspaces the graph holds from direct calls (and the tuning runs) were
    // allocated with the caller's allocator: release them on this thread
    CFC_HIP(hipStreamSynchronize(s->ctx->stream));
    g->ws.clear();
    CFC_HIP(hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking));
    GraphWorker* wp = w.get();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      w->gid = (int)s->graphs.size();
      s->graphs.push_back(std::move(w));
    }
    rel.keep = true;
    wp->th = std::thread([wp] { wp->run(); });
    if (gid) *gid = wp->gid;
    return CFC_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return CFC_E_INTERNAL;
  }
}

int cfc_server_submit(cfc_server* s, const cfc_query* q, uint64_t* ticket) {
  try {
    if (!s || !q || !ticket) fail(CFC_E_INVALID, "NULL argument");
    if (q->nnodes < 1 || q->nnodes > 1024 || !q->nodes) fail(CFC_E_INVALID, "nnodes must be 1..1024");
    if (q->kind != CFC_QUERY_SAMPLING && q->kind != CFC_QUERY_JL) fail(CFC_E_INVALID, "bad query kind");
    GraphWorker* w;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (q->graph < 0 || q->graph >= (int)s->graphs.size()) fail(CFC_E_INVALID, "bad graph id");
      w = s->graphs[q->graph].get();
      if (s->open_queries >= s->opts.max_queue) fail(CFC_E_BUSY, "server queue full");
    }
    Graph* g = w->g;
    auto st = std::make_unique<QueryState>();
    st->gid = q->graph;
    st->kind = q->kind;
    st->nodes.assign(q->nodes, q->nodes + q->nnodes);
    for (int64_t v : st->nodes)
      if (v < 0 || v >= g->n) fail(CFC_E_INVALID, "node id out of range");
    st->seed = q->seed ? q->seed : s->opts.seed;
    st->k = std::min<int64_t>(q->k > 0 ? q->k : s->opts.sampling_k, g->n);
    st->far.assign(q->nnodes, 0.0);
    st->clo.assign(q->nnodes, 0.0);
    st->sums.assign(q->nnodes, 0.0);
    st->left.assign(q->nnodes, 0);
    st->t_arrive = Clock::now();
    std::vector<ColTask> cols;
    if (q->kind == CFC_QUERY_SAMPLING) {
      std::vector<int64_t> piv;
      for (int i = 0; i < q->nnodes; ++i) {
        sampling_pivots(st->seed, st->nodes[i], g->n, st->k, piv);
        for (int64_t x : piv) {
          if (x == st->nodes[i]) continue;
          ColTask c;
          c.q = st.get();
          c.node = i;
          c.s_row = g->H.perm[st->nodes[i]];
          c.t_row = g->H.perm[x];
          cols.push_back(c);
          st->left[i]++;
        }
        if (st->left[i] == 0) st->clo[i] = INFINITY;
      }
      st->cols_left = (int64_t)cols.size();
    }
    std::lock_guard<std::mutex> lk(s->mu);
    st->ticket = s->next_ticket++;
    *ticket = st->ticket;
    if (!s->have_first) {
      s->have_first = true;
      s->t_first = st->t_arrive;
    }
    s->submitted++;
    s->open_queries++;
    QueryState* raw = st.get();
    s->queries[raw->ticket] = std::move(st);
    if (raw->kind == CFC_QUERY_JL) {
      w->jlq.push_back(raw);
    } else if (raw->cols_left == 0) {
      s->complete(raw);
    } else {
      for (auto& c : cols) w->pending.push_back(c);
    }
    s->cv_work.notify_all();
    return CFC_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return CFC_E_INTERNAL;
  }
}

static int take_result(cfc_server* s, uint64_t ticket, cfc_result* r, std::unique_lock<std::mutex>& lk,
                       double timeout_ms) {
  auto it = s->queries.find(ticket);
  if (it == s->queries.end()) fail(CFC_E_INVALID, "unknown ticket");
  QueryState* q = it->second.get();
  if (!q->done && timeout_ms != 0) {
    auto pred = [&] { return q->done; };
    if (timeout_ms < 0) s->cv_done.wait(lk, pred);
    else s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), pred);
  }
  if (!q->done) return CFC_E_STATE;
  if (r) {
    r->status = q->status;
    r->nnodes = (int32_t)q->nodes.size();
    r->latency_ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_arrive).count();
    if (r->far) std::copy(q->far.begin(), q->far.end(), r->far);
    if (r->clo) std::copy(q->clo.begin(), q->clo.end(), r->clo);
  }
  s->queries.erase(it);
  return CFC_OK;
}

int cfc_server_poll(cfc_server* s, uint64_t ticket, cfc_result* r) {
  try {
    if (!s) fail(CFC_E_INVALID, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    int rc = take_result(s, ticket, r, lk, 0);
    if (rc == CFC_E_STATE) set_last_error("query pending");
    return rc;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  }
}

int cfc_server_wait(cfc_server* s, uint64_t ticket, double timeout_ms, cfc_result* r) {
  try {
    if (!s) fail(CFC_E_INVALID, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    int rc = take_result(s, ticket, r, lk, timeout_ms);
    if (rc == CFC_E_STATE) set_last_error("query still pending at timeout");
    return rc;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  }
}

int cfc_server_get_stats(cfc_server* s, cfc_server_stats* st) {
  try {
    if (!s || !st) fail(CFC_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(st, 0, sizeof(*st));
    st->submitted = s->submitted;
    st->completed = s->completed;
    int64_t q = 0, f = 0;
    for (auto& w : s->graphs) {
      q += (int64_t)w->pending.size() + (int64_t)w->jlq.size();
      f += w->active;
    }
    st->queued = q;
    st->in_flight = f;
    if (!s->lat.empty()) {
      std::vector<double> l = s->lat;
      std::sort(l.begin(), l.end());
      auto pct = [&](double pp) {
        const double pos = pp * (double)(l.size() - 1);
        const size_t i = (size_t)pos;
        const double fr = pos - (double)i;
        return i + 1 < l.size() ? l[i] * (1 - fr) + l[i + 1] * fr : l[i];
      };
      st->p50_ms = pct(0.50);
      st->p99_ms = pct(0.99);
      double m = 0;
      for (double x : l) m += x;
      st->mean_ms = m / (double)l.size();
      const double wall = std::chrono::duration<double>(s->t_last - s->t_first).count();
      st->queries_per_s = wall > 0 ? (double)s->completed / wall : 0.0;
    }
    st->device_bytes = s->admitted_bytes;
    return CFC_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  }
}

void cfc_server_destroy(cfc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_admit.notify_all();
  for (auto& w : s->graphs)
    if (w->th.joinable()) w->th.join();
  for (auto& w : s->graphs) {
    if (w->stream) {
      (void)hipStreamSynchronize(w->stream);
      (void)hipStreamDestroy(w->stream);
    }
    w->g->server.store(nullptr);  // direct calls are allowed again
  }
  delete s;
}

}  // extern "C"
