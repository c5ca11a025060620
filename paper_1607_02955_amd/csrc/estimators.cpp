// Right-hand-side blocks for the paper's three ways of computing farness and
// the reductions that turn block solutions into resistances and farness:
//   exact     -- n-1 systems L p = e_v - e_w per node (Sec. 4, Eq. 3);
//   Sampling  -- k pivots per node, (n/k) sum of d_ER(v, s) (Sec. 5.1);
//   projection -- k systems L z_i = (Q W^(1/2) B)_i (Sec. 5.2, Algorithm 1).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

#include "block.hpp"
#include "kern.hpp"
#include "solver.hpp"

namespace cfc {

cfc_solve_params default_solve() {
  cfc_solve_params p;
  p.tol = 1e-6;
  p.precision = CFC_PREC_MIXED;
  p.block = 0;
  p.max_refine = 20;
  p.max_inner = 300;
  p.inner_tol = 0;  // autotuned
  p.use_graph = 0;
  p.check_every = 1;
  p.levels = 0;
  p.pad = 0;
  return p;
}

static bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

void check_params(const cfc_solve_params& p) {
  if (!(p.tol > 0 && p.tol < 1)) fail(CFC_E_INVALID, "tol must be in (0, 1)");
  if (p.precision != CFC_PREC_MIXED && p.precision != CFC_PREC_FP64) fail(CFC_E_INVALID, "bad precision");
  if (p.max_refine < 0 || p.max_inner < 1) fail(CFC_E_INVALID, "bad iteration limits");
  if (!(p.inner_tol >= 0 && p.inner_tol < 1)) fail(CFC_E_INVALID, "inner_tol must be in [0, 1)");
  if (p.block != 0 && !kern_table(p.block, false)) fail(CFC_E_INVALID, "block must be 0, 1, 32, 64, 128, 256 or 512");
  if (p.levels < 0 || p.levels > CFC_MAX_LEVELS) fail(CFC_E_INVALID, "levels must be in [0, 32]");
}

// ---------------------------------------------------------------------------
// Autotuner: the block width W and the V-cycle depth that minimise device
// time per solved column.  Each candidate solves W sample pair right-hand
// sides for one refinement step (to the reduction a real inner solve is
// asked for, at most 200 PCG iterations) twice with one solver, and is
// scored by the second block's time / (W * decades of residual
// reduction).  Depth is chosen first at W = 256 (or the fixed W), then W
// at that depth, then (inner_tol = 0) the refinement split (tune_split
// below).  Results are cached in the graph and, when CFC_TUNE_CACHE names
// a file, on disk as "n nnz levels precision requested-W W depth one-step"
// lines.

static std::string tune_key(const Graph& g, int prec) {
  std::ostringstream o;
  o << g.n << ' ' << g.col.size() << ' ' << g.H.lv.size() << ' ' << prec;
  return o.str();
}

static double tune_score(Graph& g, const cfc_solve_params& p0, int W, int depth) {
  cfc_solve_params p = p0;
  p.block = W;
  p.levels = depth;
  p.max_refine = 1;
  p.max_inner = 200;
  p.check_every = 4;
  // the reduction the real solves ask of an inner solve: 1e-4 for FP32 (the
  // floor of the first of two refinement steps, with no outer tolerance to
  // stop at), the tolerance itself (at least 1e-8) for FP64, whose inner
  // solves aim at the outer tolerance.  A cheaper target favours the
  // shallow cycles, whose early iterations converge fastest (32^2 grid,
  // FP64 to 1e-10: aiming at 1e-3 picked depth 2, 104,138 RHS/s, over the
  // full depth, 175,864), and the FP64 target must not be 0: it would run
  // every candidate to rounding level.
  if (p0.precision == CFC_PREC_FP64) {
    p.tol = std::max(p0.tol, 1e-8);
  } else {
    p.inner_tol = 1e-4;
    p.tol = 1e-300;
  }
  Solver S(g, p);
  Workspace& w = *S.ws;
  int* ps = w.pairs.as<int>();
  std::vector<int> hp(2 * W);
  for (int j = 0; j < W; ++j) {
    int64_t s = (int64_t)((uint64_t(j) * 2654435761ull + 12345) % uint64_t(g.n));
    int64_t t = (int64_t)((uint64_t(j) * 40503ull + 17 + uint64_t(g.n) / 2) % uint64_t(g.n));
    if (s == t) t = (t + 1) % g.n;
    hp[j] = g.H.perm[s];
    hp[W + j] = g.H.perm[t];
  }
  CFC_HIP(hipMemcpyAsync(ps, hp.data(), 2 * W * sizeof(int), hipMemcpyHostToDevice, S.stream));
  RhsArgs r;
  r.kind = 1;
  r.ps = ps;
  r.pt = ps + W;
  std::vector<double> rel(W);
  // the first block allocates, captures the HIP graphs and learns when to
  // check convergence, as the first block of a real solve does; the second
  // is timed
  S.solve_block(r, W, p, nullptr, rel.data());
  hipEvent_t a = nullptr, b = nullptr;
  CFC_HIP(hipEventCreate(&a));
  CFC_HIP(hipEventCreate(&b));
  CFC_HIP(hipEventRecord(a, S.stream));
  S.solve_block(r, W, p, nullptr, rel.data());
  CFC_HIP(hipEventRecord(b, S.stream));
  CFC_HIP(hipEventSynchronize(b));
  float ms = 0;
  CFC_HIP(hipEventElapsedTime(&ms, a, b));
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  cfc_solve_stats st{};
  S.finish(&st);
  double worst = 0;
  for (double x : rel) worst = std::max(worst, std::isfinite(x) ? x : 1.0);
  const double relr = std::max(worst, 1e-12);
  const double digits = relr < 1 ? -std::log10(relr) : 1e-3;
  if (std::getenv("CFC_DEBUG"))
    std::fprintf(stderr, "[cfc] tune W %d depth %d: %.3f ms, %lld iterations (two blocks), rel %.3g\n", W,
                 depth, ms, (long long)st.inner_iters, worst);
  return ms / (W * digits);
}

// Refinement split: aim each FP32 inner solve at 1e-4 (two refinement steps
// to 1e-6), or straight at the target (one step, inner floor 1e-7, about
// FP32 rounding) when the FP32 iteration can get there without stalling.
// Both are timed on W sample pair right-hand sides to the requested
// tolerance; one step wins only if every column converges and it is faster.
constexpr double kTwoStep = 1e-4, kOneStep = 1e-7;

static int tune_split(Graph& g, const cfc_solve_params& p0, int W, int depth) {
  if (p0.precision == CFC_PREC_FP64) return 0;  // FP64 inner solves aim at the target anyway
  cfc_solve_params q = p0;
  q.block = W;
  q.levels = depth;
  std::vector<int64_t> s(W), t(W);
  for (int j = 0; j < W; ++j) {
    s[j] = (int64_t)((uint64_t(j) * 2654435761ull + 777) % uint64_t(g.n));
    t[j] = (int64_t)((uint64_t(j) * 40503ull + 91 + uint64_t(g.n) / 3) % uint64_t(g.n));
    if (s[j] == t[j]) t[j] = (t[j] + 1) % g.n;
  }
  std::vector<double> out(W);
  cfc_solve_stats two{}, one{};
  q.inner_tol = kTwoStep;
  for (int rep = 0; rep < 2; ++rep) {
    two = cfc_solve_stats{};
    pair_solves(g, W, s.data(), t.data(), out.data(), q, &two, nullptr);
  }
  if (two.converged < W) return 0;
  q.inner_tol = kOneStep;
  q.max_inner = (int)std::min<int64_t>(q.max_inner, std::max<int64_t>(10, 2 * two.inner_iters));
  pair_solves(g, W, s.data(), t.data(), out.data(), q, &one, nullptr);
  return (one.converged == W && one.solve_ms < 0.97 * two.solve_ms) ? 1 : 0;
}

static bool width_fits(const Graph& g, int W, int prec) {
  double n = 0;
  for (const auto& l : g.D->lv) n += (double)l.n;
  const double n0 = (double)g.D->lv[0].n;
  const double es = prec == CFC_PREC_FP64 ? 8 : 4;
  const double need = ((n0 * (6 * es + 16) + 2 * (n - n0) * es) * W + (double)heavy_partial_bytes(g, W)) * 1.1;
  const uint64_t budget = g.ctx->budget;
  if (budget && g.ctx->in_use + need > (double)budget) return false;
  size_t freeb = 0, totalb = 0;
  if (hipMemGetInfo(&freeb, &totalb) == hipSuccess && need > 0.7 * (double)freeb) return false;
  return true;
}

cfc_solve_params tune_params(Graph& g, const cfc_solve_params& p0, int64_t ncols) {
  cfc_solve_params p = p0;
  auto split = [&](int one_step) {
    if (p0.inner_tol == 0) p.inner_tol = one_step ? kOneStep : kTwoStep;
  };
  if (p.block && p.levels) {
    split(0);
    return p;
  }
  const int prec = p.precision;
  const int nlev = (int)g.D->lv.size();
  for (const auto& t : g.tuned)
    if (t[0] == prec && t[1] == p0.block) {
      if (!p.block) p.block = t[2];
      if (!p.levels) p.levels = t[3];
      split(t[4]);
      return p;
    }
  const char* cache = std::getenv("CFC_TUNE_CACHE");
  const std::string key = tune_key(g, prec) + " " + std::to_string(p0.block);
  if (cache) {
    std::ifstream f(cache);
    std::string line;
    while (std::getline(f, line)) {
      if (line.rfind(key + " ", 0) != 0) continue;
      std::istringstream is(line.substr(key.size() + 1));
      int W = 0, d = 0, one = 0;
      is >> W >> d >> one;
      if (kern_table(W, false) && d >= 1 && d <= nlev) {
        g.tuned.push_back({prec, p0.block, W, d, one ? 1 : 0});
        if (!p.block) p.block = W;
        if (!p.levels) p.levels = d;
        split(one);
        return p;
      }
    }
  }
  std::vector<int> widths = prec == CFC_PREC_FP64 ? std::vector<int>{64, 128, 256}
                                                   : std::vector<int>{64, 128, 256, 512};
  std::vector<int> ok;
  for (int W : widths) {
    if (ncols > 0 && W > 64 && W / 2 >= ncols) continue;  // would leave most columns idle
    if (width_fits(g, W, prec)) ok.push_back(W);
  }
  if (ok.empty()) ok.push_back(64);
  int W0 = p.block;
  if (!W0) {
    W0 = ok.front();
    for (int W : ok)
      if (W <= 256) W0 = W;
  }
  int best_d = p.levels;
  if (!best_d) {
    std::vector<int> depths = {1, 2, 3, nlev};
    std::sort(depths.begin(), depths.end());
    depths.erase(std::unique(depths.begin(), depths.end()), depths.end());
    double bs = 1e300;
    for (int d : depths) {
      if (d < 1 || d > nlev) continue;
      const double sc = tune_score(g, p, W0, d);
      if (std::getenv("CFC_DEBUG"))
        std::fprintf(stderr, "[cfc] tune W %d depth %d: %.4g ms per column and digit\n", W0, d, sc);
      if (sc < bs) { bs = sc; best_d = d; }
    }
  }
  int best_W = p.block;
  if (!best_W) {
    double bs = 1e300;
    for (int W : ok) {
      const double sc = tune_score(g, p, W, best_d);
      if (std::getenv("CFC_DEBUG"))
        std::fprintf(stderr, "[cfc] tune W %d depth %d: %.4g ms per column and digit\n", W, best_d, sc);
      if (sc < bs) { bs = sc; best_W = W; }
    }
  }
  // release workspaces of the losing widths
  g.ws.erase(std::remove_if(g.ws.begin(), g.ws.end(),
                            [&](const std::unique_ptr<Workspace>& w) { return w->W != best_W; }),
             g.ws.end());
  const int one = p0.inner_tol == 0 ? tune_split(g, p, best_W, best_d) : 0;
  if (!p0.levels) {
    g.tuned.push_back({prec, p0.block, best_W, best_d, one});
    if (cache) {
      std::ofstream f(cache, std::ios::app);
      f << key << ' ' << best_W << ' ' << best_d << ' ' << one << '\n';
    }
  }
  p.block = best_W;
  p.levels = best_d;
  split(one);
  return p;
}

// ---------------------------------------------------------------------------

void solve_dense(Graph& g, int64_t nrhs, const double* B, double* X, const cfc_solve_params& p0,
                 cfc_solve_stats* st, int32_t* col_status) {
  check_params(p0);
  if (nrhs < 0 || (nrhs > 0 && (!B || !X))) fail(CFC_E_INVALID, "bad B/X");
  const int64_t n = g.n;
  cfc_solve_params p = tune_params(g, p0, nrhs);
  Solver S(g, p);
  Workspace& w = *S.ws;
  const int W = w.W;
  if (!w.rhs.p) w.rhs.alloc(g.ctx, (size_t)n * W * sizeof(double));
  // Column blocks of B and X are contiguous (column-major), so a host buffer
  // moves as one copy per block through a device staging block; the
  // transposes, the checks and the centring run on the device.
  const bool bdev = is_device_ptr(B), xdev = is_device_ptr(X);
  DBuf stage, part, stat;
  if (!bdev || !xdev) stage.alloc(g.ctx, (size_t)n * W * sizeof(double));
  part.alloc(g.ctx, (size_t)kColStatGrid * 2 * W * sizeof(double));
  stat.alloc(g.ctx, 2 * (size_t)W * sizeof(double));
  std::vector<double> hs(2 * (size_t)W);
  const int* perm = g.D->perm.as<int>();
  double* rhs = w.rhs.as<double>();
  double* x64 = w.x64.as<double>();
  double* sd = stage.as<double>();
  for (int64_t c0 = 0; c0 < nrhs; c0 += W) {
    const int nc = (int)std::min<int64_t>(W, nrhs - c0);
    const double* Bc = B + c0 * n;
    if (!bdev) {
      CFC_HIP(hipMemcpyAsync(sd, Bc, (size_t)nc * n * sizeof(double), hipMemcpyHostToDevice, S.stream));
      Bc = sd;
    }
    block_in((int)n, W, nc, Bc, perm, rhs, S.stream);
    col_stats((int)n, W, rhs, part.as<double>(), stat.as<double>(), S.stream);
    CFC_HIP(hipMemcpyAsync(hs.data(), stat.p, hs.size() * sizeof(double), hipMemcpyDeviceToHost,
                           S.stream));
    CFC_HIP(hipStreamSynchronize(S.stream));
    for (int j = 0; j < nc; ++j) {
      const double s = hs[j], a = hs[W + j];
      if (!std::isfinite(a))
        fail(CFC_E_INVALID, "B column " + std::to_string(c0 + j) + " is not finite");
      if (std::fabs(s) > 1e-12 * a + 1e-300 && a > 0)
        fail(CFC_E_INVALID, "B column " + std::to_string(c0 + j) + " does not sum to zero");
    }
    RhsArgs r;
    r.kind = 0;
    r.dense = rhs;
    S.solve_block(r, nc, p, col_status ? col_status + c0 : nullptr, nullptr);
    // X = x - mean(x): the returned copy is exactly mean-zero up to rounding
    col_stats((int)n, W, x64, part.as<double>(), stat.as<double>(), S.stream);
    double* Xc = xdev ? X + c0 * n : sd;
    block_out((int)n, W, nc, x64, perm, stat.as<double>(), Xc, S.stream);
    if (!xdev)
      CFC_HIP(hipMemcpyAsync(X + c0 * n, sd, (size_t)nc * n * sizeof(double), hipMemcpyDeviceToHost,
                             S.stream));
    CFC_HIP(hipStreamSynchronize(S.stream));
  }
  S.finish(st);
  if (S.converged < S.columns) fail(CFC_E_NOT_CONVERGED, "some columns missed the tolerance");
}

void pair_solves(Graph& g, int64_t npairs, const int64_t* s, const int64_t* t, double* out,
                 const cfc_solve_params& p0, cfc_solve_stats* st, int32_t* col_status) {
  check_params(p0);
  for (int64_t j = 0; j < npairs; ++j)
    if (s[j] < 0 || s[j] >= g.n || t[j] < 0 || t[j] >= g.n) fail(CFC_E_INVALID, "node id out of range");
  cfc_solve_params p = tune_params(g, p0, npairs);
  Solver S(g, p);
  Workspace& w = *S.ws;
  const int W = w.W;
  int* ps = w.pairs.as<int>();
  int* pt = ps + W;
  double* dd = w.dvec.as<double>();
  std::vector<int> hp(2 * W);
  std::vector<double> res(W);
  std::vector<int32_t> stat(W);
  for (int64_t c0 = 0; c0 < npairs; c0 += W) {
    const int nc = (int)std::min<int64_t>(W, npairs - c0);
    for (int j = 0; j < W; ++j) {
      if (j < nc) {
        hp[j] = g.H.perm[s[c0 + j]];
        hp[W + j] = g.H.perm[t[c0 + j]];
        if (hp[j] == hp[W + j]) hp[j] = hp[W + j] = -1;  // e_v - e_v = 0
      } else {
        hp[j] = hp[W + j] = -1;
      }
    }
    CFC_HIP(hipMemcpyAsync(ps, hp.data(), 2 * W * sizeof(int), hipMemcpyHostToDevice, S.stream));
    RhsArgs r;
    r.kind = 1;
    r.ps = ps;
    r.pt = pt;
    S.pair_out = dd;
    S.solve_block(r, nc, p, stat.data(), nullptr);
    if (!S.pair_used) pair_diff(W, nc, w.x64.as<double>(), ps, pt, dd, S.stream);
    CFC_HIP(hipMemcpyAsync(res.data(), dd, nc * sizeof(double), hipMemcpyDeviceToHost, S.stream));
    CFC_HIP(hipStreamSynchronize(S.stream));
    for (int j = 0; j < nc; ++j) {
      out[c0 + j] = res[j];
      if (col_status) col_status[c0 + j] = stat[j];
    }
  }
  S.finish(st);
}

// ---------------------------------------------------------------------------
// projection estimator

void jl_sketch(Graph& g, int64_t k, uint64_t seed, const cfc_solve_params& p0, cfc_solve_stats* st) {
  check_params(p0);
  if (k < 1) fail(CFC_E_INVALID, "k must be >= 1");
  cfc_solve_params p = tune_params(g, p0, k);
  g.jl.valid = false;
  const int n0 = g.D->lv[0].n;
  Solver S(g, p);
  Workspace& w = *S.ws;
  const int W = w.W;
  if (!w.rhs.p) w.rhs.alloc(g.ctx, (size_t)n0 * W * sizeof(double));
  if (g.jl.N_dev.bytes != (size_t)n0 * 8) {
    g.jl.N_dev.alloc(g.ctx, (size_t)n0 * 8);
    g.jl.S2_dev.alloc(g.ctx, 1024 * 8 + 8);
  }
  w.kt->zero(g.jl.N_dev.p, g.jl.N_dev.bytes, S.stream);
  LevelArgs l64 = w.la64;
  std::vector<int32_t> stat(W);
  for (int64_t i0 = 0; i0 < k; i0 += W) {
    const int nc = (int)std::min<int64_t>(W, k - i0);
    // the right-hand sides, with the refinement's first residual (r = y in
    // the inner precision) and its norms formed in the same pass
    const int rows = w.kt->jl_rhs(l64, g.D->iperm.as<int>(), seed, i0, k, w.rhs.as<double>(), w.ra.p,
                                  w.part_ptr(P_PQ), S.stream);
    S.bytes += (double)n0 * W * (8 + w.kt->esize) + 4.0 * g.D->lv[0].nnz + 8.0 * n0;
    RhsArgs r;
    r.kind = 0;
    r.dense = w.rhs.as<double>();
    r.r0_rows = rows;
    S.solve_block(r, nc, p, stat.data(), nullptr);
    // per-node |Z_v|^2 (the solutions are mean-zero, so sum_w Z_w = 0)
    w.kt->jl_rownorm(n0, w.x64.as<double>(), nc, g.jl.N_dev.as<double>(), nullptr, S.stream);
    S.bytes += (double)n0 * W * 8 + 2.0 * n0 * 8;
  }
  double* part = g.jl.S2_dev.as<double>() + 1;
  reduce_sum(n0, g.jl.N_dev.as<double>(), part, g.jl.S2_dev.as<double>(), S.stream);
  double S2 = 0;
  CFC_HIP(hipMemcpyAsync(&S2, g.jl.S2_dev.p, 8, hipMemcpyDeviceToHost, S.stream));
  CFC_HIP(hipStreamSynchronize(S.stream));
  S.finish(st);
  g.jl.k = k;
  g.jl.seed = seed;
  g.jl.S2 = S2;
  g.jl.valid = S.converged == S.columns;
  if (!g.jl.valid) fail(CFC_E_NOT_CONVERGED, "projection solves missed the tolerance");
}

void jl_farness(Graph& g, int64_t q, const int64_t* nodes, double* far, double* clo, Ctx* mem,
                hipStream_t stream) {
  if (!g.jl.valid) fail(CFC_E_STATE, "no projection sketch (call cfc_jl_sketch)");
  if (q < 0 || (q > 0 && (!nodes || !far))) fail(CFC_E_INVALID, "bad arguments");
  std::vector<int> idx(q);
  for (int64_t i = 0; i < q; ++i) {
    if (nodes[i] < 0 || nodes[i] >= g.n) fail(CFC_E_INVALID, "node id out of range");
    idx[i] = g.H.perm[nodes[i]];
  }
  if (q == 0) return;
  Ctx* c = mem ? mem : g.ctx;
  DBuf di, dn;
  di.alloc(c, q * sizeof(int));
  dn.alloc(c, q * sizeof(double));
  hipStream_t s = stream ? stream : g.ctx->stream;
  CFC_HIP(hipMemcpyAsync(di.p, idx.data(), q * sizeof(int), hipMemcpyHostToDevice, s));
  gather((int)q, g.jl.N_dev.as<double>(), di.as<int>(), dn.as<double>(), s);
  std::vector<double> hn(q);
  CFC_HIP(hipMemcpyAsync(hn.data(), dn.p, q * sizeof(double), hipMemcpyDeviceToHost, s));
  CFC_HIP(hipStreamSynchronize(s));
  const double n = (double)g.n;
  for (int64_t i = 0; i < q; ++i) {
    // sum_w |Z_v - Z_w|^2 = n |Z_v|^2 - 2 Z_v . sum_w Z_w + |Z|_F^2, and
    // sum_w Z_w = 0 because every solve returns the mean-zero L^+ y_i
    const double f = n * hn[i] + g.jl.S2;
    far[i] = f;
    if (clo) clo[i] = f > 0 ? (n - 1) / f : INFINITY;
  }
}

}  // namespace cfc
