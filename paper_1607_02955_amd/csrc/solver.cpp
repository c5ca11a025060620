// Solve loop: device copy of the hierarchy, per-block workspaces, the
// preconditioned CG inner solver, FP64 iterative refinement, and the
// estimator reductions.
//
// One block of W right-hand sides is solved at a time (Eq. 1, L x = b):
//   outer (FP64):  r = b - L x, per-column ||r|| / ||b|| <= tol (Sec. 3.1),
//                  else solve L d ~= r and x += d - mean(d) (the
//                  mean-zero representative, Sec. 2: x is fixed only up to
//                  an additive constant);
//   inner (T = float in mixed mode, double in FP64 mode): CG preconditioned
//                  by one symmetric V-cycle of the aggregation hierarchy.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>

#include "kern.hpp"
#include "solver.hpp"

static_assert(cfc::kElimDeg == CFC_ELIM_MAX_DEGREE, "eliminated-row neighbour slots");

namespace cfc {

// ---------------------------------------------------------------------------
// device upload

namespace {
// Copies complete before returning, so the host vector may be a temporary.
template <class T>
void upload(Ctx* c, DBuf& d, const std::vector<T>& h, hipStream_t s) {
  d.alloc(c, h.size() * sizeof(T));
  if (h.empty()) return;
  CFC_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  CFC_HIP(hipStreamSynchronize(s));
}
}  // namespace

// Light CSR (rows of degree <= heavy_deg) plus heavy rows in their own CSR
// cut into segments of heavy_deg edges, FP32 and FP64 weights.
static void upload_csr(Ctx* c, DevLevel& d, int64_t n, const std::vector<int32_t>& rowptr,
                       const std::vector<int32_t>& col, const std::vector<double>& w, bool unit,
                       int heavy_deg, int seg_len, hipStream_t s) {
  std::vector<int32_t> lptr(n + 1, 0), lcol, hid(n, -1), hptr(1, 0), hcol, hseg(1, 0), seg_e(1, 0),
      seg_row;
  std::vector<double> lw, hw;
  lcol.reserve(col.size());
  lw.reserve(w.size());
  d.nheavy = 0;
  for (int64_t r = 0; r < n; ++r) {
    const int32_t e0 = rowptr[r], e1 = rowptr[r + 1];
    if (e1 - e0 > heavy_deg) {
      hid[r] = d.nheavy++;
      for (int32_t e = e0; e < e1; ++e) {
        hcol.push_back(col[e]);
        hw.push_back(w[e]);
        if ((int)(hcol.size() - hptr.back()) % seg_len == 0) seg_e.push_back((int32_t)hcol.size());
      }
      if (seg_e.back() != (int32_t)hcol.size()) seg_e.push_back((int32_t)hcol.size());
      hptr.push_back((int32_t)hcol.size());
      hseg.push_back((int32_t)seg_e.size() - 1);
      seg_row.resize(seg_e.size() - 1, (int32_t)r);
    } else {
      for (int32_t e = e0; e < e1; ++e) {
        lcol.push_back(col[e]);
        lw.push_back(w[e]);
      }
    }
    lptr[r + 1] = (int32_t)lcol.size();
  }
  d.light_nnz = (int)lcol.size();
  d.nseg = (int)seg_e.size() - 1;
  upload(c, d.rowptr, lptr, s);
  upload(c, d.col, lcol, s);
  if (!unit) {
    std::vector<float> w32(lw.size()), hw32(hw.size());
    for (size_t k = 0; k < lw.size(); ++k) w32[k] = (float)lw[k];
    for (size_t k = 0; k < hw.size(); ++k) hw32[k] = (float)hw[k];
    upload(c, d.w32, w32, s);
    upload(c, d.w64, lw, s);
    upload(c, d.hw32, hw32, s);
    upload(c, d.hw64, hw, s);
  }
  if (d.nheavy) {
    upload(c, d.heavy, hid, s);
    upload(c, d.hseg, hseg, s);
    upload(c, d.hptr, hptr, s);
    upload(c, d.hcol, hcol, s);
    upload(c, d.seg_e, seg_e, s);
    upload(c, d.seg_row, seg_row, s);
  }
}

template <class T>
static std::vector<float> to_f32(const std::vector<T>& v) {
  std::vector<float> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (float)v[i];
  return o;
}

static uint64_t level_bytes(const DevLevel& d) {
  uint64_t b = 0;
  for (const DBuf* x : {&d.rowptr, &d.col, &d.w32, &d.w64, &d.deg32, &d.deg64, &d.sdinv32, &d.sdinv64,
                        &d.agg, &d.aggptr, &d.heavy, &d.hseg, &d.hptr, &d.hcol, &d.hw32, &d.hw64,
                        &d.seg_e, &d.seg_row, &d.enb, &d.ew32, &d.ew64, &d.einv32, &d.einv64})
    b += x->bytes;
  return b;
}

void upload_hierarchy(Graph& g) {
  Ctx* c = g.ctx;
  if (c->host_only()) return;
  CFC_HIP(hipSetDevice(c->device));
  auto D = std::make_unique<DevHierarchy>();
  const Hierarchy& H = g.H;
  const int L = (int)H.lv.size();
  D->lv.resize(L);
  hipStream_t s = c->stream;
  // rows longer than 64 entries are summed by segments in the pre-pass: in
  // the row kernels a long row holds up its whole workgroup (W = 512, FP8
  // z: R-MAT-20 Sampling 8,972 / 9,414 / 9,434 RHS/s at thresholds 256 / 64
  // / 96, BA-100k projection 72,785 / 78,611 / 76,062, 48 and 32 no better;
  // earlier, at W = 256, 256 had beaten 512; CFC_HEAVY_DEG overrides)
  static const int heavy_deg = [] {
    const char* e = std::getenv("CFC_HEAVY_DEG");
    return e ? std::max(16, std::atoi(e)) : 64;
  }();
  // edges per heavy-row segment (one pre-pass workgroup per segment and
  // slice): 512 (R-MAT-20 Sampling at W = 512 with FP8 z: operator product
  // 3.67 ms against 3.76 at 256 and 3.74 at 1024; BA-100k unchanged)
  static const int seg_len = [] {
    const char* e = std::getenv("CFC_SEG_LEN");
    return e ? std::max(16, std::atoi(e)) : 512;
  }();
  for (int l = 0; l < L; ++l) {
    const HostLevel& h = H.lv[l];
    DevLevel& d = D->lv[l];
    d.n = (int)h.n;
    d.nnz = (int)h.nnz();
    d.nagg = h.aggptr.empty() ? 0 : (int)h.aggptr.size() - 1;
    d.unit = (l == 0) && g.unit;
    upload_csr(c, d, h.n, h.rowptr, h.col, h.w, d.unit, heavy_deg, seg_len, s);
    std::vector<float> deg32(h.n), sd32(h.n);
    std::vector<double> sd64(h.n);
    for (int64_t r = 0; r < h.n; ++r) {
      // FP32 diagonal = FP32 sum of the FP32 off-diagonals, so that the FP32
      // operator keeps its row sums (L 1 = 0) as closely as FP32 allows.
      float sacc = 0.f;
      for (int32_t e = h.rowptr[r]; e < h.rowptr[r + 1]; ++e) sacc += (float)h.w[e];
      deg32[r] = sacc;
      sd32[r] = sacc > 0 ? (float)(H.omega / (double)sacc) : 0.f;
      sd64[r] = h.deg[r] > 0 ? H.omega / h.deg[r] : 0.0;
    }
    upload(c, d.deg32, deg32, s);
    upload(c, d.deg64, h.deg, s);
    upload(c, d.sdinv32, sd32, s);
    upload(c, d.sdinv64, sd64, s);
    if (!h.agg.empty()) {
      upload(c, d.agg, h.agg, s);
      upload(c, d.aggptr, h.aggptr, s);
    }
    if (h.nC > 0) {
      // elimination level: forward operator (kept rows x eliminated rows;
      // hubs with many eliminated neighbours go to short heavy segments)
      d.nC = (int)h.nC;
      upload_csr(c, D->fwd, h.nC, h.fptr, h.fcol, h.fcoef, false, 64, 64, s);
      D->fwd.n = (int)h.nC;
      D->fwd.nnz = (int)h.fcol.size();
      upload(c, d.enb, h.enb, s);
      upload(c, d.ew64, h.ew, s);
      upload(c, d.ew32, to_f32(h.ew), s);
      upload(c, d.einv64, h.einv, s);
      upload(c, d.einv32, to_f32(h.einv), s);
      D->bytes += level_bytes(D->fwd);
    }
    d.omega64 = H.omega;
    D->bytes += level_bytes(d);
  }
  // coarsest pseudoinverse, zero-padded to a multiple of 16 (none when the
  // complexity budget stopped coarsening on a large level)
  const int nc = H.cpinv.empty() ? 0 : (int)H.lv[L - 1].n;
  const int ncp = (nc + 15) / 16 * 16;
  std::vector<double> P((size_t)ncp * ncp, 0.0);
  for (int i = 0; i < nc; ++i)
    for (int j = 0; j < nc; ++j) P[(size_t)i * ncp + j] = H.cpinv[(size_t)i * nc + j];
  upload(c, D->cpinv, P, s);
  D->nc = nc;
  upload(c, D->iperm, H.iperm, s);
  upload(c, D->perm, H.perm, s);
  D->bytes += D->cpinv.bytes + D->iperm.bytes + D->perm.bytes;
  CFC_HIP(hipStreamSynchronize(s));
  g.ws.clear();
  g.D = std::move(D);
  g.jl = JLSketch();
}

// ---------------------------------------------------------------------------
// workspace

static LevelArgs level_args(const Graph& g, int l, bool fp64) {
  const DevLevel& d = g.D->lv[l];
  LevelArgs a;
  a.n = d.n;
  a.nagg = d.nagg;
  a.rowptr = d.rowptr.as<int>();
  a.col = d.col.as<int>();
  a.w = fp64 ? (const void*)d.w64.p : (const void*)d.w32.p;
  if (d.unit) a.w = nullptr;
  a.deg = fp64 ? d.deg64.p : d.deg32.p;
  a.sd = fp64 ? d.sdinv64.p : d.sdinv32.p;
  a.agg = d.agg.as<int>();
  a.aggptr = d.aggptr.as<int>();
  a.omega = g.H.omega;
  a.mu = g.H.mu;
  // long rows (dense coarse levels, heavy-tailed graphs): several row groups
  // share a row; about 8 edges per row group
  static const double per_group = [] {
    const char* e = std::getenv("CFC_SPLIT_EDGES");
    return e ? std::atof(e) : 8.0;
  }();
  const double avg = d.n > 0 ? (double)d.light_nnz / d.n : 0.0;
  a.split = avg >= 16 * per_group ? 16 : (avg >= 4 * per_group ? 4 : 1);
  a.nheavy = d.nheavy;
  a.nseg = d.nseg;
  if (d.nheavy) {
    a.heavy = d.heavy.as<int>();
    a.hseg = d.hseg.as<int>();
    a.hptr = d.hptr.as<int>();
    a.hcol = d.hcol.as<int>();
    a.hw = d.unit ? nullptr : (fp64 ? (const void*)d.hw64.p : (const void*)d.hw32.p);
    a.seg_e = d.seg_e.as<int>();
    a.seg_row = d.seg_row.as<int>();
  }
  if (d.nC > 0) {
    a.nC = d.nC;
    a.enb = d.enb.as<int>();
    a.ew = fp64 ? d.ew64.p : d.ew32.p;
    a.einv = fp64 ? d.einv64.p : d.einv32.p;
  }
  return a;
}

// The forward operator of an elimination level 0 (kept rows x all rows).
static LevelArgs fwd_args(const Graph& g, bool fp64) {
  const DevLevel& d = g.D->fwd;
  LevelArgs a;
  a.n = d.n;
  a.rowptr = d.rowptr.as<int>();
  a.col = d.col.as<int>();
  a.w = fp64 ? (const void*)d.w64.p : (const void*)d.w32.p;
  a.split = 1;
  a.nheavy = d.nheavy;
  a.nseg = d.nseg;
  if (d.nheavy) {
    a.heavy = d.heavy.as<int>();
    a.hseg = d.hseg.as<int>();
    a.hptr = d.hptr.as<int>();
    a.hcol = d.hcol.as<int>();
    a.hw = fp64 ? (const void*)d.hw64.p : (const void*)d.hw32.p;
    a.seg_e = d.seg_e.as<int>();
    a.seg_row = d.seg_row.as<int>();
  }
  return a;
}

Workspace::~Workspace() {
  if (pinned) (void)hipHostFree(pinned);
  if (mirror) (void)hipHostFree(mirror);
}

Workspace& get_workspace(Graph& g, int W, bool fp64, hipStream_t s, Ctx* mem) {
  for (auto& w : g.ws)
    if (w->W == W && w->fp64 == fp64) return *w;
  Ctx* c = mem ? mem : g.ctx;
  auto ws = std::make_unique<Workspace>();
  Workspace& w = *ws;
  w.W = W;
  w.fp64 = fp64;
  w.kt = kern_table(W, fp64);
  if (!w.kt) fail(CFC_E_INVALID, "unsupported block width " + std::to_string(W));
  const int L = (int)g.D->lv.size();
  w.nlev = L;
  w.la.resize(L);
  for (int l = 0; l < L; ++l) w.la[l] = level_args(g, l, fp64);
  w.la64 = level_args(g, 0, true);
  // segment partials of heavy rows, one region per level (FP64-sized so the
  // FP64 residual can share level 0's region)
  w.hpart.resize(L);
  w.hsum.resize(L);
  for (int l = 0; l < L; ++l)
    if (g.D->lv[l].nseg) {
      w.hpart[l].alloc(c, (size_t)g.D->lv[l].nseg * W * 8);
      w.hsum[l].alloc(c, (size_t)g.D->lv[l].nheavy * W * 8);
      w.la[l].hpart = w.hpart[l].p;
      w.la[l].hsum = w.hsum[l].p;
      if (l == 0) {
        w.la64.hpart = w.hpart[0].p;
        w.la64.hsum = w.hsum[0].p;
      }
    }
  if (g.D->lv[0].nC > 0) {
    w.lf = fwd_args(g, fp64);
    if (g.D->fwd.nseg) {
      w.fpart.alloc(c, (size_t)g.D->fwd.nseg * W * 8);
      w.fsum.alloc(c, (size_t)g.D->fwd.nheavy * W * 8);
      w.lf.hpart = w.fpart.p;
      w.lf.hsum = w.fsum.p;
    }
  }
  const size_t es = fp64 ? 8 : 4;
  const size_t n0 = (size_t)g.D->lv[0].n;
  const size_t blk = n0 * W * es;
  for (DBuf* b : {&w.x, &w.ra, &w.rb, &w.p, &w.q, &w.z}) b->alloc(c, blk);
  w.b.resize(L);
  w.xl.resize(L);
  for (int l = 1; l < L; ++l) {
    w.b[l].alloc(c, (size_t)g.D->lv[l].n * W * es);
    // below an elimination level the kept rows of z hold level 1's iterate
    if (l > 1 || g.D->lv[0].nC == 0) w.xl[l].alloc(c, (size_t)g.D->lv[l].n * W * es);
  }
  w.x64.alloc(c, n0 * W * 8);
  w.pairs.alloc(c, 2 * W * sizeof(int) + 2 * (W + 1) * sizeof(int));
  w.part.alloc(c, (size_t)P_COUNT * kMaxGrid * W * sizeof(double));
  w.scal.alloc(c, (size_t)S_N * W * sizeof(double));
  w.dvec.alloc(c, (size_t)(W + 1024) * sizeof(double));
  CFC_HIP(hipHostMalloc(&w.pinned, (size_t)(4 * W + 64) * sizeof(double), hipHostMallocDefault));
  CFC_HIP(hipHostMalloc(&w.mirror, (size_t)S_N * W * sizeof(double),
                        hipHostMallocMapped | hipHostMallocCoherent));
  CFC_HIP(hipHostGetDevicePointer((void**)&w.mirror_dev, w.mirror, 0));
  w.kt->zero(w.scal.p, w.scal.bytes, s);
  w.kt->zero(w.part.p, w.part.bytes, s);
  g.ws.push_back(std::move(ws));
  return *g.ws.back();
}

double* Workspace::part_ptr(int which) const {
  return part.as<double>() + (size_t)which * kMaxGrid * W;
}

// ---------------------------------------------------------------------------
// model of algorithmic bytes (compulsory traffic per launch; gathered rows
// counted once) used by the roofline report

static double mat_bytes(const DevLevel& d, bool weighted, size_t es) {
  return 4.0 * (d.n + 1) + 4.0 * d.nnz + (weighted ? es * (double)d.nnz : 0.0) + 2.0 * es * d.n;
}

// ---------------------------------------------------------------------------
// one V-cycle (and, when update is set, the PCG update of level 0 fused into
// its first kernel): z = V(r)

void Solver::vcycle(bool update, bool first_x, const void* r_in, void* r_out) {
  Workspace& w = *ws;
  const KernTable& k = *w.kt;
  hipStream_t s = stream;
  const int L = nuse;                 // levels this cycle visits
  const bool exact = nuse == w.nlev && g->D->nc > 0;  // deepest visited level is the true coarsest
  const size_t es = w.fp64 ? 8 : 4;
  const double nw = (double)w.W * es;
  const int b0 = base;  // the level the CG runs on
  const DevLevel& d0 = g->D->lv[b0];
  const void* rsrc = update ? r_out : r_in;
  if (jac_top) {
    // depth one: Jacobi-preconditioned CG on the base level, z = S r
    const DevLevel& db = g->D->lv[base];
    const LevelArgs& lb = w.la[base];
    if (update) {
      prof_begin(K_RESTRICT0);
      k.update_jacobi(lb, r_in, w.q.p, w.p.p, w.x.p, r_out, bfz ? w.z.p : nullptr,
                      w.scal.as<double>(), first_x, w.part_ptr(P_RR), w.part_ptr(P_CS),
                      w.part_ptr(P_RZ), zfmt(), xfu ? 1 : 0, s);
      const double ub = db.n * nw * upd_blocks(first_x) + 2.0 * es * db.n + (bfz ? zbytes() * db.n * w.W : 0.0);
      prof_end(K_RESTRICT0, ub);
      bytes += ub;
      g_rr = zf8 ? grid_for(db.n, k.rg8, slices_of(w.W) / k.ns8) : grid_for(db.n, k.rg);
      g_cs = xfu ? 0 : g_rr;  // with xfu the sums of x come with the last update
    } else {
      // r . S r (and the bfloat16 copy of z = S r when the product gathers it)
      k.jacobi(lb, r_in, bfz ? w.z.p : nullptr, w.part_ptr(P_RZ), zfmt(), s);
      bytes += db.n * nw + es * db.n + (bfz ? zbytes() * db.n * w.W : 0.0);
    }
    g_rz = zf8 ? grid_for(db.n, k.rg8, slices_of(w.W) / k.ns8) : grid_for(db.n, k.rg);
    return;
  }
  if (!schur && d0.nC > 0 && L >= 2) {
    vcycle_elim(update, first_x, r_in, r_out);
    return;
  }
  if (L - b0 == 1) {  // the base level is the coarsest: the preconditioner is its L^+
    if (update) {
      LevelArgs a = w.la[b0];
      a.nagg = 0;
      k.update_restrict(a, r_in, w.q.p, w.p.p, w.x.p, r_out, nullptr, w.scal.as<double>(), first_x,
                        1, w.part_ptr(P_RR), w.part_ptr(P_CS), xfu ? 1 : 0, s);
      g_rr = k.rows_grid(a, d0.n);
      g_cs = xfu ? 0 : g_rr;
      bytes += d0.n * nw * upd_blocks(first_x);
    }
    k.coarse(g->D->nc, (g->D->nc + 15) / 16 * 16, g->D->cpinv.as<double>(), rsrc, w.z.p, s);
    k.dot(d0.n, rsrc, w.z.p, w.part_ptr(P_RZ), s);
    g_rz = grid_for(d0.n, k.rg);
    bytes += d0.n * nw * 3 + 8.0 * d0.n * d0.n;
    return;
  }
  if (update) prof_begin(K_RESTRICT0);
  k.update_restrict(w.la[b0], r_in, w.q.p, w.p.p, w.x.p, r_out, w.b[b0 + 1].p, w.scal.as<double>(),
                    first_x, update ? 1 : 0, w.part_ptr(P_RR), w.part_ptr(P_CS), xfu ? 1 : 0, s);
  const double rb = d0.n * nw * (update ? upd_blocks(first_x) : 1) + d0.nagg * nw +
                    mat_bytes(d0, !d0.unit, es) + 4.0 * (d0.nagg + 1);
  if (update) {
    prof_end(K_RESTRICT0, rb);
    g_rr = k.rows_grid(w.la[b0], d0.nagg);
    g_cs = xfu ? 0 : g_rr;
  }
  bytes += rb;
  for (int l = b0 + 1; l + 1 < L; ++l) {
    const DevLevel& d = g->D->lv[l];
    k.restrict_(w.la[l], w.b[l].p, w.b[l + 1].p, s);
    bytes += d.n * nw + d.nagg * nw + mat_bytes(d, true, es) + 4.0 * (d.nagg + 1);
  }
  if (exact) {
    const int nc = g->D->nc;
    k.coarse(nc, (nc + 15) / 16 * 16, g->D->cpinv.as<double>(), w.b[L - 1].p, w.xl[L - 1].p, s);
    bytes += 2.0 * nc * nw + 8.0 * nc * nc;
  } else {
    const DevLevel& d = g->D->lv[L - 1];
    k.jacobi(w.la[L - 1], w.b[L - 1].p, w.xl[L - 1].p, nullptr, 0, s);
    bytes += 2.0 * d.n * nw + es * d.n;
  }
  for (int l = L - 2; l >= b0 + 1; --l) {
    const DevLevel& d = g->D->lv[l];
    k.prolong_smooth(w.la[l], w.b[l].p, w.xl[l + 1].p, w.xl[l].p, nullptr, s);
    bytes += 2.0 * d.n * nw + d.nagg * nw + mat_bytes(d, true, es) + 4.0 * d.n;
  }
  prof_begin(K_PROLONG0);
  k.prolong_smooth(w.la[b0], rsrc, w.xl[b0 + 1].p, w.z.p, w.part_ptr(P_RZ), s);
  const double pb = 2.0 * d0.n * nw + d0.nagg * nw + mat_bytes(d0, !d0.unit, es) + 4.0 * d0.n;
  prof_end(K_PROLONG0, pb);
  g_rz = k.rows_grid(w.la[b0], d0.n);
  bytes += pb;
}

// V-cycle whose level 0 is an elimination level: the CG update on all rows,
// the forward step onto the kept rows (level 1's rows), the cycle from level
// 1 with its iterate in the kept rows of z, and the back substitution.
void Solver::vcycle_elim(bool update, bool first_x, const void* r_in, void* r_out) {
  Workspace& w = *ws;
  const KernTable& k = *w.kt;
  hipStream_t s = stream;
  const int L = nuse;
  const bool exact = nuse == w.nlev && g->D->nc > 0;
  const size_t es = w.fp64 ? 8 : 4;
  const double nw = (double)w.W * es;
  const DevLevel& d0 = g->D->lv[0];
  const DevLevel& fw = g->D->fwd;
  const int n = d0.n, nc = d0.nC;
  const void* rsrc = update ? r_out : r_in;
  if (update) {
    prof_begin(K_RESTRICT0);
    LevelArgs a = w.la[0];
    a.nagg = 0;
    k.update_restrict(a, r_in, w.q.p, w.p.p, w.x.p, r_out, nullptr, w.scal.as<double>(), first_x, 1,
                      w.part_ptr(P_RR), w.part_ptr(P_CS), xfu ? 1 : 0, s);
    const double ub = n * nw * upd_blocks(first_x);
    prof_end(K_RESTRICT0, ub);
    bytes += ub;
    g_rr = k.rows_grid(a, n);
    g_cs = xfu ? 0 : g_rr;
  }
  const double fb = 2.0 * nc * nw + (double)(n - nc) * nw + 8.0 * fw.nnz + 4.0 * nc;
  const double bb = (double)(n - nc) * nw * 2 + 2.0 * (n - nc) * nw + 16.0 * (n - nc);
  if (L == 2 && !exact) {
    // Schur complement smoothed once: z_C = S t_C, fused into the forward
    // step (z in bfloat16 when the product gathers it so)
    k.elim_fwd(w.lf, rsrc, w.z.p, w.la[1].sd, w.part_ptr(P_RZ), bfz ? 2 : 1, s);
    const int g1 = k.elim_grid(nc);
    k.elim_back(w.la[0], rsrc, w.z.p, w.part_ptr(P_RZ) + (size_t)g1 * w.W, 0, bfz ? 1 : 0, s);
    g_rz = g1 + k.elim_grid(n - nc);
    // a bfloat16 z moves 2 bytes per value instead of es
    const double zs = bfz ? (es - 2.0) * w.W : 0.0;
    bytes += fb + bb - zs * (nc + 3.0 * (n - nc));
    return;
  }
  k.elim_fwd(w.lf, rsrc, w.b[1].p, nullptr, nullptr, 0, s);
  bytes += fb;
  auto xl = [&](int l) { return l == 1 ? w.z.p : w.xl[l].p; };
  for (int l = 1; l + 1 < L; ++l) {
    const DevLevel& d = g->D->lv[l];
    k.restrict_(w.la[l], w.b[l].p, w.b[l + 1].p, s);
    bytes += d.n * nw + d.nagg * nw + mat_bytes(d, true, es) + 4.0 * (d.nagg + 1);
  }
  if (exact) {
    const int ncs = g->D->nc;
    k.coarse(ncs, (ncs + 15) / 16 * 16, g->D->cpinv.as<double>(), w.b[L - 1].p, xl(L - 1), s);
    bytes += 2.0 * ncs * nw + 8.0 * ncs * ncs;
  } else {
    const DevLevel& d = g->D->lv[L - 1];
    k.jacobi(w.la[L - 1], w.b[L - 1].p, xl(L - 1), nullptr, 0, s);
    bytes += 2.0 * d.n * nw + es * d.n;
  }
  for (int l = L - 2; l >= 1; --l) {
    const DevLevel& d = g->D->lv[l];
    k.prolong_smooth(w.la[l], w.b[l].p, xl(l + 1), xl(l), nullptr, s);
    bytes += 2.0 * d.n * nw + d.nagg * nw + mat_bytes(d, true, es) + 4.0 * d.n;
  }
  k.elim_back(w.la[0], rsrc, w.z.p, w.part_ptr(P_RZ), 1, 0, s);
  g_rz = k.elim_grid(n);
  bytes += bb + 2.0 * nc * nw;
}

void Solver::prof_begin(int which) {
  if (!profile) return;
  ProfEv e{which, 0.0, nullptr, nullptr};
  CFC_HIP(hipEventCreate(&e.a));
  CFC_HIP(hipEventRecord(e.a, stream));
  prof_ev.push_back(e);
}
void Solver::prof_end(int which, double b) {
  if (!profile || prof_ev.empty() || prof_ev.back().kind != which || prof_ev.back().b) return;
  ProfEv& e = prof_ev.back();
  CFC_HIP(hipEventCreate(&e.b));
  CFC_HIP(hipEventRecord(e.b, stream));
  e.bytes = b;
}
void Solver::prof_collect() {
  for (auto& e : prof_ev) {
    if (e.b) {
      float ms = 0;
      CFC_HIP(hipEventSynchronize(e.b));
      CFC_HIP(hipEventElapsedTime(&ms, e.a, e.b));
      prof_ms[e.kind] += ms;
      prof_bytes[e.kind] += e.bytes;
      prof_launches[e.kind]++;
      (void)hipEventDestroy(e.b);
    }
    (void)hipEventDestroy(e.a);
  }
  prof_ev.clear();
}

// Read the per-column squared residuals S_RR to the host (synchronises).
void Solver::read_scal(int which, double* out) {
  Workspace& w = *ws;
  if (which == S_RR || which == S_R64) {
    // written to host-mapped memory by the finalize step
    CFC_HIP(hipStreamSynchronize(stream));
    std::memcpy(out, w.mirror + (size_t)which * w.W, w.W * sizeof(double));
    return;
  }
  CFC_HIP(hipMemcpyAsync(w.pinned, w.scal.as<double>() + (size_t)which * w.W, w.W * sizeof(double),
                         hipMemcpyDeviceToHost, stream));
  CFC_HIP(hipStreamSynchronize(stream));
  std::memcpy(out, w.pinned, w.W * sizeof(double));
}

// One PCG iteration on level 0 (operator product, step length, update fused
// into the first V-cycle kernel, V-cycle, direction scalars).
void Solver::iteration(bool first, void* r_in, void* r_out) {
  Workspace& w = *ws;
  const KernTable& k = *w.kt;
  const DevLevel& d0 = g->D->lv[base];
  const size_t es = w.fp64 ? 8 : 4;
  const double nw = (double)w.W * es;
  const int W = w.W;
  prof_begin(K_SPMM);
  // depth one: z = S r_in is formed inside the product kernel
  // (or gathered from its bfloat16 copy in ws.z)
  // one Jacobi step as the whole preconditioner (no exact solve on level 0)
  const bool jac = jac_top;
  k.spmm_pq(w.la[base], jac && !bfz ? r_in : w.z.p, w.p.p, w.q.p, xfu ? w.x.p : nullptr,
            w.scal.as<double>(), first, w.part_ptr(P_PQ), bfz ? (zf8 ? 3 : 2) : (jac ? 1 : 0), stream);
  const double sb = (bfz ? d0.n * (double)W * (zbytes() + es * (first ? 2 : 4)) + mat_bytes(d0, !d0.unit, es)
                         : d0.n * nw * (first ? 3 : 5) + mat_bytes(d0, !d0.unit, es) +
                               (jac ? es * d0.n : 0.0)) +
                    (xfu && !first ? 2.0 * d0.n * nw : 0.0);
  prof_end(K_SPMM, sb);
  bytes += sb;
  finalize(W, F_ALPHA, zf8 ? k.rows_grid8(w.la[base], d0.n) : k.rows_grid(w.la[base], d0.n),
           w.part_ptr(P_PQ), 0, nullptr, 0, nullptr, w.scal.as<double>(), stream);
  vcycle(true, first, r_in, r_out);
  finalize(W, F_BETA, g_rz, w.part_ptr(P_RZ), g_rr, w.part_ptr(P_RR), g_cs, w.part_ptr(P_CS),
           w.scal.as<double>(), stream, w.mirror_dev);
}

void Solver::capture_iterations() {
  Workspace& w = *ws;
  const double b0 = bytes;
  const bool prof = profile;
  profile = false;  // no event records inside the captured graphs
  for (int k = 0; k < 2; ++k) {
    CFC_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    if (k == 0)
      iteration(false, w.rb.p, r_alt());
    else
      iteration(false, r_alt(), w.rb.p);
    CFC_HIP(hipStreamEndCapture(stream, &graph[k]));
    CFC_HIP(hipGraphInstantiate(&gexec[k], graph[k], nullptr, nullptr, 0));
  }
  profile = prof;
  iter_bytes = (bytes - b0) / 2;
  bytes = b0;
}

// Preconditioned CG on L d = r0 (r0 in ws.ra); result d in ws.x.  Returns
// the iteration count.  After the first iteration the residual alternates
// between ws.rb and ws.ra; with use_graph the later iterations replay a
// captured pair of iterations.
int Solver::pcg(const std::vector<double>& rr0, const std::vector<double>& itol, int max_inner,
                int check_every) {
  Workspace& w = *ws;
  const KernTable& k = *w.kt;
  const double es = w.fp64 ? 8 : 4;
  if (!schur) {
    r0 = w.ra.p;
    const int it = pcg_iterations(rr0, itol, max_inner, check_every);
    if (xfu) {
      // the product kernels applied every x update but the last one
      const DevLevel& d0 = g->D->lv[0];
      const int gcs = grid_for(d0.n, k.rg);
      k.xfinal(d0.n, w.x.p, w.p.p, w.scal.as<double>(), w.part_ptr(P_CS), stream);
      finalize(w.W, F_CS, gcs, w.part_ptr(P_CS), 0, nullptr, 0, nullptr, w.scal.as<double>(), stream);
      bytes += 3.0 * d0.n * w.W * es;
    }
    return it;
  }
  // Schur mode.  With the kept rows C first and the eliminated rows F an
  // independent set, L d = r is L_CC d_C + L_CF d_F = r_C, L_FC d_C + D_F d_F
  // = r_F, so d_C solves S d_C = t_C with t_C = r_C - L_CF D_F^-1 r_F
  // (t_c = r_c + sum_f w_cf / d_f r_f) and d_F = D_F^-1 (r_F - L_FC d_C).
  const DevLevel& d0 = g->D->lv[0];
  const DevLevel& fw = g->D->fwd;
  const int n = d0.n, nc = d0.nC;
  if (!w.rt.p) w.rt.alloc(g->ctx, (size_t)nc * w.W * (size_t)es);
  // the inner tolerance is relative to the folded residual, whose squared
  // norms the fold kernel sums as it writes it
  k.elim_fwd(w.lf, w.ra.p, w.rt.p, nullptr, w.part_ptr(P_RR), 0, stream);
  bytes += 2.0 * nc * w.W * es + (double)(n - nc) * w.W * es + 8.0 * fw.nnz + 4.0 * nc;
  finalize(w.W, F_R64, k.elim_grid(nc), w.part_ptr(P_RR), 0, nullptr, 0, nullptr, w.scal.as<double>(),
           stream, w.mirror_dev);
  std::vector<double> rrt(w.W);
  read_scal(S_R64, rrt.data());
  for (int j = 0; j < w.W; ++j)
    if (!(rr0[j] > 0)) rrt[j] = 0;  // columns the caller left out stay out
  r0 = w.rt.p;
  const int it = pcg_iterations(rrt, itol, max_inner, check_every);
  if (xfu) {
    k.xfinal(nc, w.x.p, w.p.p, w.scal.as<double>(), w.part_ptr(P_CS), stream);
    bytes += 3.0 * nc * w.W * es;
  }
  // d_F from d_C (ws.x's first nc rows) and r_F (rows nc.. of ws.ra, which
  // the level-1 iterations never touch), then the column sums of d over all
  // rows for the mean projection
  k.elim_back(w.la[0], w.ra.p, w.x.p, w.part_ptr(P_RZ), 0, 0, stream);
  bytes += (n - nc) * (double)w.W * es * 2 + 2.0 * (n - nc) * w.W * es + 16.0 * (n - nc);
  if (!pairs_now) {  // pair differences need no mean
    k.dot(n, w.x.p, nullptr, w.part_ptr(P_CS), stream);
    finalize(w.W, F_CS, grid_for(n, k.rg), w.part_ptr(P_CS), 0, nullptr, 0, nullptr,
             w.scal.as<double>(), stream);
    bytes += n * (double)w.W * es;
  }
  return it;
}

int Solver::pcg_iterations(const std::vector<double>& rr0, const std::vector<double>& itol, int max_inner,
                           int check_every) {
  Workspace& w = *ws;
  const int W = w.W;
  vcycle(false, false, r0, nullptr);
  finalize(W, F_RZINIT, g_rz, w.part_ptr(P_RZ), 0, nullptr, 0, nullptr, w.scal.as<double>(), stream);
  std::vector<double> rr(W), tol2(W);
  double tight = 1;  // the strictest target of a tested column
  for (int j = 0; j < W; ++j) {
    tol2[j] = itol[j] * itol[j];
    if (rr0[j] > 0) tight = std::min(tight, itol[j]);
  }
  // no convergence test (and so no host synchronisation) before the fewest
  // iterations an earlier block needed at this refinement step, less one
  const std::array<int, 3> key{nuse, cur_step, (int)std::lround(4.0 * std::log10(std::max(tight, 1e-300)))};
  const auto hit = cur_step >= 0 ? w.min_its.find(key) : w.min_its.end();
  const int first_check = hit != w.min_its.end() ? std::max(1, hit->second - 1) : 1;
  auto record = [&](int n_it) {
    if (cur_step < 0 || n_it >= max_inner) return n_it;  // capped runs teach nothing
    auto ins = w.min_its.emplace(key, n_it);
    if (!ins.second) ins.first->second = std::min(ins.first->second, n_it);
    return n_it;
  };
  auto converged = [&]() {
    read_scal(S_RR, rr.data());
    for (int j = 0; j < W; ++j) {
      if (!(rr0[j] > 0)) continue;
      if (!std::isfinite(rr[j])) continue;  // reported by the outer residual
      if (rr[j] > tol2[j] * rr0[j]) return false;
    }
    return true;
  };
  int it = 1;
  iteration(true, r0, w.rb.p);
  if (max_inner == 1 || (first_check <= 1 && 1 % check_every == 0 && converged())) return record(it);
  if (params.use_graph) {
    // the residual is in r_b after odd iterations, in r_alt() after even ones
    if (!gexec[0]) capture_iterations();
    while (it < max_inner) {
      CFC_HIP(hipGraphLaunch(gexec[it % 2 == 1 ? 0 : 1], stream));
      ++it;
      bytes += iter_bytes;
      graph_replays++;
      if (it >= first_check && (it % check_every == 0 || it == max_inner) && converged()) break;
    }
    return record(it);
  }
  void* ra = w.rb.p;  // current residual
  void* rb = r_alt();
  while (it < max_inner) {
    ++it;
    iteration(false, ra, rb);
    std::swap(ra, rb);
    if (it >= first_check && (it % check_every == 0 || it == max_inner) && converged()) break;
  }
  return record(it);
}

// Solve one block.  rhs describes b (pairs or dense FP64 in ws.rhs, internal
// numbering); ncols columns are live.  On return ws.x64 holds x (mean-zero).
void Solver::solve_block(const RhsArgs& rhs, int ncols, const cfc_solve_params& p, int32_t* status,
                         double* final_rel) {
  Workspace& w = *ws;
  const KernTable& k = *w.kt;
  hipStream_t s = stream;
  const int W = w.W;
  const DevLevel& d0 = g->D->lv[0];
  const size_t es = w.fp64 ? 8 : 4;
  std::vector<double> r64(W), b2(W), rel(W, 0.0), itol(W);
  bool have_x = false;
  const int gres = k.rows_grid(w.la64, d0.n);
  double cur_max = 1.0;
  int step = 0;
  // FP32 inner solves aimed straight at tol (or FP64 ones) are expected to
  // finish in one refinement step unless an earlier block of this solve
  // needed more; otherwise the FP64 residual is kept for the next step
  const bool direct = p.precision == CFC_PREC_FP64 || p.inner_tol < 1e-6;
  bool r64_valid = false;  // ws.r64 = b - L x64 in FP64
  // In Schur mode the inner solve leaves ws.ra (the FP32 residual it was
  // given) untouched, so the next step reads r_prev from there in FP32.
  // Rounding r_prev to FP32 moves the computed residual by at most
  // 2^-24 |r_prev| per entry; those bounds are added up per column (ebound)
  // and counted against the tolerance, so the FP64 test still certifies it.
  const bool r32 = schur && !w.fp64;
  std::vector<double> ebound(W, 0.0);
  // Pair right-hand sides whose caller only wants x[s_j] - x[t_j]: in FP32
  // Schur mode no residual reads x64 (they gather the FP32 corrections), so
  // each step's correction d adds d[s_j] - d[t_j] to pair_out[j] (the mean
  // projection cancels in the difference) and x64 is not formed.
  pairs_now = pair_out && r32 && rhs.kind == 1;
  pair_used = pairs_now;
  for (;; ++step) {
    // x64 = x64_prev + d - mean(d) with d the FP32 inner solution still in
    // ws.x, and L 1 = 0, so b - L x64 = r_prev - L d up to FP64 rounding,
    // where r_prev is b after the first step and the kept FP64 residual
    // after later ones.  That residual gathers the FP32 d (half the bytes of
    // x64) and computes in FP64; without a kept residual (a step that was
    // expected to be the last) it gathers x64.
    const bool x32 = have_x && !w.fp64 && (step == 1 || r64_valid || r32);
    RhsArgs rr = rhs;
    if (x32 && step >= 2) {
      if (r32) {
        rr.kind = 2;
        rr.dense32 = static_cast<const float*>(w.ra.p);
      } else {
        rr.kind = 0;
        rr.dense = w.r64.as<double>();
      }
    }
    const bool keep = !r32 && !w.fp64 && have_x && (!direct || multi_step) && step < p.max_refine;
    if (keep) {
      if (!w.r64.p) w.r64.alloc(g->ctx, (size_t)d0.n * W * sizeof(double));
      rr.r64_out = w.r64.as<double>();
    }
    // the first residual r = b may come with the right-hand sides
    const bool pre = step == 0 && rhs.r0_rows > 0;
    if (!pre) {
      k.residual64(w.la64, have_x ? (x32 ? w.x.p : w.x64.p) : nullptr, x32 ? 1 : 0, rr, w.ra.p,
                   w.part_ptr(P_PQ), s);
      bytes += d0.n * (double)W * ((have_x ? (x32 ? 4.0 : 8.0) : 0.0) +
                                   (rr.kind == 0 ? 8.0 : (rr.kind == 2 ? 4.0 : 0.0)) + es +
                                   (keep ? 8.0 : 0.0)) +
               (have_x ? mat_bytes(d0, !d0.unit, 8) : 0.0);
    }
    r64_valid = keep;
    finalize(W, F_R64, pre ? rhs.r0_rows : gres, w.part_ptr(P_PQ), 0, nullptr, 0, nullptr,
             w.scal.as<double>(), s, w.mirror_dev);
    read_scal(S_R64, r64.data());
    if (step == 0) b2 = r64;
    bool all = true;
    cur_max = 0;
    for (int j = 0; j < W; ++j) {
      if (j >= ncols || !(b2[j] > 0)) { rel[j] = 0; continue; }
      rel[j] = (std::sqrt(r64[j]) + ebound[j]) / std::sqrt(b2[j]);
      if (!std::isfinite(rel[j])) continue;
      cur_max = std::max(cur_max, rel[j]);
      if (rel[j] > p.tol) all = false;
    }
    if (debug) {
      std::fprintf(stderr, "[cfc] W=%d prec=%d step %d max_rel %.3e (col0 %.3e)\n", W, p.precision, step,
                   cur_max, rel[0]);
    }
    if (all || step >= p.max_refine) break;
    // the next step reads this residual rounded to FP32 (ws.ra); from the
    // second step on that is the previous residual, not b
    if (r32 && step >= 1)
      for (int j = 0; j < W; ++j) ebound[j] += 0x1p-24 * std::sqrt(std::max(r64[j], 0.0));
    // Inner target as a fraction of what is left to reach tol: 0.9 when the
    // inner solve can be trusted to land near it (FP64 inner solves, or FP32
    // ones aimed straight at the target, inner_tol < 1e-6); 0.5 when FP32
    // rounding may leave the true residual above the recursive one.  Each
    // column is held to its own remaining reduction, aim tol / rel_j: one
    // block's columns can stand decades apart after a step, and those near
    // tol need not follow the worst one down.
    const double aim = direct ? 0.9 : 0.5;
    double tight = 0.5;
    for (int j = 0; j < W; ++j) {
      const double relj = (rel[j] > 0 && std::isfinite(rel[j])) ? rel[j] : std::max(cur_max, 1e-300);
      const double t = p.precision == CFC_PREC_FP64 ? std::max(aim * p.tol / relj, 1e-15)
                                                     : std::max(p.inner_tol, aim * p.tol / relj);
      itol[j] = std::min(t, 0.5);
      if (j < ncols && b2[j] > 0) tight = std::min(tight, itol[j]);
    }
    cur_step = step;
    const int its = pcg(r64, itol, p.max_inner, std::max(1, p.check_every));
    cur_step = -1;
    if (debug) std::fprintf(stderr, "[cfc]   pcg its %d (strictest inner tol %.2e)\n", its, tight);
    inner_iters += its;
    if (pairs_now) {
      pair_acc(W, ncols, static_cast<const float*>(w.x.p), rhs.ps, rhs.pt, pair_out, have_x ? 0 : 1, s);
    } else {
      k.xupdate64(d0.n, w.x64.as<double>(), w.x.p, w.scal.as<double>(), have_x ? 0 : 1, s);
      bytes += d0.n * (double)W * ((have_x ? 16.0 : 8.0) + es);
    }
    have_x = true;
    refine_steps++;
    if (step >= 1) multi_step = true;
  }
  if (!have_x) {
    if (pairs_now)
      zero_fill(pair_out, (size_t)W * sizeof(double), s);
    else
      k.zero(w.x64.p, (size_t)d0.n * W * 8, s);
  }
  pairs_now = false;
  for (int j = 0; j < ncols; ++j) {
    int32_t st = CFC_COL_OK;
    if (!(b2[j] > 0)) st = (b2[j] == 0) ? CFC_COL_SKIPPED : CFC_COL_DIVERGED;
    else if (!std::isfinite(rel[j])) st = CFC_COL_DIVERGED;
    else if (rel[j] > p.tol) st = CFC_COL_NOT_CONVERGED;
    if (status) status[j] = st;
    if (final_rel) final_rel[j] = rel[j];
    if (st == CFC_COL_OK || st == CFC_COL_SKIPPED) converged++;
    if (std::isfinite(rel[j])) max_rel = std::max(max_rel, rel[j]);
    else max_rel = INFINITY;
  }
  columns += ncols;
  blocks++;
}

Solver::Solver(Graph& gr, const cfc_solve_params& p, hipStream_t so, Ctx* mem) : g(&gr), params(p) {
  if (!g->D) fail(CFC_E_STATE, "hierarchy not built on a device (call cfc_hierarchy_build)");
  stream = so ? so : g->ctx->stream;
  const char* dbg = std::getenv("CFC_DEBUG");
  debug = dbg && dbg[0] == '1';
  const char* pe = std::getenv("CFC_PROFILE");
  profile = pe && pe[0] == '1';
  ws = &get_workspace(*g, p.block, p.precision == CFC_PREC_FP64, stream, mem);
  nuse = (p.levels >= 1 && p.levels <= ws->nlev) ? p.levels : ws->nlev;
  // FP32 inner solves whose preconditioner is one Jacobi step on level 0
  // (depth one) or an elimination level plus one Jacobi step on its Schur
  // complement: keep z as bfloat16 for the product's gathers (CFC_BF16_Z=0
  // keeps it FP32).
  const char* bz = std::getenv("CFC_BF16_Z");
  // the deepest level the cycle visits is smoothed, not solved exactly
  const bool smoothed = nuse < ws->nlev || g->D->nc == 0;
  const bool jac1 = nuse == 1 && smoothed;
  const bool elim2 = g->D->lv[0].nC > 0 && nuse == 2 && smoothed;
  // An elimination level and at least one level behind it: CG on the Schur
  // complement (CFC_SCHUR=0 keeps CG on level 0 with the elimination inside
  // the preconditioner).
  const char* sc = std::getenv("CFC_SCHUR");
  schur = g->D->lv[0].nC > 0 && nuse >= 2 && !(sc && sc[0] == '0');
  base = schur ? 1 : 0;
  jac_top = nuse - base == 1 && smoothed;
  bfz = !ws->fp64 && (jac1 || elim2) && !(bz && bz[0] == '0');
  // FP8 z (one scale per row and column slice) when the preconditioner is
  // one Jacobi step on the level the CG runs on (CFC_Z_FP8=0 keeps
  // bfloat16): with 128-column slices a gathered FP8 row is 128 bytes and
  // serves twice the columns of a bfloat16 one; R-MAT-20's operator product
  // at W = 512 measured 3.96 ms against 4.58 ms, BA-100k's 229 against
  // 258 us, with the same iteration counts
  const char* z8 = std::getenv("CFC_Z_FP8");
  zf8 = bfz && jac_top && ws->W >= 32 && !(z8 && z8[0] == '0');
  // The product kernel carries the x updates (CFC_FUSE_X=0 keeps them in
  // the update kernel).
  const char* fx = std::getenv("CFC_FUSE_X");
  xfu = !(fx && fx[0] == '0');
  CFC_HIP(hipEventCreate(&ev0));
  CFC_HIP(hipEventCreate(&ev1));
  CFC_HIP(hipEventRecord(ev0, stream));
}

Solver::~Solver() {
  for (int k = 0; k < 2; ++k) {
    if (gexec[k]) (void)hipGraphExecDestroy(gexec[k]);
    if (graph[k]) (void)hipGraphDestroy(graph[k]);
  }
  for (auto& e : prof_ev) {
    (void)hipEventDestroy(e.a);
    if (e.b) (void)hipEventDestroy(e.b);
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
}

void Solver::finish(cfc_solve_stats* st) {
  CFC_HIP(hipEventRecord(ev1, stream));
  CFC_HIP(hipEventSynchronize(ev1));
  float ms = 0;
  CFC_HIP(hipEventElapsedTime(&ms, ev0, ev1));
  prof_collect();
  if (!st) return;
  st->columns += columns;
  st->converged += converged;
  st->inner_iters += inner_iters;
  st->refine_steps += refine_steps;
  st->blocks += blocks;
  st->block_width = ws->W;
  st->precision = params.precision;
  st->levels_used = nuse;
  st->z_format = zfmt();
  st->max_rel_residual = std::max(st->max_rel_residual, max_rel);
  st->solve_ms += ms;
  st->model_bytes += bytes;
  for (int k = 0; k < 3; ++k) {
    st->kernel_ms[k] += prof_ms[k];
    st->kernel_bytes[k] += prof_bytes[k];
    st->kernel_launches[k] += prof_launches[k];
  }
}

}  // namespace cfc
