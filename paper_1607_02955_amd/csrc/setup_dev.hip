// Device side of the hierarchy setup: test-vector relaxation and edge
// affinities, Galerkin quotient graphs (P^T L P for piecewise-constant P)
// and the final renumbering of every level's CSR; with device = 2 also the
// aggregation itself (parallel handshake matching).  The elimination choice
// and the locality keys stay on the host.
//
// With device = 1 every result equals the host build bit for bit (the
// parallel aggregation of device = 2 forms other aggregates): the kernels perform the
// host's FP64 operations in the host's order with contraction switched off,
// sums over a coarse edge run over the fine edges in CSR order (a stable
// radix sort keeps that order inside each key), and a coarse row's degree
// adds its entries in ascending column order.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include "rng.hpp"
#include "setup.hpp"

namespace cfc {

namespace {

constexpr int kT = 256;

inline unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kT - 1) / kT); }

struct DevCSR {
  int64_t n = 0, nnz = 0;
  DBuf rowptr, col, w, deg, erow;  // erow[e] = row of entry e
};

__global__ void k_erow(int64_t n, const int32_t* __restrict__ rowptr, int32_t* __restrict__ erow) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  for (int32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) erow[e] = (int32_t)u;
}

// X[u, k] uniform in [-1, 1) from the counter hash of (seed, level, k, u)
__global__ void k_testvec(int64_t n, int K, uint64_t seed, int level, double* __restrict__ X) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * K) return;
  const int64_t u = i / K;
  const int k = (int)(i % K);
  const uint64_t h = key_hash(seed, kTagTestVec, uint64_t(level) * 1024 + k, uint64_t(u));
  X[i] = double(h >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

// one damped Jacobi sweep on L x = 0 for every test vector: thread (u, k),
// edges in CSR order (the host's order for every (u, k))
__global__ void k_relax(int64_t n, int K, const int32_t* __restrict__ rowptr,
                        const int32_t* __restrict__ col, const double* __restrict__ w,
                        const double* __restrict__ deg, const double* __restrict__ X,
                        double* __restrict__ Y, double om) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * K) return;
  const int64_t u = i / K;
  const int k = (int)(i % K);
  const double du = deg[u];
  const double sc = du > 0 ? om / du : 0.0;
  double acc = du * X[i];
  for (int32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) acc -= w[e] * X[(int64_t)col[e] * K + k];
  Y[i] = X[i] - sc * acc;
}

// mean of column k, summed in node order by one thread (as the host does);
// the workgroup stages chunks of the column in LDS for that thread
__global__ __launch_bounds__(256) void k_colmean(int64_t n, int K, const double* __restrict__ X,
                                                 double* __restrict__ mean) {
#pragma clang fp contract(off)
  __shared__ double buf[1024];
  const int k = blockIdx.x;
  double s = 0;
  for (int64_t base = 0; base < n; base += 1024) {
    const int64_t cnt = n - base < 1024 ? n - base : 1024;
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) buf[j] = X[(base + j) * K + k];
    __syncthreads();
    if (threadIdx.x == 0)
      for (int j = 0; j < cnt; ++j) s += buf[j];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[k] = s / double(n);
}

__global__ void k_center(int64_t n, int K, double* __restrict__ X, const double* __restrict__ mean,
                         double* __restrict__ nx) {
#pragma clang fp contract(off)
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  for (int k = 0; k < K; ++k) X[u * K + k] -= mean[k];
  double s = 0;
  for (int k = 0; k < K; ++k) s += X[u * K + k] * X[u * K + k];
  nx[u] = s;
}

__global__ void k_affinity(int64_t nnz, int K, const int32_t* __restrict__ erow,
                           const int32_t* __restrict__ col, const double* __restrict__ w,
                           const double* __restrict__ X, const double* __restrict__ nx,
                           double* __restrict__ aff) {
#pragma clang fp contract(off)
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int64_t u = erow[e], v = col[e];
  double s = 0;
  for (int k = 0; k < K; ++k) s += X[u * K + k] * X[v * K + k];
  const double den = nx[u] * nx[v];
  const double a = den > 0 ? s * s / den : 0.0;
  aff[e] = a * (1.0 + 1e-12 * w[e]);
}

// ---- parallel aggregation (device = 2) --------------------------------------
// Handshake matching on the affinities: every unassigned node picks its
// strongest unassigned neighbour (ties to the lower id); two nodes that pick
// each other form an aggregate labelled by the lower id.  After a few rounds
// every node still unassigned joins the aggregate of its strongest assigned
// neighbour, and a node with none founds its own.  All steps read labels of
// the previous step only, so the result does not depend on thread order.

__global__ void k_agg_pick(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                           const double* __restrict__ aff, const int32_t* __restrict__ agg,
                           int32_t* __restrict__ pick) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int32_t best = -1;
  double ba = -1.0;
  if (agg[u] < 0)
    for (int32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
      const int32_t v = col[e];
      if (agg[v] >= 0) continue;
      const double a = aff[e];
      if (a > ba || (a == ba && v < best)) {
        ba = a;
        best = v;
      }
    }
  pick[u] = best;
}

__global__ void k_agg_match(int64_t n, const int32_t* __restrict__ pick, int32_t* __restrict__ agg,
                            int32_t* __restrict__ matched) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  const int32_t v = pick[u];
  if (v > u && pick[v] == (int32_t)u) {  // mutual: the lower id writes both labels
    agg[u] = (int32_t)u;
    agg[v] = (int32_t)u;
    matched[0] = 1;
  }
}

// unassigned u -> label of its strongest assigned neighbour (or its own id
// when found = 1 and it has none); assigned nodes keep theirs
__global__ void k_agg_attach(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                             const double* __restrict__ aff, const int32_t* __restrict__ agg,
                             int32_t* __restrict__ out, int found) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int32_t lab = agg[u];
  if (lab < 0) {
    int32_t best = -1;
    double ba = -1.0;
    for (int32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
      const int32_t v = col[e];
      if (agg[v] < 0) continue;
      const double a = aff[e];
      if (a > ba || (a == ba && v < best)) {
        ba = a;
        best = v;
      }
    }
    lab = best >= 0 ? agg[best] : (found ? (int32_t)u : -1);
  }
  out[u] = lab;
}

// Matching between aggregates (labels are root ids): every edge between two
// aggregates offers its affinity to the aggregate of its row; each aggregate
// keeps the largest offer from an aggregate it may merge with (the merged
// size within cap), ties to the lower label.  The offer is packed as
// (float bits of the affinity, ~label) so one 64-bit atomicMax keeps it; the
// maximum does not depend on the order of the atomics.
__global__ void k_agg_size(int64_t n, const int32_t* __restrict__ lab, int32_t* __restrict__ size) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) atomicAdd(&size[lab[u]], 1);
}

__global__ void k_agg_offer(int64_t nnz, const int32_t* __restrict__ erow, const int32_t* __restrict__ col,
                            const double* __restrict__ aff, const int32_t* __restrict__ lab,
                            const int32_t* __restrict__ size, int cap,
                            unsigned long long* __restrict__ best) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const int32_t A = lab[erow[e]], B = lab[col[e]];
  if (A == B || size[A] + size[B] > cap) return;
  const float a = (float)aff[e];  // affinities are >= 0, so the bits order like the values
  const unsigned long long key = ((unsigned long long)__float_as_uint(a) << 32) | (0xFFFFFFFFull - (uint32_t)B);
  atomicMax(&best[A], key);
}

__global__ void k_agg_merge(int64_t n, const int32_t* __restrict__ lab, const unsigned long long* __restrict__ best,
                            int32_t* __restrict__ into, int32_t* __restrict__ merged) {
  const int64_t A = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= n || lab[A] != (int32_t)A || best[A] == 0) return;
  const int32_t B = (int32_t)(0xFFFFFFFFull - (best[A] & 0xFFFFFFFFull));
  if (B <= A || best[B] == 0) return;
  const int32_t back = (int32_t)(0xFFFFFFFFull - (best[B] & 0xFFFFFFFFull));
  if (back == (int32_t)A) {  // mutual: B's members take label A
    into[B] = (int32_t)A;
    merged[0] = 1;
  }
}

__global__ void k_agg_iota(int64_t n, int32_t* __restrict__ x) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) x[u] = (int32_t)u;
}

__global__ void k_agg_relabel(int64_t n, const int32_t* __restrict__ lab, const int32_t* __restrict__ into,
                              int32_t* __restrict__ out) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) out[u] = into[lab[u]];
}

__global__ void k_agg_roots(int64_t n, const int32_t* __restrict__ agg, int32_t* __restrict__ root) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) root[u] = agg[u] == (int32_t)u ? 1 : 0;
}

__global__ void k_agg_compact(int64_t n, const int32_t* __restrict__ agg, const int32_t* __restrict__ id,
                              int32_t* __restrict__ out) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) out[u] = id[agg[u]];
}

constexpr uint64_t kNoKey = ~0ull;

// coarse key (I, J) of every fine entry; entries inside an aggregate sort last
__global__ void k_gal_keys(int64_t nnz, const int32_t* __restrict__ erow,
                           const int32_t* __restrict__ col, const int32_t* __restrict__ agg,
                           uint64_t* __restrict__ key) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const uint32_t I = (uint32_t)agg[erow[e]], J = (uint32_t)agg[col[e]];
  key[e] = I == J ? kNoKey : ((uint64_t)I << 32) | J;
}

// first index of every run of equal keys among the nv valid sorted keys
__global__ void k_run_flags(int64_t nv, const uint64_t* __restrict__ key, int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  flag[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void k_run_starts(int64_t nv, const int32_t* __restrict__ flag,
                             const int32_t* __restrict__ rid, int32_t* __restrict__ start) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  if (flag[i]) start[rid[i]] = (int32_t)i;
}

// coarse entry r: weight = fine weights of its run added left to right
__global__ void k_run_sum(int64_t nruns, int64_t nv, const int32_t* __restrict__ start,
                          const uint64_t* __restrict__ key, const double* __restrict__ val,
                          int32_t* __restrict__ crow, int32_t* __restrict__ ccol,
                          double* __restrict__ cw) {
#pragma clang fp contract(off)
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nruns) return;
  const int64_t a = start[r], b = r + 1 < nruns ? start[r + 1] : nv;
  double s = 0;
  for (int64_t i = a; i < b; ++i) s += val[i];
  cw[r] = s;
  crow[r] = (int32_t)(key[a] >> 32);
  ccol[r] = (int32_t)(key[a] & 0xffffffffu);
}

// row pointers of the coarse CSR from the sorted entry rows
__global__ void k_rowptr(int64_t nruns, int64_t nc, const int32_t* __restrict__ crow,
                         int32_t* __restrict__ rowptr) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nruns) return;
  const int32_t lo = r == 0 ? 0 : crow[r - 1] + 1;
  for (int32_t I = lo; I <= crow[r]; ++I) rowptr[I] = (int32_t)r;
  if (r == nruns - 1)
    for (int64_t I = crow[r] + 1; I <= nc; ++I) rowptr[I] = (int32_t)nruns;
}

__global__ void k_rowsum(int64_t nc, const int32_t* __restrict__ rowptr, const double* __restrict__ cw,
                         double* __restrict__ deg) {
#pragma clang fp contract(off)
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  double d = 0;
  for (int32_t r = rowptr[I]; r < rowptr[I + 1]; ++r) d += cw[r];
  deg[I] = d;
}

__global__ void k_renum_keys(int64_t nnz, const int32_t* __restrict__ erow,
                             const int32_t* __restrict__ col, const int32_t* __restrict__ newid,
                             uint64_t* __restrict__ key) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  key[e] = ((uint64_t)(uint32_t)newid[erow[e]] << 32) | (uint32_t)newid[col[e]];
}

__global__ void k_low_word(int64_t nnz, const uint64_t* __restrict__ key, int32_t* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  out[e] = (int32_t)(key[e] & 0xffffffffu);
}

template <class T>
void put(Ctx* c, DBuf& d, const std::vector<T>& h, hipStream_t s) {
  d.alloc(c, std::max<size_t>(1, h.size()) * sizeof(T));
  if (!h.empty()) CFC_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  CFC_HIP(hipStreamSynchronize(s));
}

template <class T>
void get(std::vector<T>& h, const DBuf& d, size_t count, hipStream_t s) {
  h.resize(count);
  if (count) CFC_HIP(hipMemcpyAsync(h.data(), d.p, count * sizeof(T), hipMemcpyDeviceToHost, s));
  CFC_HIP(hipStreamSynchronize(s));
}

}  // namespace

struct DeviceSetup::Impl {
  Ctx* ctx;
  hipStream_t s;
  std::vector<std::unique_ptr<DevCSR>> lv;
  DBuf tmp;  // radix-sort / scan scratch
  DBuf aff;  // affinities kept for the device aggregation of level aff_lv
  int aff_lv = -1;

  void* scratch(size_t bytes) {
    if (tmp.bytes < bytes) tmp.alloc(ctx, bytes);
    return tmp.p;
  }
  // stable LSD radix sort of (key, val) pairs by the low `bits` bits
  template <class V>
  void sort_pairs(const uint64_t* kin, uint64_t* kout, const V* vin, V* vout, int64_t n, int bits) {
    size_t bytes = 0;
    CFC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, kin, kout, vin, vout, n, 0, bits, s));
    void* t = scratch(bytes);
    CFC_HIP(hipcub::DeviceRadixSort::SortPairs(t, bytes, kin, kout, vin, vout, n, 0, bits, s));
  }
};

DeviceSetup::DeviceSetup(Ctx* ctx) : d(std::make_unique<Impl>()) {
  d->ctx = ctx;
  d->s = ctx->stream;
  CFC_HIP(hipSetDevice(ctx->device));
}

DeviceSetup::~DeviceSetup() = default;

int DeviceSetup::add(const BLevel& L) {
  auto c = std::make_unique<DevCSR>();
  c->n = L.n;
  c->nnz = (int64_t)L.col.size();
  put(d->ctx, c->rowptr, L.rowptr, d->s);
  put(d->ctx, c->col, L.col, d->s);
  put(d->ctx, c->w, L.w, d->s);
  put(d->ctx, c->deg, L.deg, d->s);
  c->erow.alloc(d->ctx, std::max<int64_t>(1, c->nnz) * sizeof(int32_t));
  if (c->n)
    hipLaunchKernelGGL(k_erow, dim3(blocks_for(c->n)), dim3(kT), 0, d->s, c->n, c->rowptr.as<int32_t>(),
                       c->erow.as<int32_t>());
  d->lv.push_back(std::move(c));
  return (int)d->lv.size() - 1;
}

std::vector<double> DeviceSetup::affinities(int lv, int level, const cfc_setup_params& p, bool keep) {
  const DevCSR& c = *d->lv[lv];
  const int64_t n = c.n;
  const int K = std::max(1, p.test_vectors);
  hipStream_t s = d->s;
  std::vector<double> out;
  if (n == 0) return out;
  DBuf X, Y, mean, nx, aff;
  X.alloc(d->ctx, n * K * 8);
  Y.alloc(d->ctx, n * K * 8);
  nx.alloc(d->ctx, n * 8);
  mean.alloc(d->ctx, 64 * 8);
  aff.alloc(d->ctx, std::max<int64_t>(1, c.nnz) * 8);
  hipLaunchKernelGGL(k_testvec, dim3(blocks_for(n * K)), dim3(kT), 0, s, n, K, p.seed, level,
                     X.as<double>());
  const double om = 0.6;  // the host build's relaxation weight
  for (int sw = 0; sw < p.relax_sweeps; ++sw) {
    hipLaunchKernelGGL(k_relax, dim3(blocks_for(n * K)), dim3(kT), 0, s, n, K, c.rowptr.as<int32_t>(),
                       c.col.as<int32_t>(), c.w.as<double>(), c.deg.as<double>(), X.as<double>(),
                       Y.as<double>(), om);
    std::swap(X.p, Y.p);
  }
  hipLaunchKernelGGL(k_colmean, dim3(K), dim3(256), 0, s, n, K, X.as<double>(), mean.as<double>());
  hipLaunchKernelGGL(k_center, dim3(blocks_for(n)), dim3(kT), 0, s, n, K, X.as<double>(),
                     mean.as<double>(), nx.as<double>());
  if (c.nnz)
    hipLaunchKernelGGL(k_affinity, dim3(blocks_for(c.nnz)), dim3(kT), 0, s, c.nnz, K,
                       c.erow.as<int32_t>(), c.col.as<int32_t>(), c.w.as<double>(), X.as<double>(),
                       nx.as<double>(), aff.as<double>());
  if (keep) {
    d->aff = std::move(aff);
    d->aff_lv = lv;
    return out;
  }
  get(out, aff, c.nnz, s);
  return out;
}

int64_t DeviceSetup::aggregate(int lv, int cap, std::vector<int32_t>& agg) {
  const DevCSR& c = *d->lv[lv];
  if (d->aff_lv != lv) fail(CFC_E_INTERNAL, "device affinities are not those of this level");
  const int64_t n = c.n;
  hipStream_t s = d->s;
  agg.assign(n, 0);
  if (n == 0) return 0;
  DBuf a0, a1, pick, flag, root, id;
  a0.alloc(d->ctx, n * 4);
  a1.alloc(d->ctx, n * 4);
  pick.alloc(d->ctx, n * 4);
  flag.alloc(d->ctx, 4);
  root.alloc(d->ctx, n * 4);
  id.alloc(d->ctx, n * 4);
  std::vector<int32_t> init(n, -1);
  CFC_HIP(hipMemcpyAsync(a0.p, init.data(), n * 4, hipMemcpyHostToDevice, s));
  const int32_t* rp = c.rowptr.as<int32_t>();
  const int32_t* cl = c.col.as<int32_t>();
  const double* af = d->aff.as<double>();
  // Matching rounds until one pairs nobody: the affinities are symmetric and
  // ties go to the lower id, so while an edge joins two unassigned nodes the
  // strongest such edge is a mutual pick, and a round without a match means
  // every unassigned node has only assigned neighbours (or none).  Then the
  // unassigned join an assigned neighbour (or found their own aggregate).
  // A round cap bounds the work; a capped pass attaches what it can and
  // starts again.
  for (int outer = 0; outer < 64; ++outer) {
    int32_t m = 1;
    for (int r = 0; r < 32 && m; ++r) {
      int32_t zero = 0;
      CFC_HIP(hipMemcpyAsync(flag.p, &zero, 4, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_agg_pick, dim3(blocks_for(n)), dim3(kT), 0, s, n, rp, cl, af, a0.as<int32_t>(),
                         pick.as<int32_t>());
      hipLaunchKernelGGL(k_agg_match, dim3(blocks_for(n)), dim3(kT), 0, s, n, pick.as<int32_t>(),
                         a0.as<int32_t>(), flag.as<int32_t>());
      CFC_HIP(hipMemcpyAsync(&m, flag.p, 4, hipMemcpyDeviceToHost, s));
      CFC_HIP(hipStreamSynchronize(s));
    }
    const int found = (m == 0 || outer == 63) ? 1 : 0;
    hipLaunchKernelGGL(k_agg_attach, dim3(blocks_for(n)), dim3(kT), 0, s, n, rp, cl, af, a0.as<int32_t>(),
                       a1.as<int32_t>(), found);
    std::swap(a0.p, a1.p);
    get(agg, a0, n, s);
    bool done = true;
    for (int64_t u = 0; u < n && done; ++u) done = agg[u] >= 0;
    if (done) break;
  }
  for (int64_t u = 0; u < n; ++u)
    if (agg[u] < 0) fail(CFC_E_INTERNAL, "device aggregation left a node unplaced");
  // Two rounds of matching between aggregates (pairs of pairs), each merge
  // within agg_cap nodes: coarsening by about four per level, as the host's
  // greedy pass does (pairs alone coarsen by ~2.2, which the complexity
  // budget cuts off long before the coarsest level on road grids).
  {
    DBuf size, best, into;
    size.alloc(d->ctx, n * 4);
    best.alloc(d->ctx, n * 8);
    into.alloc(d->ctx, n * 4);
    for (int r = 0; r < 2; ++r) {
      CFC_HIP(hipMemsetAsync(size.p, 0, n * 4, s));
      CFC_HIP(hipMemsetAsync(best.p, 0, n * 8, s));
      int32_t zero = 0, m = 0;
      CFC_HIP(hipMemcpyAsync(flag.p, &zero, 4, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_agg_size, dim3(blocks_for(n)), dim3(kT), 0, s, n, a0.as<int32_t>(), size.as<int32_t>());
      if (c.nnz)
        hipLaunchKernelGGL(k_agg_offer, dim3(blocks_for(c.nnz)), dim3(kT), 0, s, c.nnz, c.erow.as<int32_t>(), cl,
                           af, a0.as<int32_t>(), size.as<int32_t>(), cap, best.as<unsigned long long>());
      hipLaunchKernelGGL(k_agg_iota, dim3(blocks_for(n)), dim3(kT), 0, s, n, into.as<int32_t>());
      hipLaunchKernelGGL(k_agg_merge, dim3(blocks_for(n)), dim3(kT), 0, s, n, a0.as<int32_t>(),
                         best.as<unsigned long long>(), into.as<int32_t>(), flag.as<int32_t>());
      hipLaunchKernelGGL(k_agg_relabel, dim3(blocks_for(n)), dim3(kT), 0, s, n, a0.as<int32_t>(),
                         into.as<int32_t>(), a1.as<int32_t>());
      std::swap(a0.p, a1.p);
      CFC_HIP(hipMemcpyAsync(&m, flag.p, 4, hipMemcpyDeviceToHost, s));
      CFC_HIP(hipStreamSynchronize(s));
      if (!m) break;
    }
  }
  // aggregates numbered in order of their root (the lower id of the pair)
  hipLaunchKernelGGL(k_agg_roots, dim3(blocks_for(n)), dim3(kT), 0, s, n, a0.as<int32_t>(), root.as<int32_t>());
  size_t bytes = 0;
  CFC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, root.as<int32_t>(), id.as<int32_t>(), n, s));
  void* t = d->scratch(bytes);
  CFC_HIP(hipcub::DeviceScan::ExclusiveSum(t, bytes, root.as<int32_t>(), id.as<int32_t>(), n, s));
  hipLaunchKernelGGL(k_agg_compact, dim3(blocks_for(n)), dim3(kT), 0, s, n, a0.as<int32_t>(), id.as<int32_t>(),
                     a1.as<int32_t>());
  get(agg, a1, n, s);
  int64_t nc = 0;
  for (int64_t u = 0; u < n; ++u) nc = std::max<int64_t>(nc, (int64_t)agg[u] + 1);
  return nc;
}

int DeviceSetup::galerkin(int lv, const std::vector<int32_t>& agg, int64_t nc, BLevel& C) {
  const DevCSR& f = *d->lv[lv];
  hipStream_t s = d->s;
  Ctx* ctx = d->ctx;
  auto cc = std::make_unique<DevCSR>();
  cc->n = nc;
  DBuf dagg, key, key2, val2;
  put(ctx, dagg, agg, s);
  const int64_t nnz = f.nnz;
  const size_t m = (size_t)std::max<int64_t>(1, nnz);
  key.alloc(ctx, m * 8);
  key2.alloc(ctx, m * 8);
  val2.alloc(ctx, m * 8);
  int64_t nv = 0, nruns = 0;
  if (nnz) {
    hipLaunchKernelGGL(k_gal_keys, dim3(blocks_for(nnz)), dim3(kT), 0, s, nnz, f.erow.as<int32_t>(),
                       f.col.as<int32_t>(), dagg.as<int32_t>(), key.as<uint64_t>());
    d->sort_pairs(key.as<uint64_t>(), key2.as<uint64_t>(), f.w.as<double>(), val2.as<double>(), nnz, 64);
    // valid keys come first; count them from the sorted order
    std::vector<uint64_t> probe;
    int64_t lo = 0, hi = nnz;  // first index holding kNoKey
    while (lo < hi) {
      const int64_t mid = (lo + hi) / 2;
      uint64_t kv = 0;
      CFC_HIP(hipMemcpyAsync(&kv, key2.as<uint64_t>() + mid, 8, hipMemcpyDeviceToHost, s));
      CFC_HIP(hipStreamSynchronize(s));
      if (kv == kNoKey) hi = mid;
      else lo = mid + 1;
    }
    nv = lo;
  }
  DBuf flag, rid, start;
  if (nv) {
    flag.alloc(ctx, nv * 4);
    rid.alloc(ctx, nv * 4);
    hipLaunchKernelGGL(k_run_flags, dim3(blocks_for(nv)), dim3(kT), 0, s, nv, key2.as<uint64_t>(),
                       flag.as<int32_t>());
    size_t bytes = 0;
    CFC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, flag.as<int32_t>(), rid.as<int32_t>(), nv, s));
    void* t = d->scratch(bytes);
    CFC_HIP(hipcub::DeviceScan::ExclusiveSum(t, bytes, flag.as<int32_t>(), rid.as<int32_t>(), nv, s));
    int32_t last_rid = 0, last_flag = 0;
    CFC_HIP(hipMemcpyAsync(&last_rid, rid.as<int32_t>() + nv - 1, 4, hipMemcpyDeviceToHost, s));
    CFC_HIP(hipMemcpyAsync(&last_flag, flag.as<int32_t>() + nv - 1, 4, hipMemcpyDeviceToHost, s));
    CFC_HIP(hipStreamSynchronize(s));
    nruns = (int64_t)last_rid + last_flag;
    start.alloc(ctx, nruns * 4);
    hipLaunchKernelGGL(k_run_starts, dim3(blocks_for(nv)), dim3(kT), 0, s, nv, flag.as<int32_t>(),
                       rid.as<int32_t>(), start.as<int32_t>());
  }
  cc->nnz = nruns;
  DBuf crow;
  crow.alloc(ctx, std::max<int64_t>(1, nruns) * 4);
  cc->col.alloc(ctx, std::max<int64_t>(1, nruns) * 4);
  cc->w.alloc(ctx, std::max<int64_t>(1, nruns) * 8);
  cc->rowptr.alloc(ctx, (nc + 1) * 4);
  cc->deg.alloc(ctx, std::max<int64_t>(1, nc) * 8);
  cc->erow.alloc(ctx, std::max<int64_t>(1, nruns) * 4);
  if (nruns) {
    hipLaunchKernelGGL(k_run_sum, dim3(blocks_for(nruns)), dim3(kT), 0, s, nruns, nv, start.as<int32_t>(),
                       key2.as<uint64_t>(), val2.as<double>(), crow.as<int32_t>(), cc->col.as<int32_t>(),
                       cc->w.as<double>());
    hipLaunchKernelGGL(k_rowptr, dim3(blocks_for(nruns)), dim3(kT), 0, s, nruns, nc, crow.as<int32_t>(),
                       cc->rowptr.as<int32_t>());
  } else {
    std::vector<int32_t> z(nc + 1, 0);
    CFC_HIP(hipMemcpyAsync(cc->rowptr.p, z.data(), (nc + 1) * 4, hipMemcpyHostToDevice, s));
    CFC_HIP(hipStreamSynchronize(s));
  }
  if (nc)
    hipLaunchKernelGGL(k_rowsum, dim3(blocks_for(nc)), dim3(kT), 0, s, nc, cc->rowptr.as<int32_t>(),
                       cc->w.as<double>(), cc->deg.as<double>());
  if (nc)
    hipLaunchKernelGGL(k_erow, dim3(blocks_for(nc)), dim3(kT), 0, s, nc, cc->rowptr.as<int32_t>(),
                       cc->erow.as<int32_t>());
  C = BLevel();
  C.n = nc;
  get(C.rowptr, cc->rowptr, nc + 1, s);
  get(C.col, cc->col, nruns, s);
  get(C.w, cc->w, nruns, s);
  get(C.deg, cc->deg, nc, s);
  d->lv.push_back(std::move(cc));
  return (int)d->lv.size() - 1;
}

void DeviceSetup::renumber(int lv, const std::vector<int32_t>& newid, std::vector<int32_t>& col,
                           std::vector<double>& w) {
  const DevCSR& f = *d->lv[lv];
  hipStream_t s = d->s;
  Ctx* ctx = d->ctx;
  const int64_t nnz = f.nnz;
  col.clear();
  w.clear();
  if (!nnz) return;
  DBuf nid, key, key2, val2, c32;
  put(ctx, nid, newid, s);
  key.alloc(ctx, nnz * 8);
  key2.alloc(ctx, nnz * 8);
  val2.alloc(ctx, nnz * 8);
  c32.alloc(ctx, nnz * 4);
  hipLaunchKernelGGL(k_renum_keys, dim3(blocks_for(nnz)), dim3(kT), 0, s, nnz, f.erow.as<int32_t>(),
                     f.col.as<int32_t>(), nid.as<int32_t>(), key.as<uint64_t>());
  d->sort_pairs(key.as<uint64_t>(), key2.as<uint64_t>(), f.w.as<double>(), val2.as<double>(), nnz, 64);
  hipLaunchKernelGGL(k_low_word, dim3(blocks_for(nnz)), dim3(kT), 0, s, nnz, key2.as<uint64_t>(),
                     c32.as<int32_t>());
  get(col, c32, nnz, s);
  get(w, val2, nnz, s);
}

}  // namespace cfc
