// Device side of the hierarchy setup: test-vector relaxation and edge
// affinities, Galerkin quotient graphs (P^T L P for piecewise-constant P)
// and the final renumbering of every level's CSR.  The greedy aggregation,
// the elimination choice and the Cuthill-McKee keys stay on the host.
//
// Every result equals the host build bit for bit: the kernels perform the
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

std::vector<double> DeviceSetup::affinities(int lv, int level, const cfc_setup_params& p) {
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
  get(out, aff, c.nnz, s);
  return out;
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
