// Allocation-free variant of the projection farness query
// (cfc_farness_jl_static): the same reduction as cfc_farness_jl (Sec. 5.2:
// f(v) = n |Z_v|^2 + |Z|_F^2 from the resident sketch, c = (n-1)/f) for
// callers that cannot allocate device memory.  Its staging lives in a
// file-scope device array of fixed size instead of buffers allocated per
// call.
//
// The array's name is only a host-side stand-in: the device address of each
// GPU's copy is looked up once per device (hipGetSymbolAddress, with that
// device current) when a context is created on it, and only that address is
// passed to kernels and copies.  Every call on one GPU shares that GPU's
// copy; calls that overlap on one GPU (two host threads, or two streams)
// race on it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "internal.hpp"

namespace cfc {

// Query nodes per call (the staging holds the node ids and both outputs).
constexpr int64_t kStaticMaxNodes = int64_t(1) << 18;
constexpr int kMaxDevices = 64;

struct StaticStage {
  int64_t nodes[kStaticMaxNodes];
  double far[kStaticMaxNodes];
  double clo[kStaticMaxNodes];
  int bad;  // set by the kernel when a node id is out of range
};

static __device__ __align__(256) StaticStage scratch;

static std::mutex g_scratch_mu;
static StaticStage* g_scratch_ptr[kMaxDevices] = {};

// Set-up for `device` (current on the calling thread): record the device
// address of this GPU's copy of the staging array.  Called by
// cfc_ctx_create; idempotent.
void noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) fail(CFC_E_INVALID, "device index beyond the staging table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  CFC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) fail(CFC_E_DEVICE, "no device address for the static staging array");
  g_scratch_ptr[device] = static_cast<StaticStage*>(ptr);
}

static StaticStage* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

__global__ void k_static_clear(StaticStage* __restrict__ st) { st->bad = 0; }

// far[i] = n N[perm[v_i]] + S2 and clo[i] = (n - 1) / far[i] for the q staged
// nodes (all_nodes: v_i = i); an id outside [0, n) sets st->bad.  Products and sums are rounded separately, as
// the host arithmetic of cfc_farness_jl rounds them (the two can still differ
// by one rounding where the host compiler contracts the pair).
__global__ __launch_bounds__(256) void k_jl_farness_static(int64_t q, int all_nodes, double n,
                                                           const int* __restrict__ perm,
                                                           const double* __restrict__ N, double S2,
                                                           StaticStage* __restrict__ st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q) return;
  const int64_t v = all_nodes ? i : st->nodes[i];
  if (v < 0 || v >= (int64_t)n) {
    st->bad = 1;
    st->far[i] = st->clo[i] = NAN;
    return;
  }
  const double f = __dadd_rn(__dmul_rn(n, N[perm[v]]), S2);
  st->far[i] = f;
  st->clo[i] = f > 0 ? (n - 1.0) / f : INFINITY;
}

}  // namespace cfc

using namespace cfc;

extern "C" int cfc_farness_jl_static(cfc_graph* gg, int64_t q, const int64_t* nodes, double* far,
                                     double* clo) {
  try {
    if (!gg) fail(CFC_E_INVALID, "graph is NULL");
    Graph* g = reinterpret_cast<Graph*>(gg);
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->server.load()) fail(CFC_E_STATE, "graph is registered with a server (destroy the server first)");
    if (g->ctx->host_only()) fail(CFC_E_STATE, "context has no device");
    if (!g->D) fail(CFC_E_STATE, "hierarchy not built (call cfc_hierarchy_build)");
    if (!g->jl.valid) fail(CFC_E_STATE, "no projection sketch (call cfc_jl_sketch)");
    const bool all = nodes == nullptr;
    if (q < 0 || (q > 0 && !far) || (all && q != g->n))
      fail(CFC_E_INVALID, "bad arguments (nodes = NULL requires q = n)");
    if (q > kStaticMaxNodes)
      fail(CFC_E_INVALID, "at most " + std::to_string(kStaticMaxNodes) + " nodes per call");
    if (q == 0) return CFC_OK;
    CFC_HIP(hipSetDevice(g->ctx->device));
    StaticStage* st = scratch_of(g->ctx->device);
    if (!st) fail(CFC_E_STATE, "static staging not set up on this device");
    hipStream_t s = g->ctx->stream;
    // node ids may sit in host or device memory: they are range-checked by
    // the kernel, which flags a bad id in the staging array
    hipLaunchKernelGGL(k_static_clear, dim3(1), dim3(1), 0, s, st);
    if (!all)
      CFC_HIP(hipMemcpyAsync(st->nodes, nodes, (size_t)q * sizeof(int64_t), hipMemcpyDefault, s));
    hipLaunchKernelGGL(k_jl_farness_static, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, q,
                       all ? 1 : 0, (double)g->n, g->D->perm.as<int>(), g->jl.N_dev.as<double>(),
                       g->jl.S2, st);
    CFC_HIP(hipGetLastError());
    int bad = 0;
    CFC_HIP(hipMemcpyAsync(&bad, &st->bad, sizeof(int), hipMemcpyDeviceToHost, s));
    CFC_HIP(hipMemcpyAsync(far, st->far, (size_t)q * sizeof(double), hipMemcpyDefault, s));
    if (clo) CFC_HIP(hipMemcpyAsync(clo, st->clo, (size_t)q * sizeof(double), hipMemcpyDefault, s));
    CFC_HIP(hipStreamSynchronize(s));
    if (bad) fail(CFC_E_INVALID, "node id out of range");
    return CFC_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return CFC_E_INTERNAL;
  }
}
