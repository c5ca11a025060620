/*
 * cfc.h -- C ABI of libcfc: current-flow closeness on AMD Instinct MI355X.
 *
 * The calls follow the problem statement of Bergamini, Wegner, Lukarski and
 * Meyerhenke, "Estimating Current-Flow Closeness Centrality with a Multigrid
 * Laplacian Solver" (arXiv 1607.02955):
 *   - a connected, undirected graph whose edge weights are conductances
 *     (Sec. 2, "Graph basics" and "Graphs as electrical networks");
 *   - its Laplacian L = D - A and the systems L p = b with sum(b) = 0,
 *     solved to a relative residual ||b - L p|| / ||b|| <= tau (Eq. 1;
 *     Sec. 3.1);
 *   - effective resistance, electrical farness and current-flow closeness
 *     (Sec. 4, Eq. 3);
 *   - the exact method (n-1 solves, Sec. 4), the Sampling estimator
 *     (Sec. 5.1, Prop. 1) and the projection estimator (Sec. 5.2,
 *     Algorithm 1).
 *
 * Conventions for every call:
 *   - Every call returns CFC_OK or a negative CFC_E_* status; no C++
 *     exception crosses the ABI.  cfc_last_error() gives a message for the
 *     last failing call on the calling thread.  Outputs are unspecified on
 *     error (except col_status, which is always written when non-NULL).
 *   - Input arrays stay owned by the caller; the library copies what it
 *     keeps.  Outputs are caller-allocated.  Array arguments documented as
 *     "host or device" may be either a host pointer or a device pointer on
 *     the context's GPU (the library tells them apart with
 *     hipPointerGetAttributes and copies accordingly).
 *   - Node ids are int64 in [0, n) where n is the node count of the loaded
 *     graph (after CFC_LCC_ONLY relabelling, see cfc_graph_load).
 *   - Device memory is owned by the library until the owning object is
 *     destroyed; it comes from the context's allocator.
 *   - A cfc_graph may be used by one thread at a time.  cfc_server calls are
 *     thread-safe.
 */
#ifndef CFC_H
#define CFC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define CFC_OK                 0
#define CFC_E_INVALID         -1  /* bad argument, id out of range, bad weight */
#define CFC_E_DISCONNECTED    -2  /* graph not connected (and no CFC_LCC_ONLY) */
#define CFC_E_NOMEM           -3  /* allocation failed or HBM budget exceeded */
#define CFC_E_DEVICE          -4  /* HIP runtime error */
#define CFC_E_NOT_CONVERGED   -5  /* some column missed the tolerance */
#define CFC_E_STATE           -6  /* call out of order / result pending */
#define CFC_E_BUSY            -7  /* server queue full */
#define CFC_E_CANCELLED       -8  /* query cancelled */
#define CFC_E_INTERNAL        -9  /* unexpected internal failure */

/* per-column status written to col_status arrays */
#define CFC_COL_OK             0
#define CFC_COL_NOT_CONVERGED  1  /* iteration caps reached above tolerance */
#define CFC_COL_DIVERGED       2  /* non-finite residual */
#define CFC_COL_SKIPPED        3  /* zero right-hand side: solution 0 */

/* graph load flags */
#define CFC_LCC_ONLY           1u /* keep the largest connected component */
#define CFC_REJECT_PARALLEL    2u /* error on repeated edges instead of summing */

/* solve precision */
#define CFC_PREC_MIXED         0  /* FP32 multigrid-PCG inside FP64 refinement */
#define CFC_PREC_FP64          1  /* FP64 multigrid-PCG throughout */

#define CFC_MAX_LEVELS        32
#define CFC_ELIM_MAX_DEGREE    4  /* eliminated nodes have at most this degree */

typedef struct cfc_ctx cfc_ctx;
typedef struct cfc_graph cfc_graph;
typedef struct cfc_server cfc_server;

typedef void* (*cfc_alloc_fn)(size_t bytes, void* user);
typedef void (*cfc_free_fn)(void* ptr, void* user);

typedef struct {
  int32_t device;       /* HIP device ordinal; -1 = host-only context
                           (graph ingest and hierarchy setup, no solves) */
  void* stream;         /* hipStream_t for all device work; NULL = the library
                           creates a default-priority stream of its own */
  cfc_alloc_fn alloc;   /* device allocator (e.g. PyTorch's caching
                           allocator); NULL = hipMalloc */
  cfc_free_fn free;     /* matching free; NULL = hipFree */
  void* user;           /* passed to alloc/free */
  uint64_t hbm_budget;  /* bytes of device memory the context may hold;
                           0 = no limit */
} cfc_ctx_opts;

typedef struct {
  int64_t n;                       /* nodes of the loaded graph */
  int64_t m;                       /* undirected edges after canonicalisation */
  int64_t input_n;                 /* node count given to cfc_graph_load */
  int32_t levels;                  /* multigrid levels (0 = no hierarchy yet) */
  int32_t unit_weights;            /* 1 if every weight is 1 */
  int64_t level_n[CFC_MAX_LEVELS];
  int64_t level_nnz[CFC_MAX_LEVELS];  /* off-diagonal entries, both directions */
  double operator_complexity;      /* sum of level nnz+n over level-0 nnz+n */
  double setup_ms;                 /* host hierarchy build time */
  uint64_t device_bytes;           /* device memory held by the graph */
  int32_t max_degree;
  int32_t eliminated;              /* nodes removed by the elimination level
                                      (0 = none) */
  double cycle_complexity;         /* the same sum from the first aggregated
                                      level a on, over level a's nnz+n (a = 1
                                      behind an elimination level: the inner
                                      solve iterates on its Schur complement) */
} cfc_graph_info;

typedef struct {
  int32_t coarsest_max;  /* stop coarsening at or below this many nodes (512) */
  int32_t agg_cap;       /* maximum aggregate size (8) */
  int32_t test_vectors;  /* relaxed vectors that define affinities (8) */
  int32_t relax_sweeps;  /* relaxation sweeps per test vector (8) */
  double omega;          /* Jacobi smoothing weight (0.8) */
  double mu;             /* coarse-correction scale, 0 < mu < 2 (1.5) */
  uint64_t seed;         /* test-vector seed (1) */
  int32_t eliminate;     /* low-degree elimination level (Sec. 3.1: LAMG
                            alternates elimination and aggregation): an
                            independent set of nodes of degree at most
                            elim_degree is removed exactly by a Schur
                            complement before aggregating.  0 = off, 1 =
                            when it removes at least 5% of the nodes
                            (default), 2 = whenever any node qualifies */
  int32_t device;        /* 1 = run the affinity, Galerkin and renumbering
                            steps on the context's GPU (default; the result
                            is bit-identical to the host build); 2 = the
                            aggregation too (Sec. 3.1's aggregation by
                            affinity, done by parallel handshake matching:
                            every unassigned node picks its strongest
                            unassigned neighbour, mutual picks pair up,
                            leftovers join their strongest neighbour's
                            aggregate; deterministic, but other aggregates
                            than the host's greedy pass); 0 = host only.
                            Host-only contexts always build on the host. */
  int32_t order;         /* locality keys of the nested renumbering:
                            1 = Cuthill-McKee sweep, 2 = input node order,
                            3 = descending degree (hubs first, which keeps
                            the most gathered rows together); 0 = auto
                            (default): descending degree when the largest
                            degree exceeds 32 times the mean, else the
                            Cuthill-McKee sweep */
  int32_t max_complexity_pct; /* operator-complexity budget x 100: the
                            hierarchy takes no aggregation level that would
                            raise sum_l (nnz_l + n_l) / (nnz_a + n_a) above
                            it, with a the first aggregated level (1 behind
                            an elimination level, whose Schur complement the
                            solver iterates on, else 0), nor one whose
                            nnz + n exceeds 0.8 of the level it coarsens.
                            On expander-like complex networks the quotient
                            graphs keep almost every edge, so the budget
                            stops coarsening early; the deepest level then
                            has no exact solve when it has more than 4096
                            nodes, and every cycle ends there with one
                            Jacobi step.  0 = default (200, i.e. 2.0),
                            -1 = no budget and no ratio limit (coarsen to
                            coarsest_max) */
  int32_t elim_degree;   /* largest degree of an eliminated node, 1 to
                            CFC_ELIM_MAX_DEGREE; 0 = default (4).  The
                            independent set is picked by degree, lowest
                            first; removing a node of degree d joins its d
                            neighbours pairwise (conductance w_a w_b / D_ff),
                            which adds up to d (d - 3) matrix entries */
  int32_t nest;          /* how far the locality numbering nests aggregates:
                            1 = through every aggregation level down to
                            coarsest_max, also those the budget leaves out;
                            2 = through the levels the solver gets only;
                            0 = auto (default): 2 when rows of more than
                            256 entries hold a third or more of the
                            entries (hub-dominated graphs), else 1 */
} cfc_setup_params;

typedef struct {
  double tol;            /* per-column relative residual target (1e-6) */
  int32_t precision;     /* CFC_PREC_MIXED (default) or CFC_PREC_FP64.  In
                            CFC_PREC_MIXED with a one-Jacobi-step
                            preconditioner (depth one, or an elimination
                            level plus one step), z = M^-1 r is rounded to
                            bfloat16 where it is formed, which halves the
                            rows the operator product gathers; the FP64
                            residual still certifies tol.  The environment
                            variable CFC_BF16_Z=0 keeps z in FP32. */
  int32_t block;         /* right-hand sides per block W in {1,32,64,128,256,512};
                            0 = autotuned for the graph */
  int32_t max_refine;    /* FP64 refinement steps (20) */
  int32_t max_inner;     /* PCG iterations per refinement step (300) */
  double inner_tol;      /* PCG relative reduction per refinement step (at
                            least the one that reaches tol); 0 = autotuned
                            (default): 1e-4 (FP32 inner solves, two
                            refinement steps to 1e-6) or 1e-7 (straight to
                            the target) by timing both on sample columns.
                            Each column stops at its own reduction: the
                            larger of inner_tol and a fraction of what its
                            FP64 residual still lacks to reach tol */
  int32_t use_graph;     /* 1 = replay a captured HIP graph per PCG iteration */
  int32_t check_every;   /* PCG iterations between host convergence checks (1) */
  int32_t levels;        /* V-cycle depth: hierarchy levels used by the
                            preconditioner (1 = Jacobi on the fine level only,
                            all levels = exact coarsest solve); a truncated
                            cycle smooths once on its deepest level;
                            0 = autotuned for the graph */
  int32_t pad;
} cfc_solve_params;

typedef struct {
  int64_t columns;        /* right-hand sides solved */
  int64_t converged;      /* columns meeting tol */
  int64_t inner_iters;    /* PCG iterations summed over blocks and steps */
  int64_t refine_steps;   /* refinement steps summed over blocks */
  int64_t blocks;         /* RHS blocks processed */
  int32_t block_width;    /* W used */
  int32_t precision;
  int32_t levels_used;    /* V-cycle depth used */
  int32_t z_format;       /* storage of the preconditioned residual that the
                             operator product gathers: 0 = the inner
                             precision, 1 = bfloat16, 2 = FP8 (e4m3) with one
                             scale per row and column slice */
  double max_rel_residual;/* largest final ||b - L x|| / ||b|| (FP64) */
  double solve_ms;        /* device time of the solve phase (HIP events) */
  double model_bytes;     /* algorithmic HBM bytes of the solve phase */
  /* Level-0 kernel timing with HIP events on the launch stream (only when
   * the environment sets CFC_PROFILE=1): index 0 = the CG operator product
   * (k_spmm_pq), 1 = prolongation + post-smoothing (k_prolong_smooth),
   * 2 = CG update fused with pre-smoothing and restriction
   * (k_update_restrict) or, at depth one, with the Jacobi step
   * (k_update_jacobi). */
  double kernel_ms[3];
  double kernel_bytes[3];  /* algorithmic bytes of those launches */
  int64_t kernel_launches[3];
} cfc_solve_stats;

/* Level view for inspection (host arrays owned by the graph; valid until
 * the hierarchy is rebuilt or the graph destroyed). */
typedef struct {
  int64_t n, nnz, n_coarse;
  const int32_t* row_ptr;   /* [n+1] */
  const int32_t* col;       /* [nnz] off-diagonal columns, both directions */
  const double* w;          /* [nnz] conductances */
  const double* deg;        /* [n] weighted degrees D_ii */
  const int32_t* agg;       /* [n] aggregate (next-level node) of each row;
                               NULL on the coarsest level */
  const int32_t* agg_ptr;   /* [n_coarse+1] aggregate row ranges (contiguous) */
  const int32_t* perm;      /* level 0 only: graph node id -> row */
  const double* coarse_pinv;/* coarsest level only: dense L_c^+ [n*n] */
  /* Elimination level (n_coarse < n, agg = NULL): rows [0, n_coarse) are
   * kept and are rows [0, n_coarse) of the next level, whose Laplacian is
   * the Schur complement; rows [n_coarse, n) are eliminated, each with at
   * most CFC_ELIM_MAX_DEGREE kept neighbours
   * elim_nb[CFC_ELIM_MAX_DEGREE (r - n_coarse) + i], ascending, then -1. */
  int32_t elimination;      /* 1 on an elimination level, else 0 */
  int32_t pad;
  const int32_t* elim_nb;
} cfc_level_view;

/* ---- context ---------------------------------------------------------------- */

/* Create a context on a device (or host-only with device = -1). */
int cfc_ctx_create(const cfc_ctx_opts* opts, cfc_ctx** out);
void cfc_ctx_destroy(cfc_ctx* ctx);
/* Message for the last failing call on this thread ("" if none). */
const char* cfc_last_error(void);
/* Library version string. */
const char* cfc_version(void);
/* Bandwidth probe, not part of the method: copy `bytes` from src to dst
 * (both device memory of the context's GPU) with the library's own
 * streaming kernel (16-byte non-temporal loads and stores per lane) on the
 * context's stream, and wait for it.  It is the achievable-bandwidth
 * reference of the roofline reports and the calibration of the HBM traffic
 * counters.  CFC_E_INVALID for NULL pointers or a host-only context. */
int cfc_device_copy(cfc_ctx* ctx, void* dst, const void* src, size_t bytes);

/* ---- graph ---------------------------------------------------------------- */

/* Load an undirected weighted graph (Sec. 2).  u, v: int64[m] endpoints in
 * [0, n) (host memory); w: float64[m] conductances > 0 and finite, or NULL
 * for unit weights.  Self-loops are dropped (Sec. 6.3 ignores them);
 * repeated edges are merged by summing conductances (parallel resistors)
 * unless CFC_REJECT_PARALLEL.  A disconnected graph is CFC_E_DISCONNECTED
 * unless CFC_LCC_ONLY, which keeps the largest connected component and
 * relabels its nodes 0.. in increasing input id (Sec. 2 handles components
 * separately; Sec. 6.3 keeps the LCC); cfc_graph_node_map gives the input id
 * of each kept node. */
int cfc_graph_load(cfc_ctx* ctx, int64_t n, int64_t m, const int64_t* u,
                   const int64_t* v, const double* w, uint32_t flags,
                   cfc_graph** out);
int cfc_graph_get_info(const cfc_graph* g, cfc_graph_info* out);
/* orig[i] = input id of graph node i (host int64[n]). */
int cfc_graph_node_map(const cfc_graph* g, int64_t* orig);
void cfc_graph_destroy(cfc_graph* g);

/* Build the aggregation multigrid hierarchy used by every solve (the
 * solver's setup phase; the paper's solver coarsens by aggregating nodes by
 * an affinity measure, Sec. 3.1).  The affinity, Galerkin and renumbering
 * steps run on the GPU unless p->device is 0 or the context is host-only;
 * the hierarchy is then uploaded for the solves.  p = NULL selects the
 * defaults listed above. */
int cfc_hierarchy_build(cfc_graph* g, const cfc_setup_params* p);
/* Inspect level `level` of the host hierarchy. */
int cfc_hierarchy_level(const cfc_graph* g, int32_t level, cfc_level_view* out);

/* ---- solves --------------------------------------------------------------- */

/* Solve L X = B (Eq. 1).  B, X: float64, column-major n x nrhs (column j at
 * B + j*n), host or device (a host buffer costs one copy of each column
 * block over PCIe each way).  Each column must be finite and sum to zero
 * within 1e-12 * ||b||_1, else CFC_E_INVALID; columns are taken in blocks of
 * the solve width, and the check of a block runs just before its solve, so
 * on that error the columns of earlier blocks of X are already solved and
 * the rest are untouched.  X is returned mean-zero (= L^+ B).  Returns
 * CFC_E_NOT_CONVERGED if any column missed p->tol (X still holds the last
 * iterate).  col_status: int32[nrhs] or NULL.  p, st may be NULL. */
int cfc_solve(cfc_graph* g, int64_t nrhs, const double* B, double* X,
              const cfc_solve_params* p, cfc_solve_stats* st,
              int32_t* col_status);

/* Effective resistances d_ER(s_j, t_j) = p(s_j) - p(t_j) with
 * L p = e_{s_j} - e_{t_j} (Sec. 4).  s, t: int64[npairs], r: float64[npairs],
 * all host.  s_j = t_j gives 0. */
int cfc_resistance(cfc_graph* g, int64_t npairs, const int64_t* s,
                   const int64_t* t, double* r, const cfc_solve_params* p,
                   cfc_solve_stats* st);

/* Exact electrical farness and closeness c_ER (Eq. 3) of q nodes by their
 * n-1 solves each (Sec. 4).  nodes: int64[q]; far, clo: float64[q]; host. */
int cfc_farness_exact(cfc_graph* g, int64_t q, const int64_t* nodes,
                      double* far, double* clo, const cfc_solve_params* p,
                      cfc_solve_stats* st);

/* Sampling estimator (Sec. 5.1): for each query node v a uniform k-subset S
 * of all nodes (v may be drawn; it contributes 0 and needs no solve), drawn
 * by cfc_sampling_pivots(seed, v, ...); far = (n/k) sum_S d_ER(v, s), the
 * unbiased estimate of Prop. 1, and clo = (k/n)(n-1)/sum_S d_ER(v, s).
 * k is clamped to n.  Host arrays. */
int cfc_farness_sampling(cfc_graph* g, int64_t q, const int64_t* nodes,
                         int64_t k, uint64_t seed, double* far, double* clo,
                         const cfc_solve_params* p, cfc_solve_stats* st);

/* Projection estimator, sketch phase (Sec. 5.2, Algorithm 1): with
 * Q in {+-1/sqrt(k)}^(k x m) (row i's sign on edge {lo<hi} is bit i mod 64
 * of cfc_jl_sign_word(seed, i/64, lo, hi), set bit = -1), B oriented
 * B(e, lo) = +1, solve L z_i = (Q W^(1/2) B)_i for i < k and keep, per node,
 * what the farness of every node needs (||Z_.v||^2, Z_.v . sum_w Z_.w and
 * ||Z||_F^2) resident on the device. */
int cfc_jl_sketch(cfc_graph* g, int64_t k, uint64_t seed,
                  const cfc_solve_params* p, cfc_solve_stats* st);
/* Projection estimate of farness sum_w ||Z_.v - Z_.w||^2 and closeness
 * (n-1)/farness (Sec. 5.2) of q nodes from the resident sketch
 * (CFC_E_STATE if none).  nodes = NULL with q = n asks for every node in
 * id order (O(n) from the sketch: the all-node closeness that Sec. 5.2's
 * sketch makes cheap).  Host arrays. */
int cfc_farness_jl(cfc_graph* g, int64_t q, const int64_t* nodes,
                   double* far, double* clo);

/* Sampling with ONE pivot set S for all q query nodes (Sec. 5.1 read
 * literally: a single uniform sample of k nodes, drawn by
 * cfc_shared_pivots(seed, n, k, ...)); far = (n/k) sum_{s in S} d_ER(v, s)
 * and clo = (k/n)(n-1)/sum as in cfc_farness_sampling.  With r the smallest
 * pivot and y_a = L^+ (e_a - e_r), d_ER(v, s) = y_v[v] - y_v[s] - y_s[v] +
 * y_s[s], so it takes |S u Q| - 1 solves instead of k q.  Host arrays;
 * CFC_E_NOT_CONVERGED if a solve misses the tolerance. */
int cfc_farness_sampling_shared(cfc_graph* g, int64_t q, const int64_t* nodes,
                                int64_t k, uint64_t seed, double* far, double* clo,
                                const cfc_solve_params* p, cfc_solve_stats* st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * projection farness and closeness as cfc_farness_jl, computed without any
 * allocation.  The node ids and both outputs are staged in a fixed device
 * array of 6 MiB per GPU (set up when a context is created on that GPU and
 * held until the process ends), so q <= 262144 nodes per call (CFC_E_INVALID
 * above that).  nodes: host or device int64[q], or NULL with q = n for every
 * node; far, clo (clo may be NULL): host or device double[q].  Calls on one
 * GPU share its staging array: calls that overlap on one GPU race.  Same
 * errors as cfc_farness_jl; node ids are range-checked on the device, and
 * after CFC_E_INVALID for a bad id the outputs hold NaN where ids were bad. */
int cfc_farness_jl_static(cfc_graph* g, int64_t q, const int64_t* nodes, double* far, double* clo);

/* ---- other Laplacian-system centralities (Sec. 3.2) ------------------------ */

/* Spanning-edge centrality of ne edges {u_i, v_i} of the loaded graph: the
 * weighted share of spanning trees that contain the edge, equal to
 * w_e d_ER(u_i, v_i) (Kirchhoff); one solve per edge.  w_e is the merged
 * conductance.  CFC_E_INVALID if a pair is not an edge.  Host arrays. */
int cfc_spanning_edge(cfc_graph* g, int64_t ne, const int64_t* u, const int64_t* v,
                      double* c, const cfc_solve_params* p, cfc_solve_stats* st);
/* Projection estimate w_e ||Z_.u - Z_.v||^2 with Z the sketch of
 * cfc_jl_sketch(k, seed) (same signs, Sec. 5.2); k solves for any number of
 * edges.  Host arrays. */
int cfc_spanning_edge_jl(cfc_graph* g, int64_t ne, const int64_t* u, const int64_t* v,
                         int64_t k, uint64_t seed, double* c,
                         const cfc_solve_params* p, cfc_solve_stats* st);

/* Current-flow throughput (the electrical view of Sec. 2): for each pair a
 * unit current enters at s_j and leaves at t_j (L p = e_s - e_t, Eq. 1), and
 * tau[v] = sum over the pairs with v not in {s_j, t_j} of
 * 1/2 sum_{x in N(v)} w_vx |p(v) - p(x)|.  tau is host double[n], written.
 * Pairs with s_j = t_j carry no current. */
int cfc_current_throughput(cfc_graph* g, int64_t npairs, const int64_t* s,
                           const int64_t* t, double* tau,
                           const cfc_solve_params* p, cfc_solve_stats* st);
/* Current-flow betweenness (Brandes and Fleischer; named in Sec. 3.2) of every
 * node: the mean throughput over the unordered pairs {s, t} of V \ {v},
 * c_CB(v) = sum tau_st(v) / C(n-1, 2).  cfc_cfb_exact solves all C(n, 2)
 * pairs (small graphs); cfc_cfb_sampled draws `count` ordered pairs with
 * cfc_random_pairs(seed, n, count, ...) and returns the unbiased estimate
 * (n / (n-2)) * mean_i tau_i(v).  cb is host double[n]; n >= 3. */
int cfc_cfb_exact(cfc_graph* g, double* cb, const cfc_solve_params* p, cfc_solve_stats* st);
int cfc_cfb_sampled(cfc_graph* g, int64_t count, uint64_t seed, double* cb,
                    const cfc_solve_params* p, cfc_solve_stats* st);

/* ---- the library's random draws (host, no device needed) ------------------ */

/* Pivot set of the Sampling estimator for query node `node`: sorted
 * int64[min(k,n)] (Floyd's subset algorithm over Lemire-bounded integers
 * from SplitMix64 words H(seed, 0x5350, node, c), c = 0, 1, ...). */
int cfc_sampling_pivots(uint64_t seed, int64_t node, int64_t n, int64_t k,
                        int64_t* out);
/* 64 projection sign bits H(seed, 0x4A4C, word, lo*2^32 + hi). */
uint64_t cfc_jl_sign_word(uint64_t seed, uint64_t word, int64_t lo, int64_t hi);
/* The shared pivot set: sorted int64[min(k,n)], Floyd's algorithm over
 * words H(seed, 0x5348, 0, c). */
int cfc_shared_pivots(uint64_t seed, int64_t n, int64_t k, int64_t* out);
/* `count` source/sink pairs, uniform over ordered pairs with s != t: pair i
 * draws s = bounded(n), b = bounded(n-1) from words H(seed, 0x4346, i, c)
 * and sets t = b + (b >= s).  n >= 2. */
int cfc_random_pairs(uint64_t seed, int64_t n, int64_t count, int64_t* s, int64_t* t);

/* ---- serving ------------------------------------------------------------- */

typedef struct {
  int32_t slots;           /* RHS columns in flight per graph (256) */
  int32_t max_queue;       /* pending queries before CFC_E_BUSY (4096) */
  int32_t jl_k;            /* sketch size built by cfc_server_add_graph (256;
                              0 = no sketch) */
  int32_t sampling_k;      /* default pivots per node (200) */
  uint64_t seed;           /* seed for sketches and pivots (1) */
  double tol;              /* solve tolerance (1e-6) */
  uint64_t hbm_budget;     /* device bytes for in-flight work (0 = no limit) */
} cfc_server_opts;

#define CFC_QUERY_SAMPLING 0
#define CFC_QUERY_JL       1

typedef struct {
  int32_t graph;           /* id from cfc_server_add_graph */
  int32_t kind;            /* CFC_QUERY_SAMPLING or CFC_QUERY_JL */
  int32_t nnodes;          /* 1..1024 */
  int32_t k;               /* pivots per node (0 = server default) */
  const int64_t* nodes;    /* host int64[nnodes], copied at submit */
  uint64_t seed;           /* 0 = server seed */
} cfc_query;

typedef struct {
  int32_t status;          /* CFC_OK or an error for this query */
  int32_t nnodes;
  double* far;             /* caller buffers of nnodes float64, or NULL */
  double* clo;
  double latency_ms;       /* arrival to completion */
} cfc_result;

typedef struct {
  int64_t submitted, completed, queued, in_flight;
  double p50_ms, p99_ms, mean_ms;
  double queries_per_s;    /* completed / wall time since the first submit */
  uint64_t device_bytes;   /* device memory held by the server */
} cfc_server_stats;

int cfc_server_create(cfc_ctx* ctx, const cfc_server_opts* opts, cfc_server** out);
/* Register a graph whose hierarchy is built; builds its sketch if jl_k > 0.
 * From then until cfc_server_destroy the server's worker thread owns the
 * graph's device state: every direct call on the graph (cfc_solve, the
 * estimators, cfc_hierarchy_build, ...) returns CFC_E_STATE, and a graph can
 * be registered with one server at a time (CFC_E_STATE otherwise).  The
 * graph must outlive the server. */
int cfc_server_add_graph(cfc_server* s, cfc_graph* g, int32_t* gid);
/* Queue a query; returns at once with a ticket (CFC_E_BUSY if full). */
int cfc_server_submit(cfc_server* s, const cfc_query* q, uint64_t* ticket);
/* CFC_E_STATE while pending; on completion fills r (copying far/clo into
 * r->far/r->clo if non-NULL) and forgets the ticket. */
int cfc_server_poll(cfc_server* s, uint64_t ticket, cfc_result* r);
/* Block until the ticket completes (timeout_ms < 0: no limit). */
int cfc_server_wait(cfc_server* s, uint64_t ticket, double timeout_ms, cfc_result* r);
int cfc_server_get_stats(cfc_server* s, cfc_server_stats* st);
void cfc_server_destroy(cfc_server* s);

#ifdef __cplusplus
}
#endif
#endif /* CFC_H */
