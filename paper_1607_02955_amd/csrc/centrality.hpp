// Shared-pivot Sampling, spanning-edge centrality and current-flow
// throughput on top of the batched solve (centrality.cpp).
#pragma once
#include <functional>
#include <vector>

#include "internal.hpp"

namespace cfc {

// Uniform k-subset of {0..n-1} (sorted) by Floyd's algorithm over
// Lemire-bounded integers from the words H(seed, tag, a, c), c = 0, 1, ...
void floyd_subset(uint64_t seed, uint64_t tag, uint64_t a, int64_t n, int64_t k,
                  std::vector<int64_t>& out);
// Pair i: s = bounded(n), b = bounded(n - 1) from H(seed, 0x4346, i, c),
// t = b + (b >= s): uniform over ordered pairs with s != t.
void random_pairs(uint64_t seed, int64_t n, int64_t count, int64_t* s, int64_t* t);
// Conductance of edge {u, v} of the loaded graph (CFC_E_INVALID if absent);
// `hint` = index of the edge in the canonical list if the caller follows it.
double edge_weight(const Graph& g, int64_t u, int64_t v, int64_t hint = -1);

void shared_sampling(Graph& g, int64_t q, const int64_t* nodes, int64_t k, uint64_t seed, double* far,
                     double* clo, const cfc_solve_params& p, cfc_solve_stats* st);
void spanning_edge(Graph& g, int64_t ne, const int64_t* u, const int64_t* v, double* c,
                   const cfc_solve_params& p, cfc_solve_stats* st);
void spanning_edge_jl(Graph& g, int64_t ne, const int64_t* u, const int64_t* v, int64_t k,
                      uint64_t seed, double* c, const cfc_solve_params& p, cfc_solve_stats* st);

// pair j -> (s, t) in graph ids
using PairSource = std::function<void(int64_t j, int64_t& s, int64_t& t)>;
// tau[v] (graph ids, host double[n]) = sum over the pairs of v's throughput
void current_throughput(Graph& g, int64_t npairs, const PairSource& pairs, double* tau,
                        const cfc_solve_params& p, cfc_solve_stats* st);

}  // namespace cfc
