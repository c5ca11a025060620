"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws graphs and query-node subsets only.  It holds none of the
method's arithmetic (no Laplacian, no solve, no estimator), so both the GPU
path and the CPU oracle may consume what it produces.
"""
from .graphs import (EdgeList, grid, road_grid, barabasi_albert, rmat, lcc,
                     random_connected, path_graph, cycle_graph, complete_graph,
                     complete_bipartite, star_graph, query_nodes, cached)

__all__ = ["EdgeList", "grid", "road_grid", "barabasi_albert", "rmat", "lcc",
           "random_connected", "path_graph", "cycle_graph", "complete_graph",
           "complete_bipartite", "star_graph", "query_nodes", "cached"]
