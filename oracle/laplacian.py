"""The graph Laplacian L = D - A (Sec. 2, "Graph basics").

A is the weighted adjacency matrix of the undirected graph, D the diagonal of
weighted degrees D_ii = sum_j w_ij.  Edge weights are conductances
(Sec. 2, "Graphs as electrical networks").  Parallel edges add up.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def adjacency(n, u, v, w=None):
    w = np.ones(len(u)) if w is None else np.asarray(w, np.float64)
    a = sp.coo_matrix((w, (u, v)), shape=(n, n))
    return (a + a.T).tocsr()


def laplacian_sparse(n, u, v, w=None) -> sp.csr_matrix:
    a = adjacency(n, u, v, w)
    d = np.asarray(a.sum(axis=1)).ravel()
    return (sp.diags(d) - a).tocsr()


def laplacian_dense(n, u, v, w=None) -> np.ndarray:
    return laplacian_sparse(n, u, v, w).toarray()


def of(g, dense=False):
    """Laplacian of a synth.EdgeList-like object (attributes n, u, v, w)."""
    return (laplacian_dense if dense else laplacian_sparse)(g.n, g.u, g.v, g.w)
