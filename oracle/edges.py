"""Spanning-edge centrality (Sec. 3.2, Laplacian systems in network analysis).

The paper names spanning-edge centrality (Mavroforakis et al., 2015) as one
of the measures computed from Laplacian systems.  Its definition: the share
of the spanning trees of G that contain edge e, each tree counted with the
product of its edge weights.  By Kirchhoff's theorem this share equals
w_e * d_ER(u, v) for e = {u, v}, with d_ER the effective resistance of
Sec. 4.  Two routes are given here:

* exact: w_e * d_ER(u, v) from the pseudoinverse (dense) or one CG solve of
  L p = e_u - e_v per edge (Sec. 4);
* projection: d_ER(u, v) replaced by ||Z_.u - Z_.v||^2 with Z the
  Johnson-Lindenstrauss sketch of Sec. 5.2 (the same right-hand sides and
  random signs as the farness estimator, see ``estimators.projection``).

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import estimators as _est
from . import resistance as _res


def edge_weights(g, u, v):
    """Conductance of each listed edge {u_i, v_i} of the edge list g."""
    u = np.atleast_1d(np.asarray(u, np.int64))
    v = np.atleast_1d(np.asarray(v, np.int64))
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = g.u * np.int64(g.n) + g.v
    want = lo * np.int64(g.n) + hi
    pos = np.searchsorted(key, want)
    if np.any(pos >= key.shape[0]) or np.any(key[np.minimum(pos, key.shape[0] - 1)] != want):
        raise ValueError("not an edge of the graph")
    return g.weights()[pos]


def spanning_edge(L, g, u, v, solver="cg", tol=1e-12, Lp=None):
    """Exact spanning-edge centrality w_e * d_ER(u, v) of the listed edges."""
    w = edge_weights(g, u, v)
    u = np.atleast_1d(u)
    v = np.atleast_1d(v)
    if solver == "dense":
        r = _res.resistance_from_inverse(Lp, u, v)
    else:
        r = _res.resistance_cg(L, u, v, tol)
    return w * r


def spanning_edge_jl(L, g, u, v, k, seed, solver="cg", tol=1e-12, Lp=None, Q=None):
    """Projection estimate w_e * ||Z_.u - Z_.v||^2 (Sec. 5.2's sketch Z)."""
    w = edge_weights(g, u, v)
    _, _, Z = _est.projection(L, g, [0], k, seed, solver=solver, tol=tol, Lp=Lp, Q=Q)
    d = Z[np.atleast_1d(u)] - Z[np.atleast_1d(v)]
    return w * np.einsum("ij,ij->i", d, d)


def spanning_tree_share_bruteforce(g):
    """Weighted share of spanning trees containing each edge, by listing every
    (n-1)-subset of the edges and keeping the acyclic ones (tiny graphs)."""
    from itertools import combinations

    n, m = g.n, g.m
    w = g.weights()
    tot = 0.0
    per = np.zeros(m)
    for sub in combinations(range(m), n - 1):
        parent = list(range(n))

        def find(a):
            while parent[a] != a:
                parent[a] = parent[parent[a]]
                a = parent[a]
            return a

        ok = True
        for e in sub:
            a, b = find(int(g.u[e])), find(int(g.v[e]))
            if a == b:
                ok = False
                break
            parent[a] = b
        if not ok:
            continue
        wt = float(np.prod(w[list(sub)]))
        tot += wt
        per[list(sub)] += wt
    return per / tot
