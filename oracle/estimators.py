"""The paper's two estimators of electrical farness / current-flow closeness.

Sampling (Sec. 5.1): for query node v draw a pivot set S of k nodes uniformly
at random, sum the effective resistances d_ER(v, s) over S and scale by n/k
(the estimator Y in the proof of Prop. 1, whose expectation is the farness
sum_w d_ER(v, w)); closeness is (k/n)(n-1)/sum_S d_ER(v, s) as in Sec. 5.1.
Reading of the sample space: a uniform k-subset of all of V drawn without
replacement, v itself allowed (it contributes d_ER(v, v) = 0 and needs no
solve), exactly the k-combinations V_k of the proof.

Projection (Sec. 5.2, Algorithm 1): Q is k x m with entries +-1/sqrt(k)
(Rademacher); Y = Q W^(1/2) B with B the m x n incidence matrix oriented
B(e, lo) = +1, B(e, hi) = -1; system i solves L z_i = (row i of Y)^T; then
d~(u, v) = ||Z_.u - Z_.v||^2 and the farness of v sums d~(v, w) over w != v.
"""
from __future__ import annotations

import numpy as np

from . import rng as _rng
from . import resistance as _res


def sampling(L, g, nodes, k, seed, solver="cg", tol=1e-12, Lp=None):
    """Sampling estimate for each query node.

    Returns (farness_est, closeness_est, per_node_pivots, per_node_d) where
    per_node_d[i][j] is d_ER(v_i, s_j) for the j-th pivot (0 when s_j = v_i).
    ``solver`` is "cg" (sparse L) or "dense" (``Lp`` = pseudoinverse given).
    """
    n = g.n
    far = []
    clo = []
    piv_all = []
    d_all = []
    for v in np.atleast_1d(nodes):
        v = int(v)
        S = _rng.pivots(seed, v, n, k)
        kk = len(S)
        others = np.array([s for s in S if s != v], np.int64)
        if others.size:
            if solver == "dense":
                d_o = _res.resistance_from_inverse(Lp, np.full(others.shape, v), others)
            else:
                d_o = _res.resistance_cg(L, np.full(others.shape, v), others, tol)
        else:
            d_o = np.zeros(0)
        d = np.zeros(kk)
        d[[i for i, s in enumerate(S) if s != v]] = d_o
        tot = float(d.sum())
        far.append(n / kk * tot)
        clo.append((kk / n) * (n - 1) / tot if tot > 0 else np.inf)
        piv_all.append(np.array(S, np.int64))
        d_all.append(d)
    return np.array(far), np.array(clo), piv_all, d_all


def sampling_shared(L, g, nodes, k, seed, solver="cg", tol=1e-12, Lp=None):
    """Sampling with one pivot set S for all query nodes (Sec. 5.1 read
    literally: a single uniform sample of k nodes, drawn by
    ``rng.shared_pivots``).  The estimate is the same (n/k) sum_S d_ER(v, s)
    as in :func:`sampling`, each d_ER by its own solve of L p = e_v - e_s.

    Returns (farness_est, closeness_est, S)."""
    n = g.n
    S = _rng.shared_pivots(seed, n, k)
    kk = len(S)
    far = []
    clo = []
    for v in np.atleast_1d(nodes):
        v = int(v)
        others = np.array([s for s in S if s != v], np.int64)
        if others.size == 0:
            tot = 0.0
        elif solver == "dense":
            tot = float(_res.resistance_from_inverse(Lp, np.full(others.shape, v), others).sum())
        else:
            tot = float(_res.resistance_cg(L, np.full(others.shape, v), others, tol).sum())
        far.append(n / kk * tot)
        clo.append((kk / n) * (n - 1) / tot if tot > 0 else np.inf)
    return np.array(far), np.array(clo), np.array(S, np.int64)


def projection_rhs(g, k, seed, Q=None):
    """Y^T (n x k): column i is (Q W^(1/2) B)_i, row i of Y (Algorithm 1's
    multiplication step).  ``Q`` overrides the random matrix (k x m), e.g. the
    identity for the exactness check."""
    u, v, w = g.u, g.v, g.weights()
    m = u.shape[0]
    if Q is None:
        Q = _rng.jl_signs(seed, k, u, v).astype(np.float64) / np.sqrt(k)
    Y = np.zeros((g.n, Q.shape[0]))
    sw = np.sqrt(w)
    for e in range(m):
        Y[u[e]] += Q[:, e] * sw[e]
        Y[v[e]] -= Q[:, e] * sw[e]
    return Y


def projection(L, g, nodes, k, seed, solver="cg", tol=1e-12, Lp=None, Q=None):
    """Projection estimate (Algorithm 1) for the query nodes.

    Returns (farness_est, closeness_est, Z) with Z the n x k matrix whose
    column i is z_i (mean-zero)."""
    Y = projection_rhs(g, k, seed, Q)
    if solver == "dense":
        Z = Lp @ Y
        Z -= Z.mean(axis=0)
    else:
        Z, _ = _res.cg(L, Y, tol)
    n = g.n
    far = []
    for v in np.atleast_1d(nodes):
        diff = Z - Z[int(v)]
        d = np.einsum("ij,ij->i", diff, diff)  # d~(v, w) for every w
        far.append(float(d.sum() - d[int(v)]))
    far = np.array(far)
    return far, (n - 1) / far, Z
