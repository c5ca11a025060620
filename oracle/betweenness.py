"""Current-flow betweenness (Sec. 3.2, last paragraph: Brandes and Fleischer).

The paper names current-flow betweenness next to current-flow closeness as
the two centralities of the electrical-network view.  Its definition, in the
electrical terms of Sec. 2:

* a unit current enters at s and leaves at t; the potentials solve
  L p = e_s - e_t (Eq. 1) and edge {u, x} carries the current
  I(u, x) = w_ux (p(u) - p(x));
* the throughput of a node v outside {s, t} is half the sum of |I| over its
  edges (every unit entering v also leaves it);
* the betweenness of v averages that throughput over the unordered pairs
  {s, t} of V \\ {v}: c_CB(v) = sum_{s<t, v not in {s,t}} tau_st(v) / C(n-1, 2).

Reading: the endpoints' own pairs are left out (Brandes and Fleischer give
them throughput 1, which adds the same constant 2 / (n - 2) to every node).

The sampled estimate draws ``count`` ordered pairs uniformly with s != t
(``rng.random_pairs``) and scales the mean throughput so that it is unbiased:
E[tau_st(v) 1(v not in {s,t})] = C(n-1, 2) c_CB(v) / C(n, 2), hence
c~(v) = (n / (n - 2)) * mean_i tau_{s_i t_i}(v) 1(v not in {s_i, t_i}).

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import rng as _rng
from . import resistance as _res


def throughput(g, P, s, t):
    """tau_{s_j t_j}(v) for every node v (rows) and pair j (columns), given the
    potentials P[:, j] of L p = e_{s_j} - e_{t_j}; zero at each pair's s and t."""
    s = np.atleast_1d(s)
    t = np.atleast_1d(t)
    w = g.weights()
    cur = np.abs(w[:, None] * (P[g.u] - P[g.v]))  # |I_e| per edge and pair
    tau = np.zeros((g.n, P.shape[1]))
    np.add.at(tau, g.u, cur)
    np.add.at(tau, g.v, cur)
    tau *= 0.5
    j = np.arange(s.shape[0])
    tau[s, j] = 0.0
    tau[t, j] = 0.0
    return tau


def potentials(L, g, s, t, solver="cg", tol=1e-12, Lp=None):
    B = _res.pair_rhs(g.n, s, t)
    if solver == "dense":
        return Lp @ B
    X, _ = _res.cg(L, B, tol)
    return X


def cfb_exact(g, Lp, block=256):
    """c_CB(v) for every node, by all C(n, 2) pairs (dense potentials)."""
    n = g.n
    iu, ju = np.triu_indices(n, 1)
    tot = np.zeros(n)
    for a in range(0, iu.shape[0], block):
        s, t = iu[a:a + block], ju[a:a + block]
        tot += throughput(g, potentials(None, g, s, t, "dense", Lp=Lp), s, t).sum(axis=1)
    return tot / ((n - 1) * (n - 2) / 2)


def cfb_sampled(L, g, count, seed, solver="cg", tol=1e-12, Lp=None, block=256):
    """Sampled estimate of c_CB(v) for every node from ``count`` random pairs."""
    n = g.n
    s, t = _rng.random_pairs(seed, n, count)
    tot = np.zeros(n)
    for a in range(0, count, block):
        ss, tt = s[a:a + block], t[a:a + block]
        tot += throughput(g, potentials(L, g, ss, tt, solver, tol, Lp), ss, tt).sum(axis=1)
    return (n / (n - 2)) * tot / count
