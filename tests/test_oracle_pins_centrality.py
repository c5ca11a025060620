"""Pins of the oracle's shared-pivot Sampling, spanning-edge centrality and
current-flow betweenness against closed forms, brute force and statistics.

As for the other oracle pins, each value is fixed by something other than the
oracle's own formula: combinatorial counts on trees and cycles, spanning-tree
enumeration, Foster's theorem, exactness at k = n or Q = I, unbiasedness.
"""
import math

import numpy as np

import synth
from oracle import betweenness as CB
from oracle import edges as SE
from oracle import estimators as E
from oracle import laplacian as LAP
from oracle import resistance as R
from oracle import rng as RNG


def _lp(g):
    return R.pinv(LAP.of(g, dense=True))


def _edgelist(n, a, b, w=None):
    a = np.asarray(a, np.int64)
    b = np.asarray(b, np.int64)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    o = np.lexsort((hi, lo))
    return synth.EdgeList(n, lo[o], hi[o], None if w is None else np.asarray(w, np.float64)[o])


# ---- shared-pivot Sampling ----------------------------------------------------

def test_shared_sampling_with_k_equal_n_is_exact():
    g = synth.random_connected(35, 90, seed=2)
    Lp = _lp(g)
    nodes = [0, 7, 34]
    f, c, S = E.sampling_shared(LAP.of(g), g, nodes, g.n, seed=9)
    assert list(S) == list(range(g.n))
    np.testing.assert_allclose(f, R.farness_dense(Lp, nodes), rtol=1e-10)
    np.testing.assert_allclose(c, (g.n - 1) / R.farness_dense(Lp, nodes), rtol=1e-10)


def test_shared_pivots_are_one_uniform_subset():
    n, k, trials = 12, 4, 6000
    counts = np.zeros(n)
    for seed in range(trials):
        S = RNG.shared_pivots(seed, n, k)
        assert len(S) == k and len(set(S)) == k and S == sorted(S)
        counts[S] += 1
    want = trials * k / n
    chi2 = float(((counts - want) ** 2 / want).sum())
    assert chi2 < 35.0  # 11 degrees of freedom; p ~ 3e-4
    assert RNG.shared_pivots(3, 50, 8) != RNG.pivots(3, 0, 50, 8)


def test_shared_sampling_is_unbiased_for_farness():
    g = synth.random_connected(30, 70, seed=5)
    Lp = _lp(g)
    v, k = 3, 6
    exact = R.farness_dense(Lp, v)[0]
    est = np.array([E.sampling_shared(None, g, [v], k, s, solver="dense", Lp=Lp)[0][0]
                    for s in range(3000)])
    assert abs(est.mean() - exact) < 5 * est.std() / math.sqrt(len(est))


# ---- spanning-edge centrality --------------------------------------------------

def test_spanning_edge_is_weighted_tree_share():
    g = synth.random_connected(6, 10, seed=13)
    want = SE.spanning_tree_share_bruteforce(g)
    got = SE.spanning_edge(None, g, g.u, g.v, solver="dense", Lp=_lp(g))
    np.testing.assert_allclose(got, want, rtol=1e-11)
    got_cg = SE.spanning_edge(LAP.of(g), g, g.u, g.v)
    np.testing.assert_allclose(got_cg, want, rtol=1e-9)


def test_spanning_edge_closed_forms():
    # Foster: the shares sum to n - 1 (every spanning tree has n - 1 edges)
    g = synth.random_connected(40, 120, seed=4)
    assert abs(SE.spanning_edge(None, g, g.u, g.v, "dense", Lp=_lp(g)).sum() - 39) < 1e-9
    # a tree: every edge lies in its only spanning tree
    rng = np.random.default_rng(2)
    n = 20
    par = [int(rng.integers(0, i)) for i in range(1, n)]
    t = _edgelist(n, par, np.arange(1, n), rng.uniform(0.5, 3, n - 1))
    np.testing.assert_allclose(SE.spanning_edge(None, t, t.u, t.v, "dense", Lp=_lp(t)), 1, atol=1e-11)
    # cycle: n spanning trees, each edge is missing from exactly one
    c = synth.cycle_graph(9)
    np.testing.assert_allclose(SE.spanning_edge(None, c, c.u, c.v, "dense", Lp=_lp(c)), 8 / 9, atol=1e-12)
    # complete graph: by symmetry (n - 1) / C(n, 2) = 2 / n
    k = synth.complete_graph(7)
    np.testing.assert_allclose(SE.spanning_edge(None, k, k.u, k.v, "dense", Lp=_lp(k)), 2 / 7, atol=1e-12)


def test_spanning_edge_projection_identity_q_exact_and_unbiased():
    g = synth.random_connected(20, 45, seed=6)
    Lp = _lp(g)
    exact = SE.spanning_edge(None, g, g.u, g.v, "dense", Lp=Lp)
    idq = SE.spanning_edge_jl(None, g, g.u, g.v, g.m, 0, "dense", Lp=Lp, Q=np.eye(g.m))
    np.testing.assert_allclose(idq, exact, rtol=1e-10)
    e = 5
    est = np.array([SE.spanning_edge_jl(None, g, g.u[e], g.v[e], 16, s, "dense", Lp=Lp)[0]
                    for s in range(600)])
    assert abs(est.mean() - exact[e]) < 5 * est.std() / math.sqrt(len(est))
    try:
        SE.edge_weights(g, [0], [0])
        raise AssertionError("a non-edge was accepted")
    except ValueError:
        pass


# ---- current-flow betweenness -------------------------------------------------

def test_cfb_path_star_complete():
    n = 9
    p = synth.path_graph(n)
    want = np.array([i * (n - 1 - i) for i in range(n)]) / ((n - 1) * (n - 2) / 2)
    np.testing.assert_allclose(CB.cfb_exact(p, _lp(p)), want, atol=1e-12)
    s = synth.star_graph(8)  # centre 0
    cs = CB.cfb_exact(s, _lp(s))
    assert abs(cs[0] - 1) < 1e-12 and np.all(np.abs(cs[1:]) < 1e-12)
    k = synth.complete_graph(8)
    np.testing.assert_allclose(CB.cfb_exact(k, _lp(k)), 1 / 8, atol=1e-12)


def test_cfb_weighted_tree_counts_paths():
    """In a tree all current follows the unique path, whatever the weights:
    c_CB(v) = #{pairs whose path passes through v} / C(n-1, 2)."""
    rng = np.random.default_rng(11)
    n = 16
    par = [-1] + [int(rng.integers(0, i)) for i in range(1, n)]
    t = _edgelist(n, par[1:], np.arange(1, n), rng.uniform(0.2, 5, n - 1))

    def path(a, b):
        up = []
        x = a
        while x != -1:
            up.append(x)
            x = par[x]
        seen = {x: i for i, x in enumerate(up)}
        down = []
        x = b
        while x not in seen:
            down.append(x)
            x = par[x]
        return up[:seen[x] + 1] + down[::-1]

    cnt = np.zeros(n)
    for a in range(n):
        for b in range(a + 1, n):
            for x in path(a, b)[1:-1]:
                cnt[x] += 1
    np.testing.assert_allclose(CB.cfb_exact(t, _lp(t)), cnt / ((n - 1) * (n - 2) / 2), atol=1e-11)


def test_cfb_weighted_cycle_current_divider():
    """On a cycle the unit current splits over the two arcs in inverse
    proportion to their series resistances; nodes inside an arc carry its share."""
    n = 10
    rng = np.random.default_rng(5)
    w = rng.uniform(0.5, 4, n)  # edge i joins i and i+1 (mod n)
    c = _edgelist(n, np.arange(n), (np.arange(n) + 1) % n, w)
    res = 1 / w
    want = np.zeros(n)
    for a in range(n):
        for b in range(a + 1, n):
            ra = res[a:b].sum()                     # arc a -> a+1 -> ... -> b
            rb = res.sum() - ra
            for x in range(a + 1, b):
                want[x] += rb / (ra + rb)
            for x in list(range(b + 1, n)) + list(range(0, a)):
                want[x] += ra / (ra + rb)
    want /= (n - 1) * (n - 2) / 2
    np.testing.assert_allclose(CB.cfb_exact(c, _lp(c)), want, atol=1e-12)


def test_random_pairs_uniform_and_cfb_sampled_unbiased():
    n, trials = 5, 20000
    s, t = RNG.random_pairs(4, n, trials)
    assert np.all(s != t) and s.min() >= 0 and t.max() < n
    counts = np.zeros((n, n))
    np.add.at(counts, (s, t), 1)
    want = trials / (n * (n - 1))
    off = ~np.eye(n, dtype=bool)
    chi2 = float(((counts[off] - want) ** 2 / want).sum())
    assert chi2 < 50.0  # 19 degrees of freedom
    g = synth.random_connected(12, 24, seed=8)
    Lp = _lp(g)
    exact = CB.cfb_exact(g, Lp)
    est = np.array([CB.cfb_sampled(None, g, 4, sd, "dense", Lp=Lp) for sd in range(1500)])
    se = est.std(axis=0) / math.sqrt(est.shape[0])
    assert np.all(np.abs(est.mean(axis=0) - exact) < 5 * se + 1e-12)
    np.testing.assert_allclose(CB.cfb_sampled(LAP.of(g), g, 30, 2),
                               CB.cfb_sampled(None, g, 30, 2, "dense", Lp=Lp), rtol=1e-9, atol=1e-12)
