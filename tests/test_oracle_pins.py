"""Pins of the CPU oracle against closed forms, brute force and identities.

Each test fixes a value by something other than the oracle's own formula, so a
dropped term, a wrong sign or index, or a transposed operand in the oracle
fails at least one of them.
"""
import itertools
import math
import os

import numpy as np
import pytest

import synth
from oracle import estimators as E
from oracle import laplacian as LAP
from oracle import resistance as R
from oracle import rng as RNG

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dense_routes(g):
    L = LAP.of(g, dense=True)
    return L, R.pinv(L), R.grounded_inverse(L, g.n // 2)


# ---- closed forms ----------------------------------------------------------

@pytest.mark.parametrize("route", [1, 2])
def test_path_resistance_is_distance(route):
    n = 9
    g = synth.path_graph(n)
    M = dense_routes(g)[route]
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    np.testing.assert_allclose(R.resistance_from_inverse(M, u, v), np.abs(u - v), atol=1e-11)
    np.testing.assert_allclose(R.farness_dense(M, 0), n * (n - 1) / 2, rtol=1e-12)


def test_weighted_path_series_resistors():
    n = 7
    w = np.array([1.0, 2.0, 0.5, 4.0, 3.0, 1.5])
    g = synth.path_graph(n, w)
    _, Lp, G = dense_routes(g)
    for a in range(n):
        for b in range(n):
            lo, hi = min(a, b), max(a, b)
            want = float(np.sum(1.0 / w[lo:hi]))
            assert abs(R.resistance_from_inverse(Lp, a, b) - want) < 1e-11
            assert abs(R.resistance_from_inverse(G, a, b) - want) < 1e-11


def test_cycle():
    n = 11
    g = synth.cycle_graph(n)
    _, Lp, G = dense_routes(g)
    for d in range(n):
        want = d * (n - d) / n
        assert abs(R.resistance_from_inverse(Lp, 0, d) - want) < 1e-12
        assert abs(R.resistance_from_inverse(G, 3, (3 + d) % n) - want) < 1e-12
    np.testing.assert_allclose(R.farness_dense(Lp, 4), (n * n - 1) / 6, rtol=1e-12)


def test_complete_graph():
    n = 8
    _, Lp, G = dense_routes(synth.complete_graph(n))
    assert abs(R.resistance_from_inverse(Lp, 1, 5) - 2 / n) < 1e-13
    assert abs(R.resistance_from_inverse(G, 0, 7) - 2 / n) < 1e-13
    np.testing.assert_allclose(R.farness_dense(Lp, 3), 2 * (n - 1) / n, rtol=1e-12)


def test_complete_bipartite():
    a, b = 3, 5
    _, Lp, G = dense_routes(synth.complete_bipartite(a, b))
    # same side (both in the a-side): 2/b; across: (a+b-1)/(ab)
    assert abs(R.resistance_from_inverse(Lp, 0, 1) - 2 / b) < 1e-12
    assert abs(R.resistance_from_inverse(Lp, a, a + 1) - 2 / a) < 1e-12
    assert abs(R.resistance_from_inverse(G, 0, a + 2) - (a + b - 1) / (a * b)) < 1e-12


def test_star():
    n = 10
    _, Lp, _ = dense_routes(synth.star_graph(n))
    assert abs(R.resistance_from_inverse(Lp, 0, 4) - 1) < 1e-12
    assert abs(R.resistance_from_inverse(Lp, 2, 7) - 2) < 1e-12
    np.testing.assert_allclose(R.farness_dense(Lp, 0), n - 1, rtol=1e-12)
    np.testing.assert_allclose(R.farness_dense(Lp, 3), 1 + 2 * (n - 2), rtol=1e-12)


def _tree_path_resistance(n, u, v, w, a, b):
    adj = {i: [] for i in range(n)}
    for x, y, ww in zip(u, v, w):
        adj[x].append((y, ww))
        adj[y].append((x, ww))
    stack = [(a, 0.0, -1)]
    while stack:
        x, acc, par = stack.pop()
        if x == b:
            return acc
        for y, ww in adj[x]:
            if y != par:
                stack.append((y, acc + 1.0 / ww, x))
    raise AssertionError


def test_weighted_tree_resistance_is_path_length():
    rng = np.random.default_rng(7)
    n = 25
    par = [int(rng.integers(0, i)) for i in range(1, n)]
    u = np.array(par, np.int64)
    v = np.arange(1, n, dtype=np.int64)
    w = rng.uniform(0.5, 3.0, n - 1)
    g = synth.EdgeList(n, np.minimum(u, v), np.maximum(u, v), w)
    _, Lp, G = dense_routes(g)
    for a, b in [(0, 24), (3, 17), (11, 12), (5, 5)]:
        want = _tree_path_resistance(n, u, v, w, a, b)
        assert abs(R.resistance_from_inverse(Lp, a, b) - want) < 1e-10
        assert abs(R.resistance_from_inverse(G, a, b) - want) < 1e-10


def test_foster_sum():
    g = synth.random_connected(30, 80, seed=3)
    _, Lp, _ = dense_routes(g)
    tot = float(np.sum(g.w * R.resistance_from_inverse(Lp, g.u, g.v)))
    assert abs(tot - (g.n - 1)) < 1e-10


# ---- brute force: Kirchhoff's spanning-forest formula -----------------------

def _forest_weight(n, edges, ws, size, sep=None):
    tot = 0.0
    for idx in itertools.combinations(range(len(edges)), size):
        parent = list(range(n))

        def f(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x
        ok = True
        prod = 1.0
        for i in idx:
            a, b = edges[i]
            ra, rb = f(a), f(b)
            if ra == rb:
                ok = False
                break
            parent[ra] = rb
            prod *= ws[i]
        if ok and (sep is None or f(sep[0]) != f(sep[1])):
            tot += prod
    return tot


def test_resistance_by_spanning_forest_enumeration():
    """R(u,v) = (weight of 2-forests separating u from v) / (weight of spanning
    trees): Kirchhoff's theorem, enumerated by brute force on a tiny graph."""
    g = synth.random_connected(6, 9, seed=11)
    edges = list(zip(g.u.tolist(), g.v.tolist()))
    trees = _forest_weight(g.n, edges, g.w, g.n - 1)
    _, Lp, G = dense_routes(g)
    for a, b in [(0, 5), (1, 3), (2, 4)]:
        want = _forest_weight(g.n, edges, g.w, g.n - 2, sep=(a, b)) / trees
        assert abs(R.resistance_from_inverse(Lp, a, b) - want) < 1e-12
        assert abs(R.resistance_from_inverse(G, a, b) - want) < 1e-12


# ---- grid spectral closed form (no oracle code involved) -------------------

def grid_spectral_farness(N, r, c):
    """Farness of node (r, c) on the N x N grid from the DCT eigenbasis of the
    path Laplacian: L^+_vv = sum phi_j(r)^2 phi_k(c)^2 / lambda_jk,
    f(v) = n L^+_vv + tr L^+ (since L^+ 1 = 0)."""
    j = np.arange(N)
    lam1 = 4.0 * np.sin(np.pi * j / (2 * N)) ** 2
    lam = lam1[:, None] + lam1[None, :]
    cj = np.where(j == 0, math.sqrt(1.0 / N), math.sqrt(2.0 / N))
    phr = cj * np.cos(np.pi * j * (r + 0.5) / N)
    phc = cj * np.cos(np.pi * j * (c + 0.5) / N)
    inv = np.zeros_like(lam)
    inv[lam > 0] = 1.0 / lam[lam > 0]
    inv[0, 0] = 0.0
    lvv = float(np.sum((phr[:, None] ** 2) * (phc[None, :] ** 2) * inv))
    return N * N * lvv + float(inv.sum())


def test_grid32_corner_farness_all_routes():
    g = synth.grid(32)
    want = grid_spectral_farness(32, 0, 0)
    L, Lp, G = dense_routes(g)
    assert abs(R.farness_dense(Lp, 0)[0] / want - 1) < 1e-11
    assert abs(R.farness_dense(G, 0)[0] / want - 1) < 1e-11
    f_cg = R.farness_exact_cg(LAP.of(g), 0, tol=1e-13)
    assert abs(f_cg / want - 1) < 1e-10
    assert abs(R.closeness(1024, f_cg) - 1023 / want) < 1e-12
    # interior node too (an index slip between rows and columns would show here)
    assert abs(R.farness_dense(Lp, 5 * 32 + 9)[0] / grid_spectral_farness(32, 5, 9) - 1) < 1e-11


def test_grounded_sparse_matches_dense_and_closed_forms():
    # weighted graph: against the dense pseudoinverse, for every choice of ground
    g = synth.random_connected(60, 200, seed=4)
    Lp = R.pinv(LAP.of(g, dense=True))
    rng = np.random.default_rng(6)
    s, t = rng.integers(0, 60, 30), rng.integers(0, 60, 30)
    for gnd in (0, int(s[0]), 59):
        np.testing.assert_allclose(R.resistance_grounded_sparse(LAP.of(g), s, t, gnd),
                                   R.resistance_from_inverse(Lp, s, t), atol=1e-12)
    # path: distance; cycle: d (n - d) / n
    np.testing.assert_allclose(R.resistance_grounded_sparse(LAP.of(synth.path_graph(9)), [0, 2], [8, 7]),
                               [8.0, 5.0], atol=1e-12)
    np.testing.assert_allclose(R.resistance_grounded_sparse(LAP.of(synth.cycle_graph(10)), [0], [3], 5),
                               [3 * 7 / 10], atol=1e-12)


def test_cg_matches_dense_on_weighted_graph():
    g = synth.random_connected(60, 200, seed=5)
    L, Lp, _ = dense_routes(g)
    s = np.array([0, 7, 33, 59])
    t = np.array([1, 50, 2, 10])
    np.testing.assert_allclose(R.resistance_cg(LAP.of(g), s, t, 1e-13),
                               R.resistance_from_inverse(Lp, s, t), rtol=1e-10)


def test_cg_solution_is_pseudoinverse_solution():
    g = synth.random_connected(50, 120, seed=9)
    L, Lp, _ = dense_routes(g)
    rng = np.random.default_rng(0)
    B = rng.standard_normal((50, 3))
    B -= B.mean(axis=0)
    X, _ = R.cg(LAP.of(g), B, 1e-13)
    np.testing.assert_allclose(X, Lp @ B, atol=1e-10)
    np.testing.assert_allclose(X.sum(axis=0), 0, atol=1e-11)


def test_scaling_and_rayleigh_monotonicity():
    g = synth.random_connected(30, 60, seed=2)
    _, Lp, _ = dense_routes(g)
    g2 = synth.EdgeList(g.n, g.u, g.v, 3.0 * g.w)
    _, Lp2, _ = dense_routes(g2)
    np.testing.assert_allclose(R.resistance_matrix(Lp2), R.resistance_matrix(Lp) / 3.0, atol=1e-12)
    g3 = synth.EdgeList(g.n, g.u.copy(), g.v.copy(), g.w.copy())
    g3.w[0] *= 5.0  # raising a conductance never raises a resistance
    _, Lp3, _ = dense_routes(g3)
    assert np.all(R.resistance_matrix(Lp3) <= R.resistance_matrix(Lp) + 1e-12)


# ---- the counter-based generator -------------------------------------------

def test_splitmix64_published_vector():
    vals = [int(x) for x in open(os.path.join(GOLD, "splitmix64_seed1234567.txt"))
            if x.strip() and not x.startswith("#")]
    g = RNG.SplitMix64(1234567)
    assert [g.next() for _ in range(5)] == vals
    # the stateless step equals one sequential step
    assert RNG.step(1234567) == vals[0]


def test_lemire_bounded_uniform():
    words = RNG.sample_stream(99, 0)
    bound = 7
    counts = np.bincount([RNG.lemire_bounded(words, bound) for _ in range(70000)], minlength=bound)
    chi2 = float(((counts - 10000) ** 2 / 10000).sum())
    assert chi2 < 30  # 6 d.o.f.; p ~ 4e-5
    # a bound that forces rejection work still stays in range
    assert all(0 <= RNG.lemire_bounded(words, (1 << 63) + 5) < (1 << 63) + 5 for _ in range(100))


def test_floyd_subsets_uniform():
    n, k = 5, 2
    counts = {}
    for seed in range(20000):
        s = tuple(RNG.floyd_subset(n, k, RNG.sample_stream(seed, 3)))
        assert len(set(s)) == k and all(0 <= x < n for x in s)
        counts[s] = counts.get(s, 0) + 1
    assert len(counts) == math.comb(n, k)
    exp = 20000 / math.comb(n, k)
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 35  # 9 d.o.f.
    assert RNG.floyd_subset(6, 6, RNG.sample_stream(1, 1)) == list(range(6))


def test_jl_sign_words_match_scalar_hash():
    lo = np.array([0, 3, 17], np.int64)
    hi = np.array([5, 9, 40], np.int64)
    wd = RNG.jl_sign_word(42, 2, lo, hi)
    for e in range(3):
        assert int(wd[e]) == RNG.hash4(42, RNG.TAG_JL, 2, (int(lo[e]) << 32) | int(hi[e]))
    S = RNG.jl_signs(42, 130, lo, hi)
    assert S.shape == (130, 3) and set(np.unique(S)) <= {-1, 1}
    assert int(S[129, 1]) == (1 if ((int(RNG.jl_sign_word(42, 2, lo, hi)[1]) >> 1) & 1) == 0 else -1)
    # roughly balanced
    big = RNG.jl_signs(1, 256, np.arange(1000), np.arange(1000) + 1000)
    assert abs(big.mean()) < 0.01


# ---- estimators: special cases and statistics ------------------------------

def test_sampling_with_k_equal_n_is_exact():
    g = synth.random_connected(40, 100, seed=1)
    L, Lp, _ = dense_routes(g)
    nodes = [0, 13, 39]
    f, c, piv, d = E.sampling(LAP.of(g), g, nodes, g.n, seed=5)
    np.testing.assert_allclose(f, R.farness_dense(Lp, nodes), rtol=1e-10)
    np.testing.assert_allclose(c, (g.n - 1) / R.farness_dense(Lp, nodes), rtol=1e-10)
    assert all(len(p) == g.n for p in piv)


def test_sampling_dense_and_cg_agree_and_pivots_are_the_generator_s():
    g = synth.random_connected(40, 100, seed=1)
    _, Lp, _ = dense_routes(g)
    f1, _, p1, d1 = E.sampling(LAP.of(g), g, [2, 9], 10, seed=3)
    f2, _, p2, d2 = E.sampling(None, g, [2, 9], 10, seed=3, solver="dense", Lp=Lp)
    np.testing.assert_allclose(f1, f2, rtol=1e-10)
    assert [list(p) for p in p1] == [RNG.pivots(3, 2, 40, 10), RNG.pivots(3, 9, 40, 10)]


def test_sampling_is_unbiased_for_farness():
    """Prop. 1: E[(n/k) sum_S d_ER(v, s)] = farness(v) (statistical), through
    the oracle's estimator itself; closeness is (k/n)(n-1)/sum_S d_ER."""
    g = synth.random_connected(40, 100, seed=1)
    _, Lp, _ = dense_routes(g)
    v, k = 4, 10
    exact = R.farness_dense(Lp, v)[0]
    est = []
    for seed in range(4000):
        f, c, piv, d = E.sampling(None, g, [v], k, seed, solver="dense", Lp=Lp)
        assert abs(c[0] - (k / g.n) * (g.n - 1) / d[0].sum()) < 1e-12 * c[0]
        est.append(f[0])
    est = np.array(est)
    se = est.std() / math.sqrt(len(est))
    assert abs(est.mean() - exact) < 5 * se
    assert est.std() > 0


def test_projection_with_identity_q_is_exact():
    g = synth.random_connected(30, 70, seed=4)
    L, Lp, _ = dense_routes(g)
    nodes = [0, 11, 29]
    f, c, Z = E.projection(LAP.of(g), g, nodes, g.m, 0, Q=np.eye(g.m))
    np.testing.assert_allclose(f, R.farness_dense(Lp, nodes), rtol=1e-10)
    f2, _, _ = E.projection(None, g, nodes, g.m, 0, solver="dense", Lp=Lp, Q=np.eye(g.m))
    np.testing.assert_allclose(f2, f, rtol=1e-10)


def test_projection_rhs_is_incidence_product():
    g = synth.random_connected(12, 20, seed=8)
    k = 70
    Y = E.projection_rhs(g, k, seed=2)
    Bm = np.zeros((g.m, g.n))
    Bm[np.arange(g.m), g.u] = 1.0
    Bm[np.arange(g.m), g.v] = -1.0
    Q = RNG.jl_signs(2, k, g.u, g.v) / np.sqrt(k)
    np.testing.assert_allclose(Y, (Q @ np.diag(np.sqrt(g.w)) @ Bm).T, atol=1e-14)
    np.testing.assert_allclose(Y.sum(axis=0), 0, atol=1e-12)


def test_projection_unbiased_and_concentrates():
    """E[d~] = d_ER for Rademacher Q; with larger k the error shrinks (JL)."""
    g = synth.random_connected(30, 70, seed=4)
    _, Lp, _ = dense_routes(g)
    exact = R.farness_dense(Lp, [5])[0]
    est = [E.projection(None, g, [5], 32, s, solver="dense", Lp=Lp)[0][0] for s in range(300)]
    est = np.array(est)
    assert abs(est.mean() - exact) < 5 * est.std() / math.sqrt(len(est))
    big = E.projection(None, g, [5], 2048, 7, solver="dense", Lp=Lp)[0][0]
    assert abs(big / exact - 1) < 0.1
