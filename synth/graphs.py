"""Seeded graph generators (numpy PCG64 streams).

Every generator returns an :class:`EdgeList` in canonical form: each undirected
edge once as (lo, hi) with lo < hi, sorted by (lo, hi), no self-loops, no
duplicates.  Weights are float64 conductances (the paper treats an edge weight
as the conductance of a resistor, Sec. 2) or ``None`` for unit weights.

The shapes stand in for the paper's benchmark networks (Sec. 6.3, Tables 2-3),
which are not available here: Barabasi-Albert and R-MAT graphs for skewed-degree
complex networks, perturbed 2D grids for road networks.
"""
from __future__ import annotations

import os
from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class EdgeList:
    n: int
    u: np.ndarray            # int64[m], lo endpoint
    v: np.ndarray            # int64[m], hi endpoint
    w: Optional[np.ndarray]  # float64[m] or None (unit weights)
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.u.shape[0])

    def weights(self) -> np.ndarray:
        return np.ones(self.m) if self.w is None else self.w


def _canon(n, a, b, w=None, name=""):
    a = np.asarray(a, np.int64)
    b = np.asarray(b, np.int64)
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    keep = lo != hi
    lo, hi = lo[keep], hi[keep]
    key = lo * np.int64(n) + hi
    if w is None:
        key = np.unique(key)
        return EdgeList(n, key // n, key % n, None, name)
    w = np.asarray(w, np.float64)[keep]
    order = np.argsort(key, kind="stable")
    key, w = key[order], w[order]
    first = np.ones(key.shape[0], bool)
    first[1:] = key[1:] != key[:-1]
    return EdgeList(n, key[first] // n, key[first] % n, w[first], name)


def _components(n, u, v):
    """Connected-component label per node (min-label propagation with
    pointer jumping; vectorised, O(log n) rounds on typical graphs)."""
    lab = np.arange(n, dtype=np.int64)
    while True:
        mn = np.minimum(lab[u], lab[v])
        new = lab.copy()
        np.minimum.at(new, u, mn)
        np.minimum.at(new, v, mn)
        new = new[new]
        if np.array_equal(new, lab):
            return lab
        lab = new


def lcc(g: EdgeList) -> EdgeList:
    """Largest connected component, relabelled in increasing original id."""
    if g.m == 0:
        return EdgeList(1, np.zeros(0, np.int64), np.zeros(0, np.int64), None if g.w is None else np.zeros(0), g.name)
    lab = _components(g.n, g.u, g.v)
    cnt = np.bincount(lab, minlength=g.n)
    big = int(np.argmax(cnt))
    keep_nodes = np.nonzero(lab == big)[0]
    newid = -np.ones(g.n, np.int64)
    newid[keep_nodes] = np.arange(keep_nodes.shape[0])
    ke = lab[g.u] == big
    return EdgeList(int(keep_nodes.shape[0]), newid[g.u[ke]], newid[g.v[ke]],
                    None if g.w is None else g.w[ke], g.name)


def _uniform_weights(rng, m, lo, hi):
    return rng.uniform(lo, hi, m) if m else np.zeros(0)


def grid(N: int, M: Optional[int] = None, name="") -> EdgeList:
    """N x M 4-neighbour grid, node id = r*M + c, unit weights."""
    M = N if M is None else M
    idx = np.arange(N * M, dtype=np.int64).reshape(N, M)
    a = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    b = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return _canon(N * M, a, b, None, name or f"grid{N}x{M}")


def road_grid(N: int, drop_frac=0.02, wlo=1.0, whi=10.0, seed=1) -> EdgeList:
    """Road-like graph: N x N grid, exactly round(drop_frac*m) edges deleted
    uniformly at random, largest connected component, weights U[wlo, whi]."""
    rng = np.random.default_rng([seed, 0x524F4144])
    g = grid(N)
    ndrop = int(round(drop_frac * g.m))
    drop = rng.choice(g.m, ndrop, replace=False)
    keep = np.ones(g.m, bool)
    keep[drop] = False
    h = EdgeList(g.n, g.u[keep], g.v[keep], None, f"road{N}")
    h = lcc(h)
    h.w = _uniform_weights(rng, h.m, wlo, whi)
    h.name = f"road{N}"
    return h


def barabasi_albert(n: int, d: int = 4, seed=1) -> EdgeList:
    """Barabasi-Albert preferential attachment: seed clique K_{d+1}, then each
    new node attaches d distinct targets drawn proportionally to degree from
    the repeated-endpoint list.  m = d*n - d(d+1)/2."""
    rng = np.random.default_rng([seed, 0x4241])
    m = d * n - d * (d + 1) // 2
    us = np.empty(m, np.int64)
    vs = np.empty(m, np.int64)
    rep = np.empty(2 * m, np.int64)
    e = 0
    for i in range(d + 1):
        for j in range(i):
            us[e], vs[e] = j, i
            rep[2 * e], rep[2 * e + 1] = i, j
            e += 1
    # draw in chunks of random numbers to keep the Python loop light
    buf = rng.random(1 << 16)
    bi = 0
    for x in range(d + 1, n):
        ln = 2 * e
        t = set()
        while len(t) < d:
            if bi == buf.shape[0]:
                buf = rng.random(1 << 16)
                bi = 0
            t.add(int(rep[int(buf[bi] * ln)]))
            bi += 1
        for y in sorted(t):
            us[e], vs[e] = y, x
            rep[2 * e], rep[2 * e + 1] = x, y
            e += 1
    return _canon(n, us, vs, None, f"ba{n}")


def rmat(scale: int, edge_factor: int = 16, a=0.57, b=0.19, c=0.19, seed=1,
         weights=(1.0, 4.0)) -> EdgeList:
    """R-MAT (Chakrabarti et al.): 2^scale vertices, edge_factor*2^scale draws,
    quadrant probabilities (a, b, c, 1-a-b-c), no label permutation;
    symmetrised, self-loops and duplicates dropped, largest connected component
    relabelled in increasing id; weights U[weights] per canonical edge
    (None = unit)."""
    rng = np.random.default_rng([seed, 0x524D4154, scale])
    n = 1 << scale
    m = edge_factor * n
    u = np.zeros(m, np.int64)
    v = np.zeros(m, np.int64)
    chunk = 1 << 22
    for s in range(0, m, chunk):
        e = min(m, s + chunk)
        uu = np.zeros(e - s, np.int64)
        vv = np.zeros(e - s, np.int64)
        for lev in range(scale):
            r = rng.random(e - s)
            bit = np.int64(1) << np.int64(scale - 1 - lev)
            down = r >= a + b                       # quadrant c or d: row bit set
            right = ((r >= a) & (r < a + b)) | (r >= a + b + c)  # b or d: column bit set
            uu |= np.where(down, bit, 0)
            vv |= np.where(right, bit, 0)
        u[s:e] = uu
        v[s:e] = vv
    g = lcc(_canon(n, u, v, None, f"rmat{scale}"))
    if weights is not None:
        g.w = _uniform_weights(rng, g.m, weights[0], weights[1])
    g.name = f"rmat{scale}"
    return g


def random_connected(n: int, m: int, seed=1, weights=(1.0, 4.0)) -> EdgeList:
    """Random spanning tree plus extra random edges; connected by construction."""
    rng = np.random.default_rng([seed, 0x52434E])
    perm = rng.permutation(n)
    parents = np.array([perm[rng.integers(0, i)] for i in range(1, n)], np.int64) if n > 1 else np.zeros(0, np.int64)
    a = list(perm[1:])
    b = list(parents)
    g = _canon(n, a, b)
    tries = 0
    while g.m < m and tries < 50:
        k = (m - g.m) * 2 + 8
        aa = rng.integers(0, n, k)
        bb = rng.integers(0, n, k)
        g2 = _canon(n, np.concatenate([g.u, aa]), np.concatenate([g.v, bb]))
        if g2.m > m:
            # keep the tree edges and enough extra edges
            key_tree = set((g.u * n + g.v).tolist())
            keys = (g2.u * n + g2.v)
            is_tree = np.array([k in key_tree for k in keys.tolist()])
            extra_idx = np.nonzero(~is_tree)[0]
            pick = np.sort(rng.choice(extra_idx, m - g.m, replace=False))
            sel = np.sort(np.concatenate([np.nonzero(is_tree)[0], pick]))
            g2 = EdgeList(n, g2.u[sel], g2.v[sel], None)
        g = g2
        tries += 1
    if weights is not None:
        g.w = _uniform_weights(rng, g.m, weights[0], weights[1])
    g.name = f"rand{n}_{m}"
    return g


def path_graph(n, w=None):
    return _canon(n, np.arange(n - 1), np.arange(1, n), w, f"path{n}")


def cycle_graph(n):
    return _canon(n, np.arange(n), (np.arange(n) + 1) % n, None, f"cycle{n}")


def complete_graph(n):
    iu = np.triu_indices(n, 1)
    return _canon(n, iu[0], iu[1], None, f"K{n}")


def complete_bipartite(a, b):
    x, y = np.meshgrid(np.arange(a), a + np.arange(b), indexing="ij")
    return _canon(a + b, x.ravel(), y.ravel(), None, f"K{a},{b}")


def star_graph(n):
    """Star with hub 0 and n-1 leaves."""
    return _canon(n, np.zeros(n - 1, np.int64), np.arange(1, n), None, f"star{n}")


def query_nodes(n: int, q: int, seed=1) -> np.ndarray:
    """q distinct query nodes drawn uniformly, sorted."""
    rng = np.random.default_rng([seed, 0x51525259])
    return np.sort(rng.choice(n, min(q, n), replace=False)).astype(np.int64)


def cached(name: str, fn, *args, **kw) -> EdgeList:
    """Memoise a generator's output as .npz under $CFC_GRAPH_CACHE (if set)."""
    root = os.environ.get("CFC_GRAPH_CACHE")
    if not root:
        return fn(*args, **kw)
    os.makedirs(root, exist_ok=True)
    path = os.path.join(root, name + ".npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        w = z["w"] if z["has_w"] else None
        return EdgeList(int(z["n"]), z["u"], z["v"], w, name)
    g = fn(*args, **kw)
    np.savez(path, n=g.n, u=g.u, v=g.v, w=g.w if g.w is not None else np.zeros(0), has_w=g.w is not None)
    return g
