"""GPU parity of shared-pivot Sampling, all-node projection closeness,
spanning-edge centrality and current-flow betweenness against the CPU oracle
(through the C ABI).

Bars: estimator outputs match the oracle for the same seed to <= 1e-6
relative (the solves run at tol 1e-9 or tighter, the oracle's at 1e-12);
exact quantities match closed forms or the dense pseudoinverse.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import betweenness as CB
from oracle import edges as SE
from oracle import estimators as E
from oracle import laplacian as LAP
from oracle import resistance as R
from oracle import rng as ORNG

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_1607_02955_amd as cfc
    return cfc.Context(0)


def load(ctx, eg, **setup):
    import paper_1607_02955_amd as cfc
    g = cfc.Graph.from_edgelist(ctx, eg)
    g.build_hierarchy(**setup)
    return g


def hubbed(n=2500, m=7000, hubs=2, hub_deg=900, seed=5):
    """Weighted random graph plus a few hubs whose degree exceeds the
    heavy-row threshold, so heavy-row segments are exercised."""
    base = synth.random_connected(n, m, seed=seed)
    rng = np.random.default_rng(seed)
    a, b, w = [base.u], [base.v], [base.w]
    for h in range(hubs):
        nb = rng.choice(np.arange(hubs, n), hub_deg, replace=False)
        a.append(np.full(hub_deg, h, np.int64))
        b.append(nb.astype(np.int64))
        w.append(rng.uniform(1, 4, hub_deg))
    a, b, w = np.concatenate(a), np.concatenate(b), np.concatenate(w)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo * n + hi
    key, first = np.unique(key, return_index=True)
    return synth.EdgeList(n, key // n, key % n, w[first])


# ---- shared-pivot Sampling ----------------------------------------------------

def test_shared_sampling_matches_oracle(ctx):
    import paper_1607_02955_amd as cfc
    eg = synth.barabasi_albert(3000, 4, seed=21)
    k, seed = 150, 7
    S = cfc.shared_pivots(seed, eg.n, k)
    # query nodes: random ones, the reference pivot S[0], another pivot, a repeat
    nodes = np.concatenate([synth.query_nodes(eg.n, 6, seed=4), [S[0], S[5], S[5]]])
    g = load(ctx, eg)
    far, clo, st = g.farness_sampling_shared(nodes, k, seed, stats=True, tol=1e-9, block=64)
    say("shared sampling", st)
    assert st["columns"] == len(set(S.tolist()) | set(nodes.tolist())) - 1
    of, oc, So = E.sampling_shared(LAP.of(eg), eg, nodes, k, seed, tol=1e-12)
    assert So.tolist() == S.tolist()
    np.testing.assert_allclose(far, of, rtol=1e-6)
    np.testing.assert_allclose(clo, oc, rtol=1e-6)


def test_shared_sampling_k_at_least_n_is_exact(ctx):
    eg = synth.random_connected(300, 900, seed=3)
    g = load(ctx, eg, coarsest_max=64)
    nodes = np.array([0, 17, 299])
    far, clo = g.farness_sampling_shared(nodes, 400, 1, tol=1e-10, precision=1)
    Lp = R.pinv(LAP.of(eg, dense=True))
    np.testing.assert_allclose(far, R.farness_dense(Lp, nodes), rtol=1e-8)


# ---- all-node projection closeness --------------------------------------------

def test_all_node_projection_closeness(ctx):
    eg = synth.random_connected(1500, 5000, seed=9)
    g = load(ctx, eg, coarsest_max=64)
    g.jl_sketch(64, seed=2, tol=1e-9, block=64)
    far, clo = g.farness_jl()
    assert far.shape == (eg.n,)
    of, oc, _ = E.projection(LAP.of(eg), eg, np.arange(eg.n), 64, 2, tol=1e-12)
    np.testing.assert_allclose(far, of, rtol=1e-6)
    np.testing.assert_allclose(clo, oc, rtol=1e-6)
    f2, _ = g.farness_jl([5, 1499])
    np.testing.assert_allclose(f2, far[[5, 1499]], rtol=0, atol=0)


# ---- spanning-edge centrality -------------------------------------------------

def test_spanning_edge_exact(ctx):
    import paper_1607_02955_amd as cfc
    eg = synth.random_connected(1200, 4000, seed=12)
    g = load(ctx, eg, coarsest_max=64)
    c = g.spanning_edge(eg.u, eg.v, tol=1e-10, block=256)
    Lp = R.pinv(LAP.of(eg, dense=True))
    want = SE.spanning_edge(None, eg, eg.u, eg.v, "dense", Lp=Lp)
    np.testing.assert_allclose(c, want, rtol=1e-7)
    assert abs(c.sum() - (eg.n - 1)) < 1e-6 * eg.n  # Foster
    # (hi, lo) order is the same edge
    np.testing.assert_allclose(g.spanning_edge(eg.v[:5], eg.u[:5], tol=1e-10), c[:5], rtol=1e-7)
    with pytest.raises(cfc.CfcError):
        g.spanning_edge([0], [0])
    with pytest.raises(cfc.CfcError):
        missing = next(x for x in range(1, eg.n) if x not in set(eg.v[eg.u == 0].tolist()))
        g.spanning_edge([0], [missing])


def test_spanning_edge_projection_matches_oracle(ctx):
    eg = hubbed(n=1500, m=4500, hubs=1, hub_deg=700, seed=8)
    g = load(ctx, eg)
    sel = np.arange(0, eg.m, 3)
    c, st = g.spanning_edge_jl(eg.u[sel], eg.v[sel], 96, seed=3, stats=True, tol=1e-9, block=64)
    say("spanning edge jl", st)
    want = SE.spanning_edge_jl(LAP.of(eg), eg, eg.u[sel], eg.v[sel], 96, 3, tol=1e-12)
    np.testing.assert_allclose(c, want, rtol=1e-6)


# ---- current-flow betweenness -------------------------------------------------

def test_cfb_exact_closed_forms(ctx):
    n = 21
    g = load(ctx, synth.path_graph(n))
    want = np.array([i * (n - 1 - i) for i in range(n)]) / ((n - 1) * (n - 2) / 2)
    np.testing.assert_allclose(g.cfb_exact(tol=1e-10), want, atol=1e-8)
    g = load(ctx, synth.star_graph(15))
    cb = g.cfb_exact(tol=1e-10)
    assert abs(cb[0] - 1) < 1e-8 and np.all(np.abs(cb[1:]) < 1e-8)
    g = load(ctx, synth.complete_graph(12))
    np.testing.assert_allclose(g.cfb_exact(tol=1e-10), 1 / 12, rtol=1e-8)


def test_cfb_exact_matches_oracle_multilevel(ctx):
    eg = synth.random_connected(140, 420, seed=6)
    g = load(ctx, eg, coarsest_max=32)
    assert g.info()["levels"] >= 2
    cb, st = g.cfb_exact(stats=True, tol=1e-10, block=128)
    say("cfb exact", st)
    assert st["columns"] == eg.n * (eg.n - 1) // 2
    want = CB.cfb_exact(eg, R.pinv(LAP.of(eg, dense=True)))
    np.testing.assert_allclose(cb, want, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("W", [64, 256, 512])
def test_cfb_sampled_heavy_rows_matches_oracle(ctx, W):
    eg = hubbed(seed=W)
    g = load(ctx, eg)
    count = 2 * W + 37  # several blocks and a ragged tail
    cb, st = g.cfb_sampled(count, seed=4, stats=True, tol=1e-9, block=W)
    say("cfb sampled", W, st)
    want = CB.cfb_sampled(LAP.of(eg), eg, count, 4, tol=1e-12)
    np.testing.assert_allclose(cb, want, rtol=1e-6, atol=1e-9 * want.max())


def test_current_throughput_raw_pairs(ctx):
    eg = synth.road_grid(30, seed=2)
    g = load(ctx, eg, coarsest_max=64)
    rng = np.random.default_rng(1)
    s = rng.integers(0, eg.n, 70)
    t = rng.integers(0, eg.n, 70)
    t[3] = s[3]  # no current
    tau = g.current_throughput(s, t, tol=1e-10, block=32)
    keep = s != t
    P = CB.potentials(LAP.of(eg), eg, s[keep], t[keep], tol=1e-12)
    want = CB.throughput(eg, P, s[keep], t[keep]).sum(axis=1)
    np.testing.assert_allclose(tau, want, rtol=1e-7, atol=1e-9 * want.max())
    # random pairs: library draws equal the oracle's
    import paper_1607_02955_amd as cfc
    a, b = cfc.random_pairs(4, eg.n, 50)
    ao, bo = ORNG.random_pairs(4, eg.n, 50)
    assert a.tolist() == ao.tolist() and b.tolist() == bo.tolist()


def test_centrality_edge_cases(ctx):
    import paper_1607_02955_amd as cfc
    g = load(ctx, synth.path_graph(3))
    np.testing.assert_allclose(g.cfb_exact(tol=1e-10), [0.0, 1.0, 0.0], atol=1e-9)
    np.testing.assert_allclose(g.current_throughput([], [], tol=1e-10), 0.0)
    assert g.spanning_edge([], []).shape == (0,)
    np.testing.assert_allclose(g.spanning_edge([0, 1], [1, 2], tol=1e-10), [1.0, 1.0], rtol=1e-9)
    far, clo = g.farness_sampling_shared([], 2, 1)
    assert far.shape == (0,)
    far, clo = g.farness_sampling_shared([0, 1, 2], 10, 1, tol=1e-10)  # k clamped to n: exact
    np.testing.assert_allclose(far, [3.0, 2.0, 3.0], rtol=1e-9)
    with pytest.raises(cfc.CfcError):
        g.cfb_sampled(0)
    with pytest.raises(cfc.CfcError):
        g.farness_sampling_shared([3], 2, 1)
    with pytest.raises(cfc.CfcError):
        g.current_throughput([0], [3])
    g2 = load(ctx, synth.path_graph(2))
    with pytest.raises(cfc.CfcError):
        g2.cfb_exact()


@pytest.mark.parametrize("order", [1, 2, 3])
def test_locality_orders_same_resistances(ctx, order):
    eg = synth.rmat(12, seed=2)
    g = load(ctx, eg, coarsest_max=64, order=order)
    rng = np.random.default_rng(order)
    s = rng.integers(0, eg.n, 100)
    t = rng.integers(0, eg.n, 100)
    Rm = R.resistance_matrix(R.pinv(LAP.of(eg, dense=True)))
    np.testing.assert_allclose(g.resistance(s, t, tol=1e-10, precision=1), Rm[s, t], rtol=1e-8, atol=1e-12)


# ---- the same estimators at the benchmark tolerance ----------------------------

@pytest.mark.parametrize("kind", ["shared", "all_node_jl", "spanning_jl", "cfb"])
def test_estimators_at_bench_tolerance(ctx, kind):
    """At the solve tolerance the benchmarks run (1e-6, mixed precision, the
    autotuned cycle) every estimator matches the oracle's (same seed,
    solves to 1e-12) to <= 1e-4 relative."""
    print(f"case: {kind} at tol 1e-6", flush=True)
    if kind == "shared":
        eg = synth.barabasi_albert(4000, 4, seed=31)
        nodes = synth.query_nodes(eg.n, 12, seed=2)
        g = load(ctx, eg)
        got, _, st = g.farness_sampling_shared(nodes, 300, 5, stats=True, tol=1e-6)
        want, _, _ = E.sampling_shared(LAP.of(eg), eg, nodes, 300, 5, tol=1e-12)
    elif kind == "all_node_jl":
        eg = synth.road_grid(60, seed=4)
        g = load(ctx, eg)
        st = g.jl_sketch(128, seed=6, tol=1e-6, stats=True)
        got, _ = g.farness_jl()
        want, _, _ = E.projection(LAP.of(eg), eg, np.arange(eg.n), 128, 6, tol=1e-12)
    elif kind == "spanning_jl":
        eg = hubbed(n=3000, m=9000, hubs=1, hub_deg=800, seed=13)
        g = load(ctx, eg)
        got, st = g.spanning_edge_jl(eg.u, eg.v, 128, seed=9, stats=True, tol=1e-6)
        want = SE.spanning_edge_jl(LAP.of(eg), eg, eg.u, eg.v, 128, 9, tol=1e-12)
    else:
        eg = synth.barabasi_albert(2500, 4, seed=33)
        g = load(ctx, eg)
        got, st = g.cfb_sampled(700, seed=8, stats=True, tol=1e-6)
        want = CB.cfb_sampled(LAP.of(eg), eg, 700, 8, tol=1e-12)
    scale = np.abs(want).max()
    err = np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-3 * scale))
    say(kind, "max rel err vs oracle", err, "max rel residual", st["max_rel_residual"])
    assert st["max_rel_residual"] <= 1e-6
    assert err <= 1e-4
