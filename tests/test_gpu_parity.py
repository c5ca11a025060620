"""GPU parity of the HIP solve path against the CPU oracle (through the C ABI).

Tolerances: the solve is checked on relative farness / resistance error
(<= 1e-6 at the tolerances used below, tighter in FP64 mode); estimator
outputs must match the oracle's for the same seed to <= 1e-4 relative.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import estimators as E
from oracle import laplacian as LAP
from oracle import resistance as R

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


def dense_R(eg):
    Lp = R.pinv(LAP.of(eg, dense=True))
    return Lp, R.resistance_matrix(Lp)


def test_single_level_is_exact_pinv(ctx):
    """n <= coarsest_max: the preconditioner is the MFMA pseudoinverse apply."""
    eg = synth.random_connected(40, 100, seed=1)
    say("single-level", eg.n, eg.m)
    g = load(ctx, eg)
    assert g.info()["levels"] == 1
    _, Rm = dense_R(eg)
    s = np.arange(40)
    t = (s * 7 + 3) % 40
    for W, prec in [(32, 1), (64, 0), (1, 1), (256, 0)]:
        r = g.resistance(s, t, block=W, precision=prec, tol=1e-10)
        np.testing.assert_allclose(r, Rm[s, t], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("W", [1, 32, 64, 128, 256, 512])
def test_block_widths_weighted_random(ctx, W):
    eg = synth.random_connected(1500, 6000, seed=W)
    say("widths", W, eg.n, eg.m)
    g = load(ctx, eg, coarsest_max=64, max_complexity=-1)
    assert g.info()["levels"] >= 3
    _, Rm = dense_R(eg)
    rng = np.random.default_rng(W)
    npairs = 3 * W + 7 if W > 1 else 9  # several blocks and a ragged tail
    s = rng.integers(0, eg.n, npairs)
    t = rng.integers(0, eg.n, npairs)
    t[0] = s[0]  # e_v - e_v = 0
    for prec, tol, rt in [(0, 1e-8, 1e-7), (1, 1e-10, 1e-9)]:
        r, st = g.resistance(s, t, block=W, precision=prec, tol=tol, stats=True)
        assert st["block_width"] == W and st["converged"] == npairs
        np.testing.assert_allclose(r, Rm[s, t], rtol=rt, atol=1e-12)
        assert r[0] == 0.0


def hub_graph(seed=21):
    """Random weighted graph plus three hubs adjacent to most nodes (rows far
    above the heavy-row degree threshold at several levels)."""
    base = synth.random_connected(3000, 9000, seed=seed)
    rng = np.random.default_rng(seed)
    u = [base.u]
    v = [base.v]
    for h, cnt in [(7, 2500), (1500, 1800), (2999, 700)]:
        nb = rng.choice(np.setdiff1d(np.arange(3000), [h]), cnt, replace=False)
        u.append(np.full(cnt, h))
        v.append(nb)
    u = np.concatenate(u)
    v = np.concatenate(v)
    lo, hi = np.minimum(u, v), np.maximum(u, v)
    key = np.unique(lo * 3000 + hi)
    w = rng.uniform(1.0, 4.0, key.shape[0])
    return synth.EdgeList(3000, key // 3000, key % 3000, w, "hubs")


@pytest.mark.parametrize("W,depth", [(64, 1), (256, 2), (512, 0), (32, 3)])
def test_heavy_rows(ctx, W, depth):
    eg = hub_graph()
    say("heavy rows", W, depth, eg.n, eg.m)
    g = load(ctx, eg, coarsest_max=64, max_complexity=-1)
    Lp, Rm = dense_R(eg)
    rng = np.random.default_rng(W)
    s = rng.integers(0, eg.n, W + 5)
    t = rng.integers(0, eg.n, W + 5)
    s[:3] = [7, 1500, 2999]
    for prec, tol, rt in [(0, 1e-8, 1e-7), (1, 1e-10, 1e-9)]:
        r = g.resistance(s, t, block=W, precision=prec, tol=tol, levels=depth, max_inner=2000)
        np.testing.assert_allclose(r, Rm[s, t], rtol=rt, atol=1e-12)
    g.jl_sketch(40, seed=3, tol=1e-9, block=W, levels=depth, max_inner=2000)
    nodes = np.array([7, 1500, 2999, 11])
    far, _ = g.farness_jl(nodes)
    of, _, _ = E.projection(None, eg, nodes, 40, 3, solver="dense", Lp=Lp)
    np.testing.assert_allclose(far, of, rtol=1e-6)


@pytest.mark.parametrize("maker", [
    lambda: synth.grid(40),
    lambda: synth.road_grid(60, seed=8),
    lambda: synth.barabasi_albert(3000, 4, seed=2),
    lambda: synth.rmat(11, seed=3),
    lambda: synth.star_graph(1500),
    lambda: leafy_graph(seed=9),
])
def test_device_aggregation(ctx, maker):
    """device = 2: the aggregation pass runs on the GPU (handshake matching).
    Every aggregation level is a partition into contiguous row ranges, the
    next level is P^T L P with zero row sums, the build is deterministic, and
    the full-depth cycle gives the oracle's resistances."""
    from tests.test_host import _check_elimination_level, _level_laplacian
    eg = maker()
    say("device aggregation", eg.n, eg.m)
    g = load(ctx, eg, coarsest_max=64, device=2, max_complexity=-1, eliminate=2)
    info = g.info()
    L = info["levels"]
    assert L >= 2 and info["level_n"][-1] <= 64
    for l in range(L - 1):
        lv, nxt = g.level(l), g.level(l + 1)
        if lv["elimination"]:
            _check_elimination_level(lv, nxt)
            continue
        agg, ap = lv["agg"], lv["agg_ptr"]
        assert ap[0] == 0 and ap[-1] == lv["n"] and np.all(np.diff(ap) >= 1)
        assert np.all(np.diff(agg) >= 0)
        Lf = _level_laplacian(lv)
        P = np.zeros((lv["n"], lv["n_coarse"]))
        P[np.arange(lv["n"]), agg] = 1.0
        Lc = _level_laplacian(nxt)
        np.testing.assert_allclose(P.T @ Lf @ P, Lc, atol=1e-9 * max(1.0, np.abs(Lc).max()))
        np.testing.assert_allclose(Lc.sum(axis=1), 0, atol=1e-9 * max(1.0, np.abs(Lc).max()))
    g2 = load(ctx, eg, coarsest_max=64, device=2, max_complexity=-1, eliminate=2)
    assert g2.info()["level_n"] == info["level_n"] and g2.info()["level_nnz"] == info["level_nnz"]
    _, Rm = dense_R(eg)
    rng = np.random.default_rng(7)
    s = rng.integers(0, eg.n, 70)
    t = rng.integers(0, eg.n, 70)
    r, st = g.resistance(s, t, block=64, tol=1e-9, levels=0, stats=True, max_inner=3000)
    say("  levels", info["level_n"], "iters", st["inner_iters"])
    np.testing.assert_allclose(r, Rm[s, t], rtol=1e-8, atol=1e-12)


def test_budget_truncated_hierarchy(ctx):
    """Under the default complexity budget a Barabasi-Albert graph (without
    an elimination level) keeps one aggregation level of more than 4096
    nodes and no exact coarsest solve: the full-depth cycle ends there with a
    Jacobi step, and every depth still gives the oracle's resistances."""
    eg = synth.barabasi_albert(15000, 4, seed=12)
    g = load(ctx, eg, coarsest_max=64, eliminate=0)
    info = g.info()
    say("budget", info["levels"], info["level_n"], info["operator_complexity"])
    assert info["operator_complexity"] <= 2.0 and info["level_n"][-1] > 4096
    assert g.level(info["levels"] - 1)["coarse_pinv"] is None
    rng = np.random.default_rng(5)
    s = rng.integers(0, eg.n, 70)
    t = rng.integers(0, eg.n, 70)
    want = R.resistance_cg(LAP.of(eg), s, t, tol=1e-12)
    for depth in (1, 2, 0):
        for prec, tol, rt in [(0, 1e-8, 1e-7), (1, 1e-10, 1e-9)]:
            r, st = g.resistance(s, t, block=64, precision=prec, tol=tol, levels=depth, stats=True)
            say("  depth", depth, prec, st["levels_used"], st["inner_iters"])
            np.testing.assert_allclose(r, want, rtol=rt, atol=1e-12)


@pytest.mark.parametrize("depth", [1, 2, 3, 0])
def test_vcycle_depths(ctx, depth):
    """Every V-cycle depth (1 = Jacobi-PCG, truncated cycles, full with the
    exact coarsest solve, 0 = autotuned) solves to the same resistances."""
    eg = synth.road_grid(60, seed=3)
    say("depth", depth, eg.n, eg.m)
    g = load(ctx, eg, coarsest_max=64)
    nlev = g.info()["levels"]
    assert nlev >= 4
    _, Rm = dense_R(eg)
    rng = np.random.default_rng(depth)
    s = rng.integers(0, eg.n, 70)
    t = rng.integers(0, eg.n, 70)
    for prec, tol, rt in [(0, 1e-8, 1e-7), (1, 1e-10, 1e-9)]:
        r, st = g.resistance(s, t, block=64, precision=prec, tol=tol, levels=depth, stats=True,
                             max_inner=3000)
        assert st["levels_used"] == (depth if depth else st["levels_used"]) and st["levels_used"] >= 1
        np.testing.assert_allclose(r, Rm[s, t], rtol=rt, atol=1e-12)


@pytest.mark.parametrize("maker,name", [
    (lambda: synth.path_graph(300), "path"),
    (lambda: synth.cycle_graph(301), "cycle"),
    (lambda: synth.star_graph(3000), "star"),
    (lambda: synth.complete_graph(80), "K80"),
])
def test_closed_forms(ctx, maker, name):
    eg = maker()
    say("closed form", name, eg.n, eg.m)
    g = load(ctx, eg, coarsest_max=32)
    n = eg.n
    s = np.array([0, 1, n // 2, n - 1, 5])
    t = np.array([n - 1, 2, 3, 0, 5])
    r = g.resistance(s, t, tol=1e-9, block=64)
    if name == "path":
        want = np.abs(s - t).astype(float)
    elif name == "cycle":
        d = np.abs(s - t)
        want = d * (n - d) / n
    elif name == "star":
        want = np.where(s == t, 0.0, np.where((s == 0) | (t == 0), 1.0, 2.0))
    else:
        want = np.where(s == t, 0.0, 2.0 / n)
    np.testing.assert_allclose(r, want, rtol=1e-7, atol=1e-12)


def test_exact_farness_grid32_fp64(ctx):
    """Plain method on the 32 x 32 grid: 1023 solves to 1e-10 (FP64)."""
    from tests.test_oracle_pins import grid_spectral_farness
    eg = synth.grid(32)
    g = load(ctx, eg)
    want = grid_spectral_farness(32, 0, 0)
    far, clo, st = g.farness_exact([0], precision=1, tol=1e-10, block=256, stats=True)
    say("exact 32x32", far, st)
    assert abs(far[0] / want - 1) < 1e-9
    assert abs(clo[0] - 1023 / want) < 1e-9 * clo[0]
    far2, _ = g.farness_exact([0, 528], tol=1e-10)  # mixed precision refined to 1e-10
    Lp, _ = dense_R(eg)
    np.testing.assert_allclose(far2, R.farness_dense(Lp, [0, 528]), rtol=1e-9)


def test_solve_dense_matches_pinv(ctx):
    import torch
    eg = synth.barabasi_albert(4000, 4, seed=7)
    g = load(ctx, eg)
    Lp, _ = dense_R(eg)
    rng = np.random.default_rng(3)
    B = rng.standard_normal((70, eg.n))
    B -= B.mean(axis=1, keepdims=True)
    X, st, status = g.solve(B, stats=True, tol=1e-8)
    say("dense solve", st)
    want = (Lp @ B.T).T
    assert np.all(status == 0)
    np.testing.assert_allclose(X, want, atol=1e-7 * np.abs(want).max())
    np.testing.assert_allclose(X.sum(axis=1), 0, atol=1e-9)
    # device tensors in, device tensors out
    Bt = torch.tensor(B[:5], device="cuda")
    Xt = g.solve(Bt, tol=1e-8)
    assert Xt.is_cuda
    np.testing.assert_allclose(Xt.cpu().numpy(), want[:5], atol=1e-7 * np.abs(want).max())
    # residual certificate with the oracle's operator
    Ls = LAP.of(eg)
    res = np.linalg.norm(B.T - Ls @ X.T, axis=0) / np.linalg.norm(B.T, axis=0)
    assert res.max() <= 1e-8 * 1.01


def test_sampling_matches_oracle_same_seed(ctx):
    eg = synth.barabasi_albert(5000, 4, seed=11)
    nodes = synth.query_nodes(eg.n, 6, seed=2)
    g = load(ctx, eg)
    far, clo, st = g.farness_sampling(nodes, k=60, seed=9, stats=True, tol=1e-8)
    say("sampling", st)
    of, oc, piv, d = E.sampling(LAP.of(eg), eg, nodes, 60, 9, tol=1e-12)
    np.testing.assert_allclose(far, of, rtol=1e-6)
    np.testing.assert_allclose(clo, oc, rtol=1e-6)


def test_projection_matches_oracle_same_seed(ctx):
    eg = synth.random_connected(2500, 9000, seed=13)
    nodes = synth.query_nodes(eg.n, 10, seed=3)
    g = load(ctx, eg)
    st = g.jl_sketch(96, seed=5, stats=True, tol=1e-9, block=64)
    say("jl", st)
    far, clo = g.farness_jl(nodes)
    of, oc, Z = E.projection(LAP.of(eg), eg, nodes, 96, 5, tol=1e-12)
    np.testing.assert_allclose(far, of, rtol=1e-6)
    np.testing.assert_allclose(clo, oc, rtol=1e-6)


@pytest.mark.parametrize("W,depth", [(64, 0), (256, 1), (32, 2)])
def test_graph_replay_matches_eager(ctx, W, depth):
    """PCG iterations replayed from a captured HIP graph give the same
    resistances as eager launches (and as the oracle)."""
    eg = synth.road_grid(40, seed=8)
    g = load(ctx, eg, coarsest_max=64)
    _, Rm = dense_R(eg)
    rng = np.random.default_rng(W)
    s = rng.integers(0, eg.n, 2 * W + 3)
    t = rng.integers(0, eg.n, 2 * W + 3)
    for prec, tol in [(0, 1e-8), (1, 1e-10)]:
        kw = dict(block=W, precision=prec, tol=tol, levels=depth, max_inner=3000)
        r_e = g.resistance(s, t, **kw)
        r_g = g.resistance(s, t, use_graph=1, **kw)
        np.testing.assert_allclose(r_g, r_e, rtol=10 * tol)
        np.testing.assert_allclose(r_g, Rm[s, t], rtol=10 * tol, atol=1e-12)


@pytest.mark.parametrize("device", [False, True])
def test_solve_dense_blocks_and_checks(ctx, device):
    """Several column blocks with a ragged tail, host or device buffers; a
    column that is not finite or does not sum to zero is rejected."""
    import torch
    import paper_1607_02955_amd as cfc
    eg = synth.random_connected(1500, 4500, seed=17)
    g = load(ctx, eg, coarsest_max=64)
    Lp, _ = dense_R(eg)
    rng = np.random.default_rng(5)
    B = rng.standard_normal((75, eg.n)) * rng.uniform(0.1, 100, (75, 1))
    B -= B.mean(axis=1, keepdims=True)
    want = (Lp @ B.T).T
    wrap = (lambda a: torch.tensor(a, device="cuda")) if device else (lambda a: a)
    unwrap = (lambda t: t.cpu().numpy()) if device else (lambda t: t)
    X = unwrap(g.solve(wrap(B), tol=1e-9, block=32))
    np.testing.assert_allclose(X, want, atol=1e-8 * np.abs(want).max())
    assert np.all(np.abs(X.sum(axis=1)) <= 1e-12 * np.abs(X).sum(axis=1))
    for bad in (np.nan, np.inf):
        Bb = B.copy()
        Bb[40, 7] = bad
        with pytest.raises(cfc.CfcError, match="not finite"):
            g.solve(wrap(Bb), tol=1e-9, block=32)
    Bb = B.copy()
    Bb[74, 3] += 1e-6 * np.abs(Bb[74]).sum()
    with pytest.raises(cfc.CfcError, match="sum to zero"):
        g.solve(wrap(Bb), tol=1e-9, block=32)


def test_edge_cases(ctx):
    import paper_1607_02955_amd as cfc
    g1 = cfc.Graph(ctx, 1, [], [])
    g1.build_hierarchy()
    assert g1.resistance([0], [0])[0] == 0.0
    g2 = cfc.Graph(ctx, 2, [0], [1], [4.0]).build_hierarchy()
    np.testing.assert_allclose(g2.resistance([0, 1], [1, 0], tol=1e-10), [0.25, 0.25], rtol=1e-10)
    far, clo = g2.farness_exact([0], tol=1e-10)
    np.testing.assert_allclose(far, [0.25], rtol=1e-10)
    with pytest.raises(cfc.CfcError):
        g2.resistance([0], [2])
    with pytest.raises(cfc.CfcError):
        g2.solve(np.array([1.0, 0.0]))  # does not sum to zero
    # dense solves at the smallest sizes: one node (only b = 0), two nodes,
    # no right-hand sides
    np.testing.assert_array_equal(g1.solve(np.zeros((3, 1)), tol=1e-10), np.zeros((3, 1)))
    np.testing.assert_allclose(g2.solve(np.array([[1.0, -1.0]]), tol=1e-10), [[0.125, -0.125]],
                               rtol=1e-9)
    assert g2.solve(np.zeros((0, 2))).shape == (0, 2)
    with pytest.raises(cfc.CfcError, match="STATE"):
        g2.farness_jl([0])


def leafy_graph(seed=31, n=3000):
    """Weighted random graph with many degree-1 and degree-2 nodes (pendant
    trees and chains hung on a core), like the low-degree fringe of
    skewed-degree networks."""
    core = synth.random_connected(n // 2, 3 * n // 2, seed=seed)
    rng = np.random.default_rng(seed)
    a, b, w = [core.u], [core.v], [core.w]
    nxt = core.n
    for _ in range(n // 2):
        kind = rng.integers(0, 3)
        anchor = int(rng.integers(0, nxt))
        if kind == 0:    # leaf
            a.append([anchor]); b.append([nxt]); nxt += 1
        elif kind == 1:  # chain of two
            a.append([anchor, nxt]); b.append([nxt, nxt + 1]); nxt += 2
        else:            # degree-2 bridge between two core nodes
            other = int(rng.integers(0, core.n))
            if other == anchor:
                continue
            a.append([anchor, nxt]); b.append([nxt, other]); nxt += 1
        w.append(rng.uniform(1, 4, len(a[-1])))
    a, b, w = np.concatenate(a), np.concatenate(b), np.concatenate(w)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key, first = np.unique(lo * nxt + hi, return_index=True)
    return synth.EdgeList(nxt, key // nxt, key % nxt, w[first])


@pytest.mark.parametrize("W,prec", [(64, 0), (256, 1), (32, 0)])
def test_elimination_level_all_depths(ctx, W, prec):
    """An elimination level (exact Schur complement of an independent set of
    nodes of degree 1 to 4) in front of the aggregation levels: every V-cycle depth
    and the full exact path give the oracle's resistances."""
    eg = leafy_graph(seed=W)
    say("elimination", W, prec, eg.n, eg.m)
    g = load(ctx, eg, coarsest_max=64, eliminate=2, max_complexity=-1)
    info = g.info()
    assert info["eliminated"] > eg.n // 10 and info["levels"] >= 4
    _, Rm = dense_R(eg)
    rng = np.random.default_rng(W)
    s = rng.integers(0, eg.n, 2 * W + 5)
    t = rng.integers(0, eg.n, 2 * W + 5)
    tol = 1e-8 if prec == 0 else 1e-10
    for depth in (1, 2, 3, 0):
        r, st = g.resistance(s, t, block=W, precision=prec, tol=tol, levels=depth, stats=True,
                             max_inner=3000)
        say("  depth", depth, st["inner_iters"], st["levels_used"])
        np.testing.assert_allclose(r, Rm[s, t], rtol=10 * tol, atol=1e-12)
    r_g = g.resistance(s, t, block=W, precision=prec, tol=tol, levels=2, use_graph=1, max_inner=3000)
    np.testing.assert_allclose(r_g, Rm[s, t], rtol=10 * tol, atol=1e-12)


@pytest.mark.parametrize("W", [64, 256])
def test_schur_cg_matches_level0_cg(ctx, W, monkeypatch):
    """An elimination level with one Jacobi step or a V-cycle behind it: CG
    on the Schur complement (the residual folded onto the kept rows, the
    eliminated rows back-substituted) and CG on level 0 with the elimination
    inside the preconditioner give the oracle's resistances in about as
    many iterations, also on an R-MAT graph whose hubs are heavy rows of the
    Schur complement, on a road grid whose degree-3 and degree-4 nodes are
    eliminated (fill between their neighbours), and with the iterations
    replayed from a HIP graph."""
    for name, eg in [("leafy", leafy_graph(seed=W + 1)), ("rmat", synth.rmat(11, seed=W)),
                     ("road", synth.road_grid(40, seed=W))]:
        g = load(ctx, eg, coarsest_max=64, eliminate=2, max_complexity=-1)
        lv0 = g.level(0)
        assert g.info()["eliminated"] > 0
        if name == "road":
            assert (lv0["elim_nb"] >= 0).sum(axis=1).max() == 4
        _, Rm = dense_R(eg)
        rng = np.random.default_rng(W)
        s = rng.integers(0, eg.n, 2 * W + 5)
        t = rng.integers(0, eg.n, 2 * W + 5)
        for depth in (2, 3, 0):
            its = {}
            for mode in ("1", "0"):
                monkeypatch.setenv("CFC_SCHUR", mode)
                for graph in (0, 1):
                    r, st = g.resistance(s, t, block=W, tol=1e-8, levels=depth, use_graph=graph,
                                         stats=True, max_inner=3000)
                    say("schur", name, W, depth, mode, graph, st["inner_iters"], st["refine_steps"],
                        st["max_rel_residual"])
                    np.testing.assert_allclose(r, Rm[s, t], rtol=1e-7, atol=1e-12)
                    its[mode, graph] = st["inner_iters"]
            assert its["1", 0] <= 1.25 * its["0", 0] + 4, its


@pytest.mark.parametrize("case", ["depth1_hubs", "elim_depth2"])
def test_bf16_z_matches_fp32_z(ctx, case, monkeypatch):
    """The bfloat16 and the FP8 copies of z = M^-1 r (depth one, or
    elimination plus one Jacobi step) give the oracle's resistances at the
    requested tolerance, as the FP32 z does, in about as many iterations."""
    if case == "depth1_hubs":
        eg = synth.barabasi_albert(3000, 3, seed=44)  # hubs above the heavy-row threshold
        g = load(ctx, eg, coarsest_max=64)
        depth, W = 1, 256
    else:
        eg = leafy_graph(seed=45)
        g = load(ctx, eg, coarsest_max=64, eliminate=2, max_complexity=-1)
        assert g.info()["eliminated"] > 0 and g.info()["levels"] >= 3
        depth, W = 2, 64
    _, Rm = dense_R(eg)
    rng = np.random.default_rng(9)
    s = rng.integers(0, eg.n, 2 * W + 3)
    t = rng.integers(0, eg.n, 2 * W + 3)
    its, res = {}, {}
    # (compressed z, FP8 rather than bfloat16, x updates in the product
    # kernel): FP32 z; bfloat16 z; FP8 z; FP8 z with fused x updates
    for bz, z8, fx, zf in (("0", "0", "0", 0), ("1", "0", "0", 1), ("1", "1", "0", 2), ("1", "1", "1", 2)):
        monkeypatch.setenv("CFC_BF16_Z", bz)
        monkeypatch.setenv("CFC_Z_FP8", z8)
        monkeypatch.setenv("CFC_FUSE_X", fx)
        r, st = g.resistance(s, t, block=W, tol=1e-8, levels=depth, stats=True, max_inner=3000)
        say("z format", case, st["z_format"], "fused x", fx, st["inner_iters"], st["refine_steps"])
        assert st["z_format"] == zf
        np.testing.assert_allclose(r, Rm[s, t], rtol=1e-7, atol=1e-12)
        its[bz + z8 + fx], res[bz + z8 + fx] = st["inner_iters"], r
    assert its["100"] <= 1.1 * its["000"] + 3
    assert its["110"] <= 1.1 * its["000"] + 3
    # carrying x in the product kernel is the same arithmetic (only the
    # order of the column sums of x may differ)
    assert its["111"] == its["110"]
    np.testing.assert_allclose(res["111"], res["110"], rtol=1e-12, atol=1e-15)


def test_pair_differences_without_x64(ctx):
    """Pair solves in FP32 Schur mode add x[s] - x[t] per refinement step
    instead of forming the mean-zero x64: the result equals the difference
    taken from full solves of the same right-hand sides (dense path), and
    the oracle's resistances, over several refinement steps and with a pair
    whose ends coincide (resistance 0)."""
    eg = leafy_graph(seed=77)
    g = load(ctx, eg, coarsest_max=64, eliminate=2, max_complexity=-1)
    assert g.info()["eliminated"] > 0
    _, Rm = dense_R(eg)
    rng = np.random.default_rng(77)
    s = rng.integers(0, eg.n, 70)
    t = rng.integers(0, eg.n, 70)
    t[5] = s[5]
    for depth in (2, 0):
        r, st = g.resistance(s, t, block=64, tol=1e-9, levels=depth, stats=True)
        say("pair acc", depth, st["refine_steps"], st["inner_iters"], st["max_rel_residual"])
        assert st["refine_steps"] >= 2 * st["blocks"]  # more than one refinement step per block
        np.testing.assert_allclose(r, Rm[s, t], rtol=1e-8, atol=1e-12)
        assert r[5] == 0.0
        B = np.zeros((len(s), eg.n))
        B[np.arange(len(s)), s] += 1.0
        B[np.arange(len(s)), t] -= 1.0
        X = g.solve(B, block=64, tol=1e-9, levels=depth)
        np.testing.assert_allclose(r, X[np.arange(len(s)), s] - X[np.arange(len(s)), t], rtol=1e-7, atol=1e-12)


def test_elimination_to_two_nodes_is_exact(ctx):
    """A star loses every leaf but one: the elimination level over a two-node
    coarsest level is an exact solver."""
    eg = synth.star_graph(1500)
    g = load(ctx, eg, coarsest_max=64, eliminate=1)
    assert g.info()["level_n"] == [1500, 2]
    s = np.arange(1, 200)
    t = np.arange(2, 201) % 1500
    r, st = g.resistance(s, t, block=256, precision=1, tol=1e-12, stats=True)
    np.testing.assert_allclose(r, np.where(s == t, 0.0, 2.0), rtol=1e-12)
    assert st["inner_iters"] <= 3 * st["blocks"]


@pytest.mark.parametrize("maker", [
    lambda: synth.grid(60),
    lambda: synth.barabasi_albert(6000, 4, seed=3),
    lambda: synth.rmat(13, seed=5),
    lambda: synth.road_grid(70, seed=6),
    lambda: leafy_graph(seed=9),
    lambda: synth.star_graph(3000),
])
def test_device_setup_equals_host_setup(ctx, maker):
    """The device build (affinities, Galerkin products, renumbering on the
    GPU) gives the host build's hierarchy bit for bit."""
    import paper_1607_02955_amd as cfc
    eg = maker()
    say("device setup", eg.name, eg.n, eg.m)
    gh = cfc.Graph.from_edgelist(ctx, eg)
    gh.build_hierarchy(coarsest_max=64, device=0)
    gd = cfc.Graph.from_edgelist(ctx, eg)
    gd.build_hierarchy(coarsest_max=64, device=1)
    ih, idv = gh.info(), gd.info()
    assert ih["level_n"] == idv["level_n"] and ih["level_nnz"] == idv["level_nnz"]
    assert ih["eliminated"] == idv["eliminated"]
    for l in range(ih["levels"]):
        a, b = gh.level(l), gd.level(l)
        for k in ("row_ptr", "col", "agg", "agg_ptr", "perm", "elim_nb"):
            if a[k] is None:
                assert b[k] is None, (l, k)
            else:
                assert np.array_equal(a[k], b[k]), (l, k)
        for k in ("w", "deg", "coarse_pinv"):
            if a[k] is not None:
                assert np.array_equal(a[k].view(np.uint64), b[k].view(np.uint64)), (l, k)
    s = np.arange(0, eg.n, max(1, eg.n // 50))
    t = (s * 7 + 1) % eg.n
    np.testing.assert_array_equal(gh.resistance(s, t, block=64, levels=2),
                                  gd.resistance(s, t, block=64, levels=2))
