"""CPU tests of the library's host side (no GPU): exports, graph ingest,
hierarchy invariants, and the counter-based draws against the oracle's."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import laplacian as LAP
from oracle import resistance as R
from oracle import rng as ORNG

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfc.h")

cfc = pytest.importorskip("paper_1607_02955_amd")
from paper_1607_02955_amd import _lib  # noqa: E402


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(cfc_\w+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 25
    L = C.CDLL(_lib.LIB_PATH)
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)
    _lib.lib()  # binds every signature


@pytest.fixture(scope="module")
def hctx():
    return cfc.Context(device=-1)


def test_ingest_errors(hctx):
    with pytest.raises(cfc.CfcError, match="INVALID"):
        cfc.Graph(hctx, 3, [0, 1], [1, 3])
    with pytest.raises(cfc.CfcError, match="INVALID"):
        cfc.Graph(hctx, 3, [0, 1], [1, 2], [1.0, float("nan")])
    with pytest.raises(cfc.CfcError, match="INVALID"):
        cfc.Graph(hctx, 3, [0, 1], [1, 2], [1.0, 0.0])
    with pytest.raises(cfc.CfcError, match="INVALID"):
        cfc.Graph(hctx, 3, [0, 1], [1, 2], [1.0, -2.0])
    with pytest.raises(cfc.CfcError, match="DISCONNECTED"):
        cfc.Graph(hctx, 4, [0, 2], [1, 3])
    with pytest.raises(cfc.CfcError, match="INVALID"):
        cfc.Graph(hctx, 3, [0, 1, 1], [1, 2, 0], flags=cfc.REJECT_PARALLEL)
    with pytest.raises(cfc.CfcError, match="INVALID"):
        cfc.Graph(hctx, 0, [], [])


def test_ingest_canonicalises(hctx):
    # self-loop dropped, parallel edges summed, orientation ignored
    g = cfc.Graph(hctx, 3, [0, 1, 1, 2, 2], [1, 0, 2, 2, 1], [1.0, 2.0, 0.5, 9.0, 0.25])
    assert g.n == 3 and g.m == 2
    g.build_hierarchy()
    lv = g.level(0)
    L = np.zeros((3, 3))
    perm = lv["perm"]
    for r in range(3):
        for e in range(lv["row_ptr"][r], lv["row_ptr"][r + 1]):
            L[r, lv["col"][e]] = -lv["w"][e]
        L[r, r] = lv["deg"][r]
    Lg = L[np.ix_(perm, perm)]  # back to graph numbering
    np.testing.assert_allclose(Lg, [[3, -3, 0], [-3, 3.75, -0.75], [0, -0.75, 0.75]])


def test_lcc_only_relabels(hctx):
    # components {0,2,5} (largest), {1,3}, {4}
    g = cfc.Graph(hctx, 6, [0, 2, 1], [2, 5, 3], flags=cfc.LCC_ONLY)
    assert g.n == 3 and g.m == 2
    np.testing.assert_array_equal(g.node_map(), [0, 2, 5])
    assert g.info()["input_n"] == 6


def _level_laplacian(lv):
    n = lv["n"]
    L = np.zeros((n, n))
    for r in range(n):
        for e in range(lv["row_ptr"][r], lv["row_ptr"][r + 1]):
            L[r, lv["col"][e]] -= lv["w"][e]
        L[r, r] += lv["deg"][r]
    return L


def _check_elimination_level(lv, nxt, max_degree=4):
    """Kept rows first; eliminated rows form an independent set of degree 1
    to 4; the next level is the Schur complement on the kept rows."""
    n, nc = lv["n"], lv["n_coarse"]
    assert l_ok(nc, n) and nxt["n"] == nc
    Lf = _level_laplacian(lv)
    F = np.arange(nc, n)
    LFF = Lf[np.ix_(F, F)]
    np.testing.assert_allclose(LFF, np.diag(np.diag(LFF)), atol=0)  # independent set
    deg = np.diff(lv["row_ptr"])[F]
    assert deg.min() >= 1 and deg.max() <= max_degree
    nb = lv["elim_nb"]
    assert nb.shape == (n - nc, 4)
    for i, r in enumerate(F):
        got = [x for x in nb[i] if x >= 0]
        assert nb[i].tolist() == got + [-1] * (4 - len(got))  # neighbours first, then -1
        assert got == sorted(lv["col"][lv["row_ptr"][r]:lv["row_ptr"][r + 1]].tolist())
        assert max(got) < nc
    C = np.arange(nc)
    S = Lf[np.ix_(C, C)] - Lf[np.ix_(C, F)] @ np.linalg.solve(LFF, Lf[np.ix_(F, C)])
    Lc = _level_laplacian(nxt)
    np.testing.assert_allclose(S, Lc, atol=1e-11 * max(1.0, np.abs(Lc).max()))


def l_ok(nc, n):
    return 2 <= nc < n


@pytest.mark.parametrize("maker", [
    lambda: synth.grid(40),
    lambda: synth.barabasi_albert(3000, 4, seed=2),
    lambda: synth.rmat(11, seed=3),
    lambda: synth.road_grid(48, seed=4),
    lambda: synth.star_graph(2000),
    lambda: synth.random_connected(1500, 2200, seed=9),
])
@pytest.mark.parametrize("elim,elim_degree", [(0, 0), (2, 2), (2, 0)], ids=["noelim", "deg2", "deg4"])
def test_hierarchy_invariants(hctx, maker, elim, elim_degree):
    eg = maker()
    g = cfc.Graph.from_edgelist(hctx, eg)
    g.build_hierarchy(coarsest_max=128, eliminate=elim, elim_degree=elim_degree,
                      max_complexity=-1)  # every level
    info = g.info()
    L = info["levels"]
    assert L >= 2 and info["level_n"][-1] <= 128
    assert all(info["level_n"][i + 1] < info["level_n"][i] for i in range(L - 1))
    lv0 = g.level(0)
    assert sorted(lv0["perm"].tolist()) == list(range(eg.n))
    # level 0 is the input Laplacian, permuted
    Lin = LAP.of(eg).toarray()
    p = lv0["perm"]
    L0 = _level_laplacian(lv0)
    np.testing.assert_allclose(L0[np.ix_(p, p)], Lin, atol=1e-12)
    for l in range(L - 1):
        lv = g.level(l)
        nxt = g.level(l + 1)
        if lv["elimination"]:
            _check_elimination_level(lv, nxt, elim_degree or 4)
            continue
        agg, ap = lv["agg"], lv["agg_ptr"]
        assert ap[0] == 0 and ap[-1] == lv["n"] and np.all(np.diff(ap) >= 1)
        assert np.all(np.diff(agg) >= 0), "aggregates must be contiguous row ranges"
        for I in range(lv["n_coarse"]):
            assert np.all(agg[ap[I]:ap[I + 1]] == I)
        assert np.diff(ap).max() <= 8
        # Galerkin: coarse Laplacian == P^T L P
        Lf = _level_laplacian(lv)
        P = np.zeros((lv["n"], lv["n_coarse"]))
        P[np.arange(lv["n"]), agg] = 1.0
        Lc = _level_laplacian(nxt)
        np.testing.assert_allclose(P.T @ Lf @ P, Lc, atol=1e-9 * max(1.0, np.abs(Lc).max()))
        np.testing.assert_allclose(Lc.sum(axis=1), 0, atol=1e-9 * max(1.0, np.abs(Lc).max()))
    last = g.level(L - 1)
    Lc = _level_laplacian(last)
    Pc = last["coarse_pinv"]
    np.testing.assert_allclose(Pc, Pc.T, atol=1e-10)
    np.testing.assert_allclose(Lc @ Pc @ Lc, Lc, atol=1e-8 * np.abs(Lc).max())
    np.testing.assert_allclose(Pc.sum(axis=1), 0, atol=1e-9)
    np.testing.assert_allclose(Pc, R.pinv(Lc), atol=1e-8 * max(1.0, np.abs(Pc).max()))


def _budget_complexity(g):
    """sum_l (nnz_l + n_l) over the aggregation levels, in units of the first
    aggregated level (level 1 behind an elimination level)."""
    info = g.info()
    a = 1 if info["levels"] > 1 and g.level(0)["elimination"] else 0
    u = [info["level_nnz"][l] + info["level_n"][l] for l in range(info["levels"])]
    assert info["cycle_complexity"] == pytest.approx(sum(u[a:]) / u[a], rel=1e-12)
    ratios = [u[l + 1] / u[l] for l in range(a, info["levels"] - 1)]
    return sum(u[a:]) / u[a], ratios


def test_complexity_budget(hctx):
    """The default budget keeps the aggregation levels' complexity <= 2: on a
    Barabasi-Albert graph the quotient graphs keep almost every edge, so it
    stops after one aggregation level, above 4096 nodes here and so with no
    exact coarsest solve; a road grid coarsens as far as without a budget.
    Behind an elimination level the budget is counted from the Schur
    complement graph."""
    ba = synth.barabasi_albert(20000, 4, seed=3)
    full = cfc.Graph.from_edgelist(hctx, ba).build_hierarchy(coarsest_max=128, eliminate=0,
                                                             max_complexity=-1)
    assert full.info()["operator_complexity"] > 2.0
    g = cfc.Graph.from_edgelist(hctx, ba).build_hierarchy(coarsest_max=128, eliminate=0)
    info = g.info()
    assert info["operator_complexity"] <= 2.0 and 2 <= info["levels"] < full.info()["levels"]
    assert info["level_n"][-1] > 4096 and g.level(info["levels"] - 1)["coarse_pinv"] is None
    g = cfc.Graph.from_edgelist(hctx, ba).build_hierarchy(coarsest_max=128, eliminate=0, max_complexity=3.0)
    assert g.info()["operator_complexity"] <= 3.0
    # degree-4 nodes eliminated first (a third of this graph's nodes); the
    # quotient graph of their Schur complement keeps over 0.8 of its size,
    # so no aggregation level follows
    g = cfc.Graph.from_edgelist(hctx, ba).build_hierarchy(coarsest_max=128)
    assert g.level(0)["elimination"] and g.info()["levels"] == 2
    assert _budget_complexity(g) == (1.0, [])
    nob = cfc.Graph.from_edgelist(hctx, ba).build_hierarchy(coarsest_max=128, max_complexity=-1)
    assert _budget_complexity(nob)[1][0] > 0.8
    rd = synth.road_grid(100, seed=2)
    for elim in (0, 1):
        a = cfc.Graph.from_edgelist(hctx, rd).build_hierarchy(coarsest_max=64, eliminate=elim)
        b = cfc.Graph.from_edgelist(hctx, rd).build_hierarchy(coarsest_max=64, eliminate=elim,
                                                              max_complexity=-1)
        oc, ratios = _budget_complexity(a)
        assert a.info()["levels"] == b.info()["levels"] and oc <= 2.0 and max(ratios) <= 0.8
    with pytest.raises(cfc.CfcError, match="INVALID"):
        cfc.Graph.from_edgelist(hctx, rd).build_hierarchy(max_complexity=0.5)


def test_tiny_graph_single_level(hctx):
    g = cfc.Graph(hctx, 1, [], [])
    g.build_hierarchy()
    assert g.info()["levels"] == 1
    eg = synth.path_graph(5)
    g = cfc.Graph.from_edgelist(hctx, eg).build_hierarchy()
    lv = g.level(0)
    np.testing.assert_allclose(lv["coarse_pinv"], R.pinv(_level_laplacian(lv)), atol=1e-12)


def test_setup_param_errors_ranges(hctx):
    g = cfc.Graph.from_edgelist(hctx, synth.grid(8))
    with pytest.raises(cfc.CfcError):
        g.build_hierarchy(mu=2.5)
    with pytest.raises(cfc.CfcError):
        g.build_hierarchy(coarsest_max=100000)


def test_solve_needs_device(hctx):
    g = cfc.Graph.from_edgelist(hctx, synth.grid(8)).build_hierarchy()
    with pytest.raises(cfc.CfcError, match="STATE"):
        g.resistance([0], [5])


# ---- the library's draws equal the oracle's, bit for bit -------------------

@pytest.mark.parametrize("n,k", [(10, 3), (1000, 20), (50, 50), (100000, 1000), (7, 100)])
def test_sampling_pivots_match_oracle(n, k):
    for seed in (1, 2, 12345678901):
        for node in (0, n // 3, n - 1):
            got = cfc.sampling_pivots(seed, node, n, k).tolist()
            assert got == ORNG.pivots(seed, node, n, k)


def test_jl_sign_words_match_oracle():
    rng = np.random.default_rng(0)
    for _ in range(200):
        lo = int(rng.integers(0, 2**31 - 2))
        hi = int(rng.integers(lo + 1, 2**31 - 1))
        seed = int(rng.integers(0, 2**63))
        word = int(rng.integers(0, 64))
        assert cfc.jl_sign_word(seed, word, lo, hi) == ORNG.hash4(seed, ORNG.TAG_JL, word, (lo << 32) | hi)


@pytest.mark.parametrize("n,k", [(1, 1), (10, 3), (1000, 1000), (100000, 512)])
def test_shared_pivots_match_oracle(n, k):
    for seed in (1, 7, 2**63 + 5):
        assert cfc.shared_pivots(seed, n, k).tolist() == ORNG.shared_pivots(seed, n, k)


def test_random_pairs_match_oracle():
    for seed, n in ((1, 2), (3, 17), (99, 1000003)):
        s, t = cfc.random_pairs(seed, n, 300)
        so, to = ORNG.random_pairs(seed, n, 300)
        assert s.tolist() == so.tolist() and t.tolist() == to.tolist()


@pytest.mark.parametrize("order", [1, 2, 3])
def test_locality_orders_give_valid_nested_hierarchies(hctx, order):
    """Every locality order yields a permutation of the nodes with contiguous
    aggregates, and the same level sizes (the order only renumbers)."""
    eg = synth.barabasi_albert(2500, 4, seed=4)
    ref = cfc.Graph.from_edgelist(hctx, eg).build_hierarchy(coarsest_max=64, order=1)
    g = cfc.Graph.from_edgelist(hctx, eg).build_hierarchy(coarsest_max=64, order=order)
    assert g.info()["level_n"] == ref.info()["level_n"]
    assert g.info()["level_nnz"] == ref.info()["level_nnz"]
    lv0 = g.level(0)
    assert sorted(lv0["perm"].tolist()) == list(range(eg.n))
    Lin = LAP.of(eg).toarray()
    p = lv0["perm"]
    np.testing.assert_allclose(_level_laplacian(lv0)[np.ix_(p, p)], Lin, atol=1e-12)
    for l in range(g.info()["levels"] - 1):
        lv = g.level(l)
        if not lv["elimination"]:
            assert np.all(np.diff(lv["agg"]) >= 0)
    if order == 3:  # hubs first: row 0 holds a node of maximum degree
        deg = np.diff(LAP.of(eg).indptr)
        assert deg[np.argsort(p)[0]] == deg.max()


@pytest.mark.parametrize("nest", [1, 2])
def test_nesting_depth_only_renumbers(hctx, nest):
    """Nesting the numbering through every aggregation level or through the
    kept levels only gives the same levels (sizes and entries), a valid
    permutation and contiguous aggregates; only the order differs."""
    eg = synth.barabasi_albert(1500, 4, seed=8)
    ref = cfc.Graph.from_edgelist(hctx, eg).build_hierarchy(coarsest_max=64, nest=0)
    g = cfc.Graph.from_edgelist(hctx, eg).build_hierarchy(coarsest_max=64, nest=nest)
    assert g.info()["level_n"] == ref.info()["level_n"]
    assert g.info()["level_nnz"] == ref.info()["level_nnz"]
    lv0 = g.level(0)
    p = lv0["perm"]
    assert sorted(p.tolist()) == list(range(eg.n))
    np.testing.assert_allclose(_level_laplacian(lv0)[np.ix_(p, p)], LAP.of(eg).toarray(), atol=1e-12)
    for l in range(g.info()["levels"] - 1):
        lv = g.level(l)
        if lv["elimination"]:
            _check_elimination_level(lv, g.level(l + 1))
        else:
            assert np.all(np.diff(lv["agg"]) >= 0)


def test_setup_param_errors_enums(hctx):
    eg = synth.path_graph(10)
    g = cfc.Graph.from_edgelist(hctx, eg)
    for kw in ({"order": 4}, {"eliminate": 3}, {"device": 3}, {"elim_degree": 5},
               {"elim_degree": -1}, {"nest": 3}, {"nest": -1}):
        with pytest.raises(cfc.CfcError):
            g.build_hierarchy(**kw)
