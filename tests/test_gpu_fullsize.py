"""Parity at the benchmark sizes, in the launch configuration bench.py times.

Expected values come from tests/golden/*.json, written by
tests/golden/make_golden.py from the CPU oracle, or from the oracle's closed
form for the undeleted 2048 x 2048 grid (oracle/spectral.py).  On the
2%-deleted road graph, properties that hold at any size are checked with the
oracle's operator as well.

The bar for the solve is <= 1e-6 relative error of every effective
resistance and farness at the benchmark tolerance (1e-6 relative residual);
estimator outputs with the same seed match the oracle's to <= 1e-4.  Where a
residual of 1e-6 does not imply 1e-6 in d_ER (d_ER(u, v) = b^T x has the error
-x^T r, bounded by ||x|| ||r||), the a-posteriori bound ||x|| ||r|| / b^T x is
printed beside the measured error.
"""
import json
import os
import sys

import numpy as np
import pytest

import synth
from oracle import laplacian as LAP
from oracle import spectral as SP

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_1607_02955_amd as cfc
    return cfc.Context(0)


def test_ba100k_projection_k512(ctx):
    import paper_1607_02955_amd as cfc
    gold = json.load(open(os.path.join(GOLD, "ba100k_jl512.json")))
    eg = synth.barabasi_albert(100000, 4, seed=1)
    g = cfc.Graph.from_edgelist(ctx, eg).build_hierarchy()
    st = g.jl_sketch(512, seed=1, block=512, tol=1e-6, stats=True)
    say("ba100k", st["levels_used"], st["inner_iters"], st["max_rel_residual"])
    far, clo = g.farness_jl(gold["nodes"])
    np.testing.assert_allclose(far, gold["farness"], rtol=1e-4)   # estimator match
    np.testing.assert_allclose(clo, gold["closeness"], rtol=1e-4)
    err = np.max(np.abs(far / np.array(gold["farness"]) - 1))
    say("ba100k max rel farness err", err)
    assert err <= 1e-6  # the solve itself to 1e-6 residual


def test_rmat20_pair_resistances(ctx):
    import paper_1607_02955_amd as cfc
    gold = json.load(open(os.path.join(GOLD, "rmat20_pairs.json")))
    eg = synth.rmat(20, 16, seed=1)
    g = cfc.Graph.from_edgelist(ctx, eg).build_hierarchy()
    # the block width of the benchmark's R-MAT-20 Sampling workload
    r, st = g.resistance(gold["s"], gold["t"], block=512, tol=1e-6, stats=True)
    say("rmat20", st["levels_used"], st["inner_iters"], r[:3], gold["resistance"][:3])
    np.testing.assert_allclose(r, gold["resistance"], rtol=1e-6)
    err = np.max(np.abs(r / np.array(gold["resistance"]) - 1))
    say("rmat20 max rel resistance err", err)
    # Sampling farness of two benchmark query nodes, k = 64, same seed
    gs = json.load(open(os.path.join(GOLD, "rmat20_sampling64.json")))
    far, clo, st = g.farness_sampling(gs["nodes"], 64, seed=1, block=512, tol=1e-6, stats=True)
    err = np.max(np.abs(far / np.array(gs["farness"]) - 1))
    say("rmat20 sampling64", st["columns"], st["max_rel_residual"], "max rel farness err", err)
    assert st["max_rel_residual"] <= 1e-6
    assert err <= 1e-6
    np.testing.assert_allclose(clo, gs["closeness"], rtol=1e-6)


def _pair_certificate(L, eg, X, s, t):
    """Measured d_ER from a dense solve and the bound ||x|| ||r|| / b^T x."""
    n = eg.n
    j = np.arange(len(s))
    B = np.zeros((n, len(s)))
    B[s, j] += 1.0
    B[t, j] -= 1.0
    Xt = X.T
    r = B - L @ Xt
    d = Xt[s, j] - Xt[t, j]
    cert = np.linalg.norm(Xt, axis=0) * np.linalg.norm(r, axis=0) / d
    res = np.linalg.norm(r, axis=0) / np.sqrt(2.0)
    return d, cert, res


@pytest.mark.parametrize("tol", [1e-6, 1e-8])
def test_grid2048_resistance_closed_form(ctx, tol):
    """The undeleted 2048 x 2048 grid (n = 4,194,304, the road graph's shape)
    through the full-depth cycle the autotuner picks for it, against the
    eigenbasis closed form."""
    import paper_1607_02955_amd as cfc
    N = 2048
    n = N * N
    print(f"case: grid2048 pair resistances at tol {tol:g}", flush=True)
    eg = synth.grid(N)
    g = cfc.Graph.from_edgelist(ctx, eg).build_hierarchy()
    s = np.array([0, 0, 0, 2047 * N + 5, 1024 * N + 1024, 1024 * N + 1024, 77 * N + 1900, 3000000])
    t = np.array([n - 1, N - 1, 1, N * N - 7, 1024 * N + 1025, 300 * N + 1700, 1990 * N + 12, 1234567])
    want = SP.grid_resistance(N, N, s, t)
    r, st = g.resistance(s, t, tol=tol, stats=True)
    err = np.abs(r / want - 1)
    say("grid2048", tol, st["levels_used"], st["block_width"], st["inner_iters"], st["max_rel_residual"])
    say("  closed form", want)
    say("  rel err", err)
    # C-9: the a-posteriori bound from a dense solve of the same pairs
    B = np.zeros((len(s), n))
    B[np.arange(len(s)), s] += 1.0
    B[np.arange(len(s)), t] -= 1.0
    X, st2, status = g.solve(B, tol=tol, stats=True)
    d, cert, res = _pair_certificate(LAP.of(eg), eg, X, s, t)
    say("  dense solve: rel err", np.abs(d / want - 1), "bound ||x|| ||r|| / b^T x", cert, "rel res", res)
    assert np.all(status == 0) and res.max() <= 1.01 * tol
    assert st["max_rel_residual"] <= tol
    assert err.max() <= 1e-6
    assert np.max(np.abs(d / want - 1)) <= 1e-6


def test_road2048_properties(ctx):
    import paper_1607_02955_amd as cfc
    eg = synth.road_grid(2048, seed=1)
    g = cfc.Graph.from_edgelist(ctx, eg).build_hierarchy()
    L = LAP.of(eg)
    rng = np.random.default_rng(4)
    n = eg.n
    B = np.zeros((3, n))
    B[0, 0], B[0, n - 1] = 1.0, -1.0
    B[1, rng.integers(0, n, 50)] = rng.standard_normal(50)
    B[1] -= B[1].mean()
    B[2, 12345], B[2, 2000000] = 1.0, -1.0
    X, st, status = g.solve(B, tol=1e-6, stats=True)
    say("road2048", st)
    assert np.all(status == 0)
    # residual certificate with the oracle's operator (independent of the library)
    res = np.linalg.norm(B.T - L @ X.T, axis=0) / np.linalg.norm(B.T, axis=0)
    assert res.max() <= 1.01e-6, res
    # mean-zero (= L^+ b) up to FP64 summation rounding
    assert np.all(np.abs(X.sum(axis=1)) <= 1e-12 * np.abs(X).sum(axis=1))
    # symmetry and the triangle inequality of effective resistance
    s = np.array([0, 12345, 777])
    t = np.array([n - 1, 2000000, 4000000])
    r1 = g.resistance(s, t, tol=1e-8)
    r2 = g.resistance(t, s, tol=1e-8)
    np.testing.assert_allclose(r1, r2, rtol=1e-6)
    rab, rbc, rac = g.resistance([0, 12345, 0], [12345, 2000000, 2000000], tol=1e-8)
    assert rac <= rab + rbc
    # R from the dense solve agrees with the pair entry point
    np.testing.assert_allclose(X[0, 0] - X[0, n - 1], r1[0], rtol=2e-6)
    # against the oracle's grounded-route values, at the benchmark tolerance
    gold = json.load(open(os.path.join(GOLD, "road2048_pairs.json")))
    gs, gt, want = np.array(gold["s"]), np.array(gold["t"]), np.array(gold["resistance"])
    r, st = g.resistance(gs, gt, tol=1e-6, stats=True)
    err = np.abs(r / want - 1)
    say("road2048 golden pairs: rel err", err, "max rel residual", st["max_rel_residual"])
    Bp = np.zeros((len(gs), n))
    Bp[np.arange(len(gs)), gs] += 1.0
    Bp[np.arange(len(gs)), gt] -= 1.0
    Xp, _, status = g.solve(Bp, tol=1e-6, stats=True)
    d, cert, res = _pair_certificate(L, eg, Xp, gs, gt)
    say("  dense solve: rel err", np.abs(d / want - 1), "bound ||x|| ||r|| / b^T x", cert, "rel res", res)
    assert np.all(status == 0)
    assert err.max() <= 1e-6
    assert np.max(np.abs(d / want - 1)) <= 1e-6
