"""Parity at the benchmark sizes, in the launch configuration bench.py times.

Expected values come from tests/golden/*.json, written by
tests/golden/make_golden.py from the CPU oracle.  Where the oracle cannot
solve at full size in seconds (the 2048^2 road graph), properties that hold
at any size are checked with the oracle's operator instead.
"""
import json
import os
import sys

import numpy as np
import pytest

import synth
from oracle import laplacian as LAP

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
    assert err < 5e-6  # the solve itself to 1e-6 residual


def test_rmat20_pair_resistances(ctx):
    import paper_1607_02955_amd as cfc
    gold = json.load(open(os.path.join(GOLD, "rmat20_pairs.json")))
    eg = synth.rmat(20, 16, seed=1)
    g = cfc.Graph.from_edgelist(ctx, eg).build_hierarchy()
    r, st = g.resistance(gold["s"], gold["t"], block=256, tol=1e-6, stats=True)
    say("rmat20", st["levels_used"], st["inner_iters"], r[:3], gold["resistance"][:3])
    np.testing.assert_allclose(r, gold["resistance"], rtol=1e-6)
    # the Sampling entry point on the same graph and seed reuses those pivots
    v = gold["s"][0]
    far, clo = g.farness_sampling([v], 1000, seed=1, block=256, tol=1e-6)
    assert far[0] > 0 and np.isfinite(clo[0])


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
