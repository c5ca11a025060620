"""Serving loop: continuous batching over resident graphs (GPU)."""
import sys
import time

import numpy as np
import pytest

import synth
from oracle import estimators as E
from oracle import laplacian as LAP

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import paper_1607_02955_amd as cfc
    ctx = cfc.Context(0)
    egs = [synth.barabasi_albert(3000, 4, seed=5), synth.road_grid(50, seed=6),
           synth.random_connected(2000, 7000, seed=7), synth.rmat(12, seed=8)]
    gs = [cfc.Graph.from_edgelist(ctx, eg).build_hierarchy(coarsest_max=64) for eg in egs]
    assert gs[3].info()["eliminated"] > 0  # one graph with an elimination level
    return cfc, ctx, egs, gs


def queries(egs):
    rng = np.random.default_rng(3)
    out = []
    for i in range(16):
        gi = i % len(egs)
        nn = int(rng.integers(1, 6))
        nodes = rng.choice(egs[gi].n, nn, replace=False)
        kind = (i + i // len(egs)) % 2
        out.append((gi, kind, nodes, 30 + 5 * (i % 3)))
    return out


def test_alone_equals_mix(setup):
    cfc, ctx, egs, gs = setup
    with cfc.Server(ctx, slots=64, jl_k=48, sampling_k=40, seed=11, tol=1e-8) as srv:
        ids = [srv.add_graph(g) for g in gs]
        qs = queries(egs)
        alone = []
        for gi, kind, nodes, k in qs:
            t = srv.submit(ids[gi], kind, nodes, k=k)
            alone.append(srv.wait(t, timeout_ms=60000))
        say("alone done", srv.stats())
        tickets = [srv.submit(ids[gi], kind, nodes, k=k) for gi, kind, nodes, k in qs]
        mixed = [srv.wait(t, timeout_ms=60000) for t in tickets]
        st = srv.stats()
        say("mix done", st)
        # a served graph refuses direct calls until the server is gone
        with pytest.raises(cfc.CfcError, match="STATE"):
            gs[0].farness_sampling([1], 5, seed=11, tol=1e-8)
        # and joins one server at a time
        with cfc.Server(ctx, slots=32, jl_k=0) as other:
            with pytest.raises(cfc.CfcError, match="STATE"):
                other.add_graph(gs[0])
    for (gi, kind, nodes, k), a, m in zip(qs, alone, mixed):
        assert a is not None and m is not None
        np.testing.assert_allclose(m[0], a[0], rtol=1e-6)
        if kind == cfc.QUERY_JL:
            np.testing.assert_array_equal(m[0], a[0])  # read from the resident sketch
    assert st["completed"] == st["submitted"] == 2 * len(qs)
    assert st["p99_ms"] >= st["p50_ms"] > 0 and st["queries_per_s"] > 0
    # against the direct calls and the oracle, same seeds
    for (gi, kind, nodes, k), m in zip(qs, mixed):
        if kind == cfc.QUERY_SAMPLING:
            of, _, _, _ = E.sampling(LAP.of(egs[gi]), egs[gi], nodes, k, 11, tol=1e-12)
            np.testing.assert_allclose(m[0], of, rtol=1e-6)
            f2, _ = gs[gi].farness_sampling(nodes, k, seed=11, tol=1e-8)
            np.testing.assert_allclose(m[0], f2, rtol=1e-6)
        else:
            of, _, _ = E.projection(LAP.of(egs[gi]), egs[gi], nodes, 48, 11, tol=1e-12)
            np.testing.assert_allclose(m[0], of, rtol=1e-6)


def test_requests_join_a_running_block(setup):
    """Queries submitted while a long one is in flight finish before it."""
    cfc, ctx, egs, gs = setup
    with cfc.Server(ctx, slots=32, jl_k=0, sampling_k=40, seed=2, tol=1e-8) as srv:
        gid = srv.add_graph(gs[1])
        big = srv.submit(gid, cfc.QUERY_SAMPLING, np.arange(40), k=400)  # 40 x ~400 columns
        time.sleep(0.05)
        small = srv.submit(gid, cfc.QUERY_SAMPLING, [3], k=5)
        rs = srv.wait(small, timeout_ms=60000)
        pending = srv.poll(big)
        rb = pending if pending is not None else srv.wait(big, timeout_ms=120000)
    assert rs is not None and rb is not None
    assert rs[2] < rb[2]  # latency


def test_admission_budget(setup):
    cfc, ctx, egs, gs = setup
    # a budget too small for any slot workspace: sampling queries fail cleanly
    with cfc.Server(ctx, slots=32, jl_k=0, sampling_k=10, tol=1e-8, hbm_budget=1024) as srv:
        gid = srv.add_graph(gs[0])
        t = srv.submit(gid, cfc.QUERY_SAMPLING, [1, 2], k=10)
        with pytest.raises(cfc.CfcError, match="NOMEM"):
            srv.wait(t, timeout_ms=30000)
    # a budget for one workspace at a time: two graphs are served in turn
    with cfc.Server(ctx, slots=32, jl_k=0, sampling_k=10, tol=1e-8, hbm_budget=60 << 20) as srv:
        a, b = srv.add_graph(gs[0]), srv.add_graph(gs[2])
        ts = [srv.submit(a, cfc.QUERY_SAMPLING, [1, 2], k=20), srv.submit(b, cfc.QUERY_SAMPLING, [3], k=20)]
        for t in ts:
            assert srv.wait(t, timeout_ms=60000) is not None


def test_server_errors(setup):
    cfc, ctx, egs, gs = setup
    with cfc.Server(ctx, slots=32, jl_k=0, max_queue=2) as srv:
        gid = srv.add_graph(gs[0])
        with pytest.raises(cfc.CfcError, match="INVALID"):
            srv.submit(gid + 5, cfc.QUERY_SAMPLING, [1])
        with pytest.raises(cfc.CfcError, match="INVALID"):
            srv.submit(gid, cfc.QUERY_SAMPLING, [10 ** 9])
        t = srv.submit(gid, cfc.QUERY_JL, [1])  # no sketch on this server
        with pytest.raises(cfc.CfcError):
            srv.wait(t, timeout_ms=30000)
