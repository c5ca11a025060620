"""The allocation-free projection farness entry point (GPU).

cfc_farness_jl_static stages its data in a fixed per-GPU device array
instead of allocating; it must give what cfc_farness_jl gives, call after
call, with host or device buffers, and refuse requests above its limit.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sketched():
    import paper_1607_02955_amd as cfc
    ctx = cfc.Context(0)
    eg = synth.barabasi_albert(20000, 4, seed=3)
    g = cfc.Graph.from_edgelist(ctx, eg).build_hierarchy()
    g.jl_sketch(64, seed=5, tol=1e-6)
    return cfc, ctx, eg, g


def test_static_equals_allocating_call_twice(sketched):
    cfc, ctx, eg, g = sketched
    rng = np.random.default_rng(1)
    # two calls in a row, the second with a smaller input (and repeated ids)
    for q in (5000, 37):
        nodes = rng.integers(0, eg.n, q)
        say(f"case: static farness, {q} host nodes")
        want_f, want_c = g.farness_jl(nodes)
        got_f, got_c = g.farness_jl_static(nodes)
        # the same two FP64 roundings per value (product, then sum): equal up
        # to one rounding of either
        np.testing.assert_allclose(got_f, want_f, rtol=1e-15, atol=0)
        np.testing.assert_allclose(got_c, want_c, rtol=1e-15, atol=0)


def test_static_device_buffers_and_all_nodes(sketched):
    import torch
    cfc, ctx, eg, g = sketched
    say("case: static farness, device buffers and every node")
    want_f, want_c = g.farness_jl()
    far = torch.empty(eg.n, dtype=torch.float64, device="cuda")
    clo = torch.empty(eg.n, dtype=torch.float64, device="cuda")
    g.farness_jl_static(None, far, clo)
    torch.cuda.synchronize()
    np.testing.assert_allclose(far.cpu().numpy(), want_f, rtol=1e-15, atol=0)
    np.testing.assert_allclose(clo.cpu().numpy(), want_c, rtol=1e-15, atol=0)
    nodes = torch.tensor([3, 19999, 0, 3], dtype=torch.int64, device="cuda")
    f2 = torch.empty(4, dtype=torch.float64, device="cuda")
    g.farness_jl_static(nodes, f2, None)
    torch.cuda.synchronize()
    np.testing.assert_allclose(f2.cpu().numpy(), want_f[[3, 19999, 0, 3]], rtol=1e-15, atol=0)


def test_static_limits_and_errors(sketched):
    cfc, ctx, eg, g = sketched
    say("case: static farness, errors")
    with pytest.raises(cfc.CfcError, match="INVALID"):
        g.farness_jl_static(np.zeros((1 << 18) + 1, np.int64))
    with pytest.raises(cfc.CfcError, match="INVALID"):
        g.farness_jl_static([eg.n])
    with pytest.raises(cfc.CfcError, match="INVALID"):
        g.farness_jl_static([4, -1])
    f, c = g.farness_jl_static(np.zeros(0, np.int64))
    assert f.shape == (0,)
    g2 = cfc.Graph.from_edgelist(ctx, synth.grid(8)).build_hierarchy()
    with pytest.raises(cfc.CfcError, match="STATE"):  # no sketch
        g2.farness_jl_static([1])
