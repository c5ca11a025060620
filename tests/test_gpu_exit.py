"""Process exit with library objects still open (GPU).

A child interpreter registers a graph with a server, submits a Sampling
query that is still in flight, and ends without closing anything.  The
binding's exit hook must then stop the server's worker (after its current
refinement step), release the graph and free every device buffer while the
interpreter and torch's allocator still exist, and the process must end
with status 0.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
import paper_1607_02955_amd as cfc
import synth
ctx = cfc.Context(0)
g = cfc.Graph.from_edgelist(ctx, synth.road_grid(64, seed=3)).build_hierarchy()
srv = cfc.Server(ctx, slots=64, jl_k=0, sampling_k=200, seed=1, tol=1e-10)
gid = srv.add_graph(g)
t = srv.submit(gid, cfc.QUERY_SAMPLING, np.arange(32), k=400)
print("child: query in flight, exiting with the server open", flush=True)
"""


def test_exit_with_open_server_and_query_in_flight():
    print("case: child process exits with a live server", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, capture_output=True, text=True,
                       timeout=180)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert "query in flight" in r.stdout
    assert r.returncode == 0, r.returncode
