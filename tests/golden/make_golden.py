"""Write expected values for the full-size parity tests (oracle only).

Run from the repository root:  python tests/golden/make_golden.py [name ...]

Every value comes from the CPU oracle (oracle/) on inputs from synth/; no
value comes from the HIP library.

* ba100k_jl512.json: projection estimate (Algorithm 1) of the farness of the
  100 benchmark query nodes on the Barabasi-Albert graph n = 100,000 (4 edges
  per new node, seed 1), k = 512, seed 1; solves by the oracle's CG to 1e-12.
* rmat20_pairs.json: effective resistances d_ER(v, s) (Sec. 4) on the R-MAT
  scale-20 LCC (weights U[1,4], seed 1) for pairs of benchmark query nodes v
  and their first Sampling pivots (seed 1, k = 1000); CG to 1e-12.
* rmat20_sampling64.json: Sampling estimate (Sec. 5.1) of the farness of the
  first two benchmark query nodes on the same graph with k = 64 pivots, seed
  1; CG to 1e-12.
* road2048_pairs.json: effective resistances on the 2%-deleted 2048 x 2048
  road graph (weights U[1,10], seed 1): two benchmark Sampling pairs and four
  long- and short-range pairs, by the grounded route of Sec. 4 (one sparse LU
  factorisation; CG to 1e-12 would take hours on this grid).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import estimators as E  # noqa: E402
from oracle import laplacian as LAP  # noqa: E402
from oracle import resistance as R  # noqa: E402
from oracle import rng as RNG  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def ba100k_jl512():
    eg = synth.cached("ba100000", synth.barabasi_albert, 100000, 4, seed=1)
    nodes = synth.query_nodes(eg.n, 100, seed=1)
    t = time.time()
    far, clo, _ = E.projection(LAP.of(eg), eg, nodes, 512, 1, tol=1e-12)
    return {"graph": "barabasi_albert(100000, 4, seed=1)", "k": 512, "seed": 1,
            "nodes": nodes.tolist(), "farness": far.tolist(), "closeness": clo.tolist(),
            "oracle": "estimators.projection, cg tol 1e-12", "seconds": round(time.time() - t, 1)}


def rmat20_pairs():
    eg = synth.cached("rmat20", synth.rmat, 20, 16, seed=1)
    nodes = synth.query_nodes(eg.n, 64, seed=1)
    s, t = [], []
    for v in nodes[:6]:
        piv = [p for p in RNG.pivots(1, int(v), eg.n, 1000) if p != v]
        for p in piv[:2]:
            s.append(int(v))
            t.append(int(p))
    t0 = time.time()
    r = R.resistance_cg(LAP.of(eg), np.array(s), np.array(t), tol=1e-12)
    return {"graph": "rmat(20, 16, seed=1) LCC, weights U[1,4]", "s": s, "t": t,
            "resistance": r.tolist(), "oracle": "resistance.resistance_cg, tol 1e-12",
            "seconds": round(time.time() - t0, 1)}


def rmat20_sampling64():
    eg = synth.cached("rmat20", synth.rmat, 20, 16, seed=1)
    nodes = synth.query_nodes(eg.n, 64, seed=1)[:2]
    t0 = time.time()
    far, clo, piv, _ = E.sampling(LAP.of(eg), eg, nodes, 64, 1, tol=1e-12)
    return {"graph": "rmat(20, 16, seed=1) LCC, weights U[1,4]", "k": 64, "seed": 1,
            "nodes": nodes.tolist(), "farness": list(map(float, far)), "closeness": list(map(float, clo)),
            "pivots": [p.tolist() for p in piv], "oracle": "estimators.sampling, cg tol 1e-12",
            "seconds": round(time.time() - t0, 1)}


def road2048_pairs():
    eg = synth.cached("road2048", synth.road_grid, 2048, seed=1)
    n = eg.n
    s, t = [], []
    for v in synth.query_nodes(n, 32, seed=1)[:2]:  # two Sampling pairs of the benchmark
        p = next(p for p in RNG.pivots(1, int(v), n, 500) if p != v)
        s.append(int(v))
        t.append(int(p))
    c = 1024 * 2048 + 1024
    s += [0, c, 12345, 3000000]
    t += [n - 1, c + 1, 2000000, 1234567]
    t0 = time.time()
    r = R.resistance_grounded_sparse(LAP.of(eg), np.array(s), np.array(t), g=n // 2)
    return {"graph": "road_grid(2048, seed=1): 2048^2 grid, 2% of edges deleted, LCC, weights U[1,10]",
            "n": n, "s": s, "t": t, "resistance": r.tolist(),
            "oracle": "resistance.resistance_grounded_sparse (sparse LU of the grounded Laplacian)",
            "seconds": round(time.time() - t0, 1)}


MAKERS = {"ba100k_jl512": ba100k_jl512, "rmat20_pairs": rmat20_pairs,
          "rmat20_sampling64": rmat20_sampling64, "road2048_pairs": road2048_pairs}

if __name__ == "__main__":
    for name in sys.argv[1:] or list(MAKERS):
        out = MAKERS[name]()
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(out, fh, indent=1)
        print(name, "done", out.get("seconds"), "s", flush=True)
