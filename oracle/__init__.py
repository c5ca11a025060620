"""CPU oracle for current-flow closeness (plain, slow, float64).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import or run
anything in this package.  The product path (the HIP library and its Python
binding) never imports it, and this package imports nothing from the product.

Contents, each function citing the passage of Bergamini, Wegner, Lukarski and
Meyerhenke, "Estimating Current-Flow Closeness Centrality with a Multigrid
Laplacian Solver" (arXiv 1607.02955) that it writes out:

* ``laplacian``  -- L = D - A (Sec. 2, "Graph basics").
* ``resistance`` -- effective resistance d_ER (Sec. 4) by the Moore-Penrose
  pseudoinverse, by the grounded-inverse identity (Sec. 4, last paragraph) and
  by conjugate gradients (Sec. 3.1); electrical farness and c_ER (Eq. 3).
* ``estimators`` -- the Sampling estimator (Sec. 5.1, Prop. 1) and the
  projection (JLT) estimator (Sec. 5.2, Algorithm 1).
* ``spectral``   -- d_ER on the undeleted N x M grid from the Laplacian's
  cosine eigenbasis (Sec. 5.2's d_ER = (e_u - e_v)^T L^+ (e_u - e_v) written
  out in that basis), which pins solves on grids too large for the dense
  routes.
* ``edges``, ``betweenness`` -- spanning-edge centrality and current-flow
  betweenness (named in Sec. 3.2).
* ``rng``        -- the counter-based generator that fixes pivots and
  projection signs for a seed (SplitMix64, Lemire's bounded integers, Floyd's
  subset sampling), written from the published definitions.

Parity status: every function here is pinned by a CPU test against closed
forms, brute force or special cases (tests/test_oracle_*.py), except where a
docstring says "parity unpinned".
"""
