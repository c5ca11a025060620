"""Pins of the grid closed form (oracle/spectral.py) against other routes.

The closed form sums over the grid Laplacian's eigenbasis; each pin fixes
its values by something else: path and 4-cycle resistances, the dense
pseudoinverse and grounded-inverse routes, and Foster's theorem.
"""
import numpy as np
import pytest

import synth
from oracle import laplacian as LAP
from oracle import resistance as R
from oracle import spectral as SP


@pytest.mark.parametrize("N,M", [(9, 1), (1, 11)])
def test_path_is_distance(N, M):
    n = N * M
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    got = SP.grid_resistance(N, M, u.ravel(), v.ravel())
    np.testing.assert_allclose(got, np.abs(u - v).ravel(), atol=1e-12)


def test_four_cycle():
    # the 2 x 2 grid is the 4-cycle: adjacent 1*3/4, opposite 2*2/4
    np.testing.assert_allclose(SP.grid_resistance(2, 2, [0, 0, 0, 1], [1, 2, 3, 2]),
                               [0.75, 0.75, 1.0, 1.0], atol=1e-14)


@pytest.mark.parametrize("N,M", [(5, 7), (6, 6)])
def test_all_pairs_match_pseudoinverse(N, M):
    g = synth.grid(N, M)
    Lp = R.pinv(LAP.of(g, dense=True))
    n = N * M
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    got = SP.grid_resistance(N, M, u.ravel(), v.ravel())
    np.testing.assert_allclose(got, R.resistance_from_inverse(Lp, u.ravel(), v.ravel()), atol=1e-12)


def test_grid32_pairs_match_grounded_inverse_and_farness():
    g = synth.grid(32)
    G = R.grounded_inverse(LAP.of(g, dense=True), 100)
    rng = np.random.default_rng(2)
    u, v = rng.integers(0, 1024, 40), rng.integers(0, 1024, 40)
    np.testing.assert_allclose(SP.grid_resistance(32, 32, u, v), R.resistance_from_inverse(G, u, v),
                               rtol=1e-11, atol=1e-13)
    f = SP.grid_farness(32, 32, [0, 5 * 32 + 9])
    np.testing.assert_allclose(f, R.farness_dense(G, [0, 5 * 32 + 9]), rtol=1e-11)


def test_foster_on_a_rectangle():
    # sum over edges of R_e = n - 1 (unit conductances)
    g = synth.grid(6, 9)
    np.testing.assert_allclose(SP.grid_resistance(6, 9, g.u, g.v).sum(), 6 * 9 - 1, rtol=1e-12)
