"""Effective resistance on the undeleted N x M grid from the Laplacian's
eigenbasis: a closed form that pins solves on grids far too large for the
dense routes.  Test infrastructure, like the rest of oracle/.

The N x M 4-neighbour grid (node id r*M + c, unit conductances) is the
Cartesian product of the paths P_N and P_M, so its Laplacian is
L_N (x) I_M + I_N (x) L_M.  The path Laplacian L_N is diagonalised by the
cosine (DCT-II) basis: eigenvalue 4 sin^2(pi j / 2N) with the orthonormal
eigenvector phi_j(x) = c_j cos(pi j (x + 1/2) / N), c_0 = sqrt(1/N),
c_j = sqrt(2/N) otherwise.  The grid's eigenpairs are the products
lambda_jk = lambda_j + lambda_k, phi_jk(r, c) = phi_j(r) phi_k(c).

With d_ER(u, v) = (e_u - e_v)^T L^+ (e_u - e_v) (Sec. 5.2) and L^+ the sum of
phi phi^T / lambda over the nonzero eigenvalues,

    d_ER(u, v) = sum over (j, k) != (0, 0) of (phi_jk(u) - phi_jk(v))^2 / lambda_jk.

Every term is positive, so the FP64 sum of the N*M terms is accurate to a
few units in the last place.
"""
from __future__ import annotations

import numpy as np


def _path_basis(N: int, x: int) -> np.ndarray:
    """phi_j(x) for j = 0..N-1 (orthonormal eigenvectors of L_N)."""
    j = np.arange(N)
    c = np.where(j == 0, np.sqrt(1.0 / N), np.sqrt(2.0 / N))
    return c * np.cos(np.pi * j * (x + 0.5) / N)


def _path_eigenvalues(N: int) -> np.ndarray:
    return 4.0 * np.sin(np.pi * np.arange(N) / (2.0 * N)) ** 2


def grid_resistance(N: int, M: int, u, v) -> np.ndarray:
    """d_ER(u_i, v_i) on the N x M grid for every pair (u_i, v_i)."""
    u = np.atleast_1d(np.asarray(u, np.int64))
    v = np.atleast_1d(np.asarray(v, np.int64))
    lam = _path_eigenvalues(N)[:, None] + _path_eigenvalues(M)[None, :]
    lam[0, 0] = np.inf  # the constant vector: no contribution
    out = np.empty(u.shape[0])
    for i in range(u.shape[0]):
        ru, cu = divmod(int(u[i]), M)
        rv, cv = divmod(int(v[i]), M)
        d = np.outer(_path_basis(N, ru), _path_basis(M, cu)) - np.outer(_path_basis(N, rv), _path_basis(M, cv))
        out[i] = float(np.sum(d * d / lam))
    return out


def grid_pinv_diag(N: int, M: int, u) -> np.ndarray:
    """L^+_uu on the N x M grid (sum of phi_jk(u)^2 / lambda_jk)."""
    u = np.atleast_1d(np.asarray(u, np.int64))
    lam = _path_eigenvalues(N)[:, None] + _path_eigenvalues(M)[None, :]
    lam[0, 0] = np.inf
    out = np.empty(u.shape[0])
    for i in range(u.shape[0]):
        r, c = divmod(int(u[i]), M)
        p = np.outer(_path_basis(N, r), _path_basis(M, c))
        out[i] = float(np.sum(p * p / lam))
    return out


def grid_pinv_trace(N: int, M: int) -> float:
    """tr(L^+) on the N x M grid (sum of 1 / lambda_jk over nonzero eigenvalues)."""
    lam = _path_eigenvalues(N)[:, None] + _path_eigenvalues(M)[None, :]
    lam[0, 0] = np.inf
    return float(np.sum(1.0 / lam))


def grid_farness(N: int, M: int, v) -> np.ndarray:
    """Electrical farness sum_{w != v} d_ER(v, w) (Eq. 3) on the N x M grid,
    as n L^+_vv + tr(L^+): summing d_ER(v, w) = L^+_vv - 2 L^+_vw + L^+_ww over
    all w, the middle terms vanish because every row of L^+ sums to zero."""
    return N * M * grid_pinv_diag(N, M, v) + grid_pinv_trace(N, M)
