"""Effective resistance, electrical farness and current-flow closeness.

Definitions followed (arXiv 1607.02955):

* Eq. (1): L p_st = b_st with b_st = e_s - e_t; p is fixed only up to an
  additive constant (L has rank n-1 on a connected graph), Sec. 2.
* Sec. 4: d_ER(u, v) = p_uv(u) - p_uv(v); d_ER(v, v) = 0.
* Eq. (3): c_ER(v) = (n-1) / sum_{w != v} d_ER(v, w); the denominator is the
  electrical farness.
* Sec. 4, last paragraph: with node g's row and column removed, the grounded
  matrix L~ is regular and d_ER(v, w) = L~^-1_vv - 2 L~^-1_vw + L~^-1_ww.
* Sec. 5.2: d_ER(u, v) = (e_u - e_v)^T L^+ (e_u - e_v) with L^+ the
  Moore-Penrose pseudoinverse.
* Sec. 3.1: an iterative solver stops when the relative residual
  ||b - L x|| / ||b|| falls below a tolerance tau; CG is the practical baseline.

Three independent routes (pseudoinverse, grounded inverse -- dense, or a
sparse LU factorisation for large graphs -- and CG) are provided so that tests
can check them against each other and against closed forms.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


# ---- dense routes ----------------------------------------------------------

def pinv(L: np.ndarray) -> np.ndarray:
    """Moore-Penrose pseudoinverse by SVD (numpy)."""
    return np.linalg.pinv(L, rcond=1e-12, hermitian=True)


def grounded_inverse(L: np.ndarray, g: int = 0) -> np.ndarray:
    """Inverse of L with row/column g removed (Cholesky), padded back to n x n
    with zeros in row and column g."""
    n = L.shape[0]
    keep = np.r_[0:g, g + 1:n]
    Lg = L[np.ix_(keep, keep)]
    c = sla.cho_factor(Lg, lower=True)
    inv = sla.cho_solve(c, np.eye(n - 1))
    out = np.zeros((n, n))
    out[np.ix_(keep, keep)] = inv
    return out


def resistance_from_inverse(M: np.ndarray, u, v):
    """d_ER(u, v) = M_uu - 2 M_uv + M_vv for M = L^+ or the padded grounded inverse."""
    u = np.asarray(u)
    v = np.asarray(v)
    return M[u, u] - 2.0 * M[u, v] + M[v, v]


def resistance_matrix(M: np.ndarray) -> np.ndarray:
    d = np.diag(M)
    return d[:, None] - 2.0 * M + d[None, :]


def farness_dense(M: np.ndarray, v):
    """Electrical farness sum_{w != v} d_ER(v, w) (Eq. 3) from an inverse."""
    R = resistance_matrix(M)
    v = np.atleast_1d(v)
    return R[v].sum(axis=1) - R[v, v]


# ---- iterative route -------------------------------------------------------

def cg(L, B, tol=1e-12, maxiter=100000):
    """Jacobi-preconditioned conjugate gradients on L X = B, column by column
    in lock-step (each column has its own step sizes), x0 = 0.  Every column of
    B must sum to zero.  Stops when every column has
    ||b - L x|| <= tol ||b||; returns X projected to mean zero (the L^+ b
    representative) and the iteration count."""
    B = np.asarray(B, np.float64)
    one_d = B.ndim == 1
    if one_d:
        B = B[:, None]
    dinv = 1.0 / L.diagonal()
    X = np.zeros_like(B)
    R = B.copy()
    bn = np.linalg.norm(B, axis=0)
    active = bn > 0
    Z = dinv[:, None] * R
    P = Z.copy()
    rz = np.einsum("ij,ij->j", R, Z)
    it = 0
    while it < maxiter:
        rn = np.linalg.norm(R, axis=0)
        if np.all(rn[active] <= tol * bn[active]):
            break
        Q = L @ P
        pq = np.einsum("ij,ij->j", P, Q)
        alpha = np.where(pq != 0, rz / np.where(pq != 0, pq, 1), 0.0)
        X += alpha * P
        R -= alpha * Q
        Z = dinv[:, None] * R
        rz_new = np.einsum("ij,ij->j", R, Z)
        beta = np.where(rz != 0, rz_new / np.where(rz != 0, rz, 1), 0.0)
        P = Z + beta * P
        rz = rz_new
        it += 1
    X -= X.mean(axis=0)
    return (X[:, 0] if one_d else X), it


def pair_rhs(n, s, t):
    """Columns b_j = e_{s_j} - e_{t_j} (Sec. 2, supply b_st)."""
    s = np.atleast_1d(s)
    t = np.atleast_1d(t)
    B = np.zeros((n, s.shape[0]))
    B[s, np.arange(s.shape[0])] += 1.0
    B[t, np.arange(t.shape[0])] -= 1.0
    return B


def resistance_cg(L, s, t, tol=1e-12):
    """d_ER(s_j, t_j) = p(s_j) - p(t_j) for L p = e_s - e_t (Sec. 4), by CG."""
    s = np.atleast_1d(s)
    t = np.atleast_1d(t)
    X, _ = cg(L, pair_rhs(L.shape[0], s, t), tol)
    j = np.arange(s.shape[0])
    return X[s, j] - X[t, j]


def resistance_grounded_sparse(L, s, t, g=0):
    """d_ER(s_j, t_j) by the grounded route of Sec. 4 on a sparse L: with row
    and column g removed the grounded Laplacian is regular, so
    L~ p = (e_s - e_t) without row g has one solution, with p(g) = 0, and
    d_ER(s, t) = p(s) - p(t).  One sparse LU factorisation (SuperLU, column
    ordering COLAMD) serves every pair; for graphs whose factor fits in host
    memory (a 2048 x 2048 grid: about 10 GB)."""
    import scipy.sparse.linalg as spla
    s = np.atleast_1d(np.asarray(s, np.int64))
    t = np.atleast_1d(np.asarray(t, np.int64))
    n = L.shape[0]
    keep = np.r_[0:g, g + 1:n]
    Lg = L.tocsr()[keep][:, keep].tocsc()
    lu = spla.splu(Lg, permc_spec="COLAMD", options=dict(SymmetricMode=True))
    B = pair_rhs(n, s, t)[keep]
    P = np.zeros((n, s.shape[0]))
    P[keep] = lu.solve(B)
    j = np.arange(s.shape[0])
    return P[s, j] - P[t, j]


def farness_exact_cg(L, v, tol=1e-12):
    """Exact farness of v by its n-1 solves L p = e_v - e_w (Sec. 4, Eq. 3)."""
    n = L.shape[0]
    others = np.array([w for w in range(n) if w != v], np.int64)
    return float(resistance_cg(L, np.full(others.shape, v), others, tol).sum())


def closeness(n, farness):
    """c_ER = (n-1) / farness (Eq. 3)."""
    return (n - 1) / np.asarray(farness, np.float64)
