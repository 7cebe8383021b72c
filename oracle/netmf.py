"""NetMF matrix and the low-rank factors of Eq. (11), in float64.

Readings of points the paper leaves open:
* trunc_log(x) = max(0, log x) (Eq. 1, natural log).  It is defined only for
  x > 0; the oracle uses log(max(x, 1)), which equals it for x > 0 and gives
  0 for x <= 0.
* vol(G) = sum_ij A_ij (Section 2), i.e. twice the number of undirected edges.
* An isolated vertex has degree 0 and D^-1 is undefined there; every power
  deg^(-beta) is taken as 0 for such a vertex, so its row and column of every
  matrix below are zero.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def adjacency(rowptr, colidx, n=None) -> sp.csr_matrix:
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    n = len(rowptr) - 1 if n is None else n
    data = np.ones(len(colidx), dtype=np.float64)
    return sp.csr_matrix((data, colidx, rowptr), shape=(n, n))


def degrees(A) -> np.ndarray:
    return np.asarray(A.sum(axis=1)).ravel().astype(np.float64)


def volume(A) -> float:
    """vol(G) = sum_i sum_j A_ij (Section 2)."""
    return float(A.sum())


def deg_power(deg: np.ndarray, beta: float) -> np.ndarray:
    """deg^beta with the isolated-vertex convention (0 where deg == 0)."""
    out = np.zeros_like(deg, dtype=np.float64)
    nz = deg > 0
    out[nz] = deg[nz] ** beta
    return out


def trunc_log(x):
    """Element-wise truncated logarithm max(0, log x) (Eq. 1)."""
    return np.log(np.maximum(x, 1.0))


def netmf_matrix(A, T: int, b: float) -> np.ndarray:
    """Eq. (1) before the truncated log: M = vol/(bT) * sum_{r=1..T} (D^-1 A)^r D^-1.

    Dense n x n result, built by repeated sparse x dense products."""
    n = A.shape[0]
    deg = degrees(A)
    dinv = deg_power(deg, -1.0)
    P = sp.diags(dinv) @ A  # D^-1 A
    X = np.diag(dinv)  # (D^-1 A)^0 D^-1
    acc = np.zeros((n, n))
    for _ in range(T):
        X = P @ X
        acc += X
    return volume(A) / (b * T) * acc


def modified_laplacian(A, alpha: float):
    """D^-alpha A D^-alpha (Section 3.2), sparse."""
    d = deg_power(degrees(A), -alpha)
    return (sp.diags(d) @ A @ sp.diags(d)).tocsr()


def eq2_matrix(A, U, lam, T: int, b: float) -> np.ndarray:
    """Eq. (2) before the truncated log:
    vol/(bT) D^-1/2 U (sum_{r=1..T} Lambda^r) U^T D^-1/2."""
    deg = degrees(A)
    dm = deg_power(deg, -0.5)
    coeff = sum(lam ** r for r in range(1, T + 1))
    G = dm[:, None] * U
    return volume(A) / (b * T) * (G * coeff) @ G.T


def eq11_factors(U, lam, deg, vol: float, alpha: float, T: int, b: float):
    """The factors of Eq. (11) (also Alg. 6 lines 2-3).

    K  = U^T D^(-1+2a) U Lambda                      (k x k)
    L' = vol/(bT) D^(-1+a) U                         (n x k)
    R' = Lambda (sum_{r=1..T} K^(r-1)) U^T D^(-1+a)  (k x n)
    """
    U = np.asarray(U, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    k = U.shape[1]
    d1 = deg_power(deg, -1.0 + alpha)
    d2 = deg_power(deg, -1.0 + 2.0 * alpha)
    Kmat = (U.T * d2) @ U @ np.diag(lam)
    S = np.zeros((k, k))
    Kp = np.eye(k)
    for _ in range(T):  # r = 1..T adds K^(r-1)
        S += Kp
        Kp = Kp @ Kmat
    Lp = vol / (b * T) * (d1[:, None] * U)
    Rp = np.diag(lam) @ S @ (U.T * d1)
    return Lp, Rp, Kmat


def core_matrix(lam, Kmat, T: int) -> np.ndarray:
    """C = Lambda * sum_{r=1..T} K^(r-1), so that R' = C U^T D^(-1+a)."""
    k = len(lam)
    S = np.zeros((k, k))
    Kp = np.eye(k)
    for _ in range(T):
        S += Kp
        Kp = Kp @ Kmat
    return np.diag(lam) @ S


def eq11_kmat(U, lam, deg, alpha: float, block: int = 1 << 20):
    """K = U^T D^(-1+2a) U Lambda of Eq. (11), summed over row blocks of U
    (the same sum as in eq11_factors, for n too large to widen U at once)."""
    lam = np.asarray(lam, dtype=np.float64)
    n, k = U.shape
    d2 = deg_power(deg, -1.0 + 2.0 * alpha)
    G = np.zeros((k, k))
    for r0 in range(0, n, block):
        Ub = np.asarray(U[r0:r0 + block], dtype=np.float64)
        G += (Ub.T * d2[r0:r0 + block]) @ Ub
    return G @ np.diag(lam)


def eq11_rows(U_rows, deg_rows, lam, Kmat, vol: float, alpha: float, T: int, b: float):
    """Rows of L' and the matching columns of R' (Eq. 11) for a subset of
    vertices: L'(i,:) = vol/(bT) d_i^(-1+a) U_i and R'(:,i) = C d_i^(-1+a) U_i^T."""
    U_rows = np.asarray(U_rows, dtype=np.float64)
    d1 = deg_power(deg_rows, -1.0 + alpha)
    C = core_matrix(lam, Kmat, T)
    return vol / (b * T) * (d1[:, None] * U_rows), C @ (U_rows.T * d1)
