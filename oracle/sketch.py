"""Sparse-sign single-pass sketch of f(L'R') (Section 3.1, Alg. 3, Eq. 4, Alg. 4).

Readings:
* Alg. 3 puts z nonzeros in each column of the n x h test matrix, at z
  distinct uniformly random rows, with independent fair signs.  Entries are
  scaled to +-1/sqrt(z); the SVD of Alg. 4 does not depend on this scale
  (orth(Y) is unchanged and the two pseudo-inverses cancel the scale of O in W).
* Alg. 4 line 4 multiplies an n x v matrix by S; it is read as S(p, :), the
  v nonzero rows of S.  Lines 6-7 reuse the name p for the unique rows of O;
  read as p_O and O(p_O, :).
* The realizations (rows, signs) are inputs (drawn by ``synth.sparse_sign``).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .netmf import trunc_log


def sparse_sign_matrix(n: int, rows: np.ndarray, signs: np.ndarray) -> sp.csr_matrix:
    """The n x cols test matrix of Alg. 3 (sparse), entries +-1/sqrt(z)."""
    cols, z = rows.shape
    c_idx = np.repeat(np.arange(cols), z)
    vals = signs.ravel().astype(np.float64) / np.sqrt(z)
    return sp.csr_matrix((vals, (rows.ravel().astype(np.int64), c_idx)), shape=(n, cols))


def sparse_sign_dense(n: int, rows: np.ndarray, signs: np.ndarray) -> np.ndarray:
    """The n x cols test matrix of Alg. 3 as a dense array (small n only)."""
    return sparse_sign_matrix(n, rows, signs).toarray()


def unique_rows(rows: np.ndarray) -> np.ndarray:
    """Alg. 3 last step: the sorted unique row coordinates p."""
    return np.unique(rows.ravel())


def sketch_dense(Lp, Rp, S, O):
    """Plain definition: X = L'R' formed densely, Y = f(X) S, Z = O^T f(X) O."""
    F = trunc_log(Lp @ Rp)
    return F @ S, O.T @ F @ O


def sketch_y_sampled(Lp, Rp, rows, signs, row_subset=None):
    """Eq. (4): Y = f(L' R'(:, p)) S(p, :), only v = |p| columns of f(L'R') formed.

    ``row_subset`` restricts the output to some rows of Y (rows of Y are
    independent: row i only needs row i of L')."""
    n = Rp.shape[1]
    p = unique_rows(rows)
    S = sparse_sign_matrix(n, rows, signs)[p, :].toarray()
    L = Lp if row_subset is None else Lp[row_subset]
    return trunc_log(L @ Rp[:, p]) @ S


def sketch_z_sampled(Lp, Rp, rows, signs):
    """Alg. 4 line 7: Z = O(p,:)^T f(L'(p,:) R'(:,p)) O(p,:)."""
    n = Rp.shape[1]
    p = unique_rows(rows)
    O = sparse_sign_matrix(n, rows, signs)[p, :].toarray()
    return O.T @ trunc_log(Lp[p, :] @ Rp[:, p]) @ O


def single_pass_svd(Y, Z, O, d: int):
    """Alg. 4 lines 5 and 8-10 given the sketches.

    Q = orth(Y); solve (O^T Q) T = Z, then (O^T Q) W^T = T^T (two least
    squares problems, Section 3.1); [U^, Sigma, V^] = svd(W);
    U_d = Q U^(:, 1:d), Sigma_d, V_d = Q V^(:, 1:d)."""
    Q, _ = np.linalg.qr(Y, mode="reduced")
    B = np.asarray(O.T @ Q)
    Tm = np.linalg.lstsq(B, Z, rcond=None)[0]
    W = np.linalg.lstsq(B, Tm.T, rcond=None)[0].T
    Uh, sig, Vh = np.linalg.svd(W)
    return Q @ Uh[:, :d], sig[:d], Q @ Vh.T[:, :d], W, Q


def reduced_matrix_from_sampled_O(Q, Z, rows, signs):
    """W of Alg. 4 line 8 with O given by coordinates (only its nonzero rows used)."""
    n = Q.shape[0]
    O = sparse_sign_matrix(n, rows, signs)
    B = np.asarray(O.T @ Q)
    Tm = np.linalg.lstsq(B, Z, rcond=None)[0]
    return np.linalg.lstsq(B, Tm.T, rcond=None)[0].T


def sketch_y_rows(L_rows, R_cols_p, n: int, rows, signs):
    """Eq. (4) for some rows of Y: f(L'(I,:) R'(:,p)) S(p,:), with R'(:,p) given
    for p = unique_rows(rows) in that (sorted) order."""
    p = unique_rows(rows)
    S = sparse_sign_matrix(n, rows, signs)[p, :].toarray()
    return trunc_log(np.asarray(L_rows) @ np.asarray(R_cols_p)) @ S


def sketch_z_parts(L_rows_p, R_cols_p, n: int, rows, signs):
    """Alg. 4 line 7 from the rows of L' and columns of R' at p = unique_rows(rows)."""
    p = unique_rows(rows)
    O = sparse_sign_matrix(n, rows, signs)[p, :].toarray()
    return O.T @ trunc_log(np.asarray(L_rows_p) @ np.asarray(R_cols_p)) @ O


# ---------------------------------------------------------------------------
# The general (non-symmetric) single pass, Eqs. (5)-(10): four sparse-sign
# test matrices C, S (n x h) and H, O (n x l) for a target f(LR) that need
# not be symmetric (L: n x k, R: k x n given).

def sketch_general_dense(L, R, C, S, H, O):
    """Eq. (5) by its definition on a dense F = f(LR) (small n only):
    K = F^T C, Y = F S, Z = H^T F O."""
    F = trunc_log(np.asarray(L) @ np.asarray(R))
    return F.T @ C, F @ S, H.T @ F @ O


def sketch_general_sampled(L, R, c_rs, s_rs, h_rs, o_rs):
    """Eq. (5) visiting only the entries of f(LR) the test matrices touch (the
    column sampling of Eq. (4) applied to each product); each *_rs is a
    (rows, signs) pair of a test matrix.
      K = f(L(p_C, :) R)^T C(p_C, :)
      Y = f(L R(:, p_S)) S(p_S, :)
      Z = H(p_H, :)^T f(L(p_H, :) R(:, p_O)) O(p_O, :)"""
    L = np.asarray(L, np.float64)
    R = np.asarray(R, np.float64)
    n = L.shape[0]

    def dense_rows(rs):
        p = unique_rows(rs[0])
        return p, sparse_sign_matrix(n, rs[0], rs[1])[p, :].toarray()

    pC, Cp = dense_rows(c_rs)
    pS, Sp = dense_rows(s_rs)
    pH, Hp = dense_rows(h_rs)
    pO, Op = dense_rows(o_rs)
    K = trunc_log(L[pC, :] @ R).T @ Cp
    Y = trunc_log(L @ R[:, pS]) @ Sp
    Z = Hp.T @ trunc_log(L[pH, :] @ R[:, pO]) @ Op
    return K, Y, Z


def single_pass_svd_general(K, Y, Z, H, O, d: int):
    """Eqs. (6)-(10) given the sketches: P = orth(K), Q = orth(Y);
    W = (H^T Q)^+ Z (P^T O)^+ by two least-squares solves; [U^, Sigma, V^] =
    svd(W); U_d = Q U^(:, 1:d), V_d = P V^(:, 1:d), Sigma_d.  H and O may be
    sparse."""
    P, _ = np.linalg.qr(K, mode="reduced")
    Q, _ = np.linalg.qr(Y, mode="reduced")
    B1 = np.asarray(H.T @ Q)           # l x h
    B2 = np.asarray(O.T @ P)           # l x h, (P^T O)^T
    Tm = np.linalg.lstsq(B1, Z, rcond=None)[0]           # (H^T Q) T = Z        (h x l)
    W = np.linalg.lstsq(B2, Tm.T, rcond=None)[0].T        # W (P^T O) = T        (h x h)
    Uh, sig, Vh = np.linalg.svd(W)
    return Q @ Uh[:, :d], sig[:d], P @ Vh.T[:, :d], W


# ---------------------------------------------------------------------------
# The full-visit reading of Alg. 3: the z nonzeros of a test matrix in every
# ROW (one set per vertex), so every entry of f(L'R') enters the sketches.

def sparse_sign_rows_matrix(n: int, width: int, cols_idx: np.ndarray, signs: np.ndarray) -> sp.csr_matrix:
    """The n x width test matrix with z nonzeros per row, entries +-1/sqrt(z)."""
    n_, z = cols_idx.shape
    r_idx = np.repeat(np.arange(n_), z)
    vals = signs.ravel().astype(np.float64) / np.sqrt(z)
    return sp.csr_matrix((vals, (r_idx, cols_idx.ravel().astype(np.int64))), shape=(n, width))


def sketch_fullvisit(Lp, Rp, s_cols, s_signs, o_cols, o_signs, h: int, l: int, row_block: int = 2048):
    """Y = f(L'R') S and Z = O^T f(L'R') O by their definitions, every entry of
    f(L'R') formed (row blocks of it at a time, so that no n x n array is
    held): Y[blk] = f(L'[blk] R') S, Z = sum_blk O[blk]^T (f(L'[blk] R') O)."""
    Lp = np.asarray(Lp, np.float64)
    Rp = np.asarray(Rp, np.float64)
    n = Lp.shape[0]
    S = sparse_sign_rows_matrix(n, h, s_cols, s_signs)
    O = sparse_sign_rows_matrix(n, l, o_cols, o_signs)
    Y = np.zeros((n, h))
    Z = np.zeros((l, l))
    for r0 in range(0, n, row_block):
        F = trunc_log(Lp[r0:r0 + row_block] @ Rp)
        Y[r0:r0 + row_block] = np.asarray(S.T @ F.T).T
        Z += np.asarray(O[r0:r0 + row_block].T @ np.asarray(O.T @ F.T).T)
    return Y, Z
