"""Alg. 5 (freigs): fast randomized eigendecomposition of a sparse symmetric X.

Readings:
* eigSVD is not defined in the paper (it cites frPCA).  It is read as: Gram
  matrix G = B^T B, symmetric eigendecomposition G = V D V^T, Q = B V D^(-1/2).
  Alg. 5 only ever uses the Q output, and its result depends on span(Q) alone
  (the power step maps spans to spans and Ritz pairs do not depend on the
  basis), so any orthonormalisation gives the same U and Lambda in exact
  arithmetic; ``orth_qr`` is provided to check exactly that.
* Line 6 computes X(XQ): two products, no orthonormalisation in between.
* Line 10 leaves the eigenpair order open; pairs are sorted by descending
  absolute eigenvalue (the order the error bound of Lemma 4 refers to), ties
  by descending eigenvalue, then by original index.
* The oversampling s is a parameter; the start block Omega is an input.
"""
from __future__ import annotations

import numpy as np


def orth_eigsvd(B: np.ndarray) -> np.ndarray:
    G = B.T @ B
    dvals, V = np.linalg.eigh(G)
    return (B @ V) / np.sqrt(dvals)[None, :]


def orth_qr(B: np.ndarray) -> np.ndarray:
    Q, _ = np.linalg.qr(B, mode="reduced")
    return Q


def sort_by_abs_desc(lam: np.ndarray) -> np.ndarray:
    """Permutation ordering eigenvalues by |lambda| desc, then lambda desc, then index."""
    idx = np.arange(len(lam))
    return np.lexsort((idx, -lam, -np.abs(lam)))


def freigs(X, Omega: np.ndarray, k: int, q: int, orth=orth_eigsvd, return_basis=False):
    """Alg. 5 with a given start block Omega (n x (k+s)).

    Returns U (n x k) and lambda (k), sorted by |lambda| descending."""
    Omega = np.asarray(Omega, dtype=np.float64)
    Y = X @ Omega                      # line 4: sketch
    Q = orth(Y)                        # line 5
    for _ in range(q):                 # lines 6-8: power iteration
        Q = orth(X @ (X @ Q))
    XQ = X @ Q
    S = Q.T @ XQ                       # line 9: reduced matrix
    S = 0.5 * (S + S.T)
    lam, Uh = np.linalg.eigh(S)        # line 10: full eigendecomposition
    order = sort_by_abs_desc(lam)
    lam, Uh = lam[order], Uh[:, order]
    U = Q @ Uh                         # line 11
    if return_basis:
        return U[:, :k], lam[:k], Q
    return U[:, :k], lam[:k]
