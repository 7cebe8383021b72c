"""Alg. 6 lines 1-5 (SketchNE without spectral propagation) and Alg. 1 (NetMF).

``sketchne`` runs the method step by step on given random realizations
(start block Omega, test matrices S and O), so its output can be compared
with another implementation that consumed the same realizations.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import netmf, freigs as fr, sketch as sk


@dataclass
class Params:
    alpha: float = 0.5
    T: int = 10
    b: float = 1.0
    k: int = 128
    s_eig: int = 32
    q: int = 2
    d: int = 32
    h: int = 80
    l: int = 1032
    z: int = 8


def eig_step(A, Omega, p: Params):
    """Alg. 6 line 1: freigs on D^-alpha A D^-alpha."""
    X = netmf.modified_laplacian(A, p.alpha)
    return fr.freigs(X, Omega, p.k, p.q)


def factor_step(A, U, lam, p: Params):
    """Alg. 6 lines 2-3."""
    deg = netmf.degrees(A)
    return netmf.eq11_factors(U, lam, deg, netmf.volume(A), p.alpha, p.T, p.b)


def sketch_step(Lp, Rp, S_rows, S_signs, O_rows, O_signs):
    """Alg. 4 lines 4 and 7 (Eq. 4 column sampling)."""
    Y = sk.sketch_y_sampled(Lp, Rp, S_rows, S_signs)
    Z = sk.sketch_z_sampled(Lp, Rp, O_rows, O_signs)
    return Y, Z


def embed_step(Y, Z, O_rows, O_signs, d: int):
    """Alg. 4 lines 5, 8-10 and Alg. 6 line 5: E = U_d Sigma_d^(1/2)."""
    n = Y.shape[0]
    O = sk.sparse_sign_matrix(n, O_rows, O_signs)
    Ud, sig, _, _, _ = sk.single_pass_svd(Y, Z, O, d)
    return Ud * np.sqrt(sig)[None, :], sig


def sketchne(A, p: Params, Omega, S_rows, S_signs, O_rows, O_signs):
    U, lam = eig_step(A, Omega, p)
    Lp, Rp, _ = factor_step(A, U, lam, p)
    Y, Z = sketch_step(Lp, Rp, S_rows, S_signs, O_rows, O_signs)
    E, sig = embed_step(Y, Z, O_rows, O_signs, p.d)
    return {"U": U, "lam": lam, "Lp": Lp, "Rp": Rp, "Y": Y, "Z": Z, "E": E, "sigma": sig}


def netmf_exact(A, k: int, d: int, T: int, b: float):
    """Alg. 1: exact eigendecomposition of D^-1/2 A D^-1/2 (top k by |lambda|),
    L and R of Problem 1, exact rank-d SVD of f(LR), E = U_d Sigma_d^(1/2)."""
    X = netmf.modified_laplacian(A, 0.5).toarray()
    lam, V = np.linalg.eigh(X)
    order = fr.sort_by_abs_desc(lam)[:k]
    lam, V = lam[order], V[:, order]
    F = netmf.trunc_log(netmf.eq2_matrix(A, V, lam, T, b))
    Uf, sig, _ = np.linalg.svd(F)
    return Uf[:, :d] * np.sqrt(sig[:d])[None, :], sig[:d]
