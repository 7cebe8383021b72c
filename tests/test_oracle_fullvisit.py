"""Pins for the oracle's full-visit sketch (z nonzeros per row of the test
matrices): a permutation test matrix returns the columns of f(L'R')
exactly, the row-blocked evaluation equals one dense product, and the single
pass recovers an exactly low-rank symmetric matrix from full-visit sketches
(Eqs. 7-10 do not depend on where the nonzeros sit).  CPU only."""
import numpy as np

import synth
from oracle import sketch as sk, netmf, metrics


def test_permutation_selects_columns():
    rng = np.random.default_rng(1)
    n, k = 64, 5
    Lp = rng.random((n, k))
    Rp = rng.standard_normal((k, n)) * 0.6 + 0.3
    perm = rng.permutation(n)
    cols = perm[:, None].astype(np.int32)          # row j -> column perm[j], one nonzero
    signs = np.ones((n, 1), np.int8)
    Y, _ = sk.sketch_fullvisit(Lp, Rp, cols, signs, cols, signs, n, n)
    F = netmf.trunc_log(Lp @ Rp)
    assert np.array_equal(Y[:, perm], F)           # exact: one term per entry


def test_blocked_equals_dense():
    rng = np.random.default_rng(2)
    n, k, h, l, z = 300, 6, 20, 50, 4
    Lp = rng.random((n, k))
    Rp = rng.standard_normal((k, n)) * 0.5 + 0.2
    sc, ss = synth.sparse_sign_rows(n, h, z, 3)
    oc, os_ = synth.sparse_sign_rows(n, l, z, 4)
    Y, Z = sk.sketch_fullvisit(Lp, Rp, sc, ss, oc, os_, h, l, row_block=37)
    F = netmf.trunc_log(Lp @ Rp)
    S = sk.sparse_sign_rows_matrix(n, h, sc, ss).toarray()
    O = sk.sparse_sign_rows_matrix(n, l, oc, os_).toarray()
    assert metrics.rel_fro(Y, F @ S) < 1e-13
    assert metrics.rel_fro(Z, O.T @ F @ O) < 1e-13


def test_single_pass_exact_with_row_sparse_tests():
    rng = np.random.default_rng(5)
    n, r, h, l, z = 500, 6, 24, 90, 4
    V = np.linalg.qr(rng.standard_normal((n, r)))[0]
    X = V @ np.diag(np.linspace(4, -2, r)) @ V.T
    sc, ss = synth.sparse_sign_rows(n, h, z, 6)
    oc, os_ = synth.sparse_sign_rows(n, l, z, 7)
    S = sk.sparse_sign_rows_matrix(n, h, sc, ss)
    O = sk.sparse_sign_rows_matrix(n, l, oc, os_)
    Y = np.asarray(S.T @ X.T).T
    Z = np.asarray(O.T @ np.asarray(O.T @ X.T).T)
    U, sig, _, _, _ = sk.single_pass_svd(Y, Z, O, r)
    assert np.allclose(sig, np.sort(np.abs(np.linspace(4, -2, r)))[::-1], rtol=1e-10)
