"""Pins for the oracle's general (non-symmetric) single pass, Eqs. (5)-(10):
exact recovery of a non-symmetric matrix of exact low rank (Eqs. 7-10 hold
with equality), the column-sampled sketches against their dense definition,
and the reduction to the symmetric form of Alg. 4 when C = S and H = O.
CPU only."""
import numpy as np

import synth
from oracle import sketch as sk, netmf, metrics


def _tests(n, h, l, z, seed):
    rs = [synth.sparse_sign(n, c, z, seed + i) for i, c in enumerate((h, h, l, l))]
    return rs, [sk.sparse_sign_dense(n, *x) for x in rs]


def test_general_exact_low_rank():
    # X = A B of rank r <= h, not symmetric: Q W P^T = X exactly, so its
    # singular values and singular subspaces are recovered
    rng = np.random.default_rng(1)
    n, r, h, l, z = 400, 7, 24, 90, 4
    X = rng.standard_normal((n, r)) @ rng.standard_normal((r, n))
    _, (C, S, H, O) = _tests(n, h, l, z, 10)
    U, sig, V, W = sk.single_pass_svd_general(X.T @ C, X @ S, H.T @ X @ O, H, O, r)
    ref = np.linalg.svd(X, compute_uv=False)[:r]
    assert np.allclose(sig, ref, rtol=1e-10)
    assert np.abs(U @ np.diag(sig) @ V.T - X).max() < 1e-10 * np.abs(X).max()
    # a transposed K (the row sketch taken from X instead of X^T) breaks it
    U2, sig2, V2, _ = sk.single_pass_svd_general(X @ C, X @ S, H.T @ X @ O, H, O, r)
    assert np.abs(U2 @ np.diag(sig2) @ V2.T - X).max() > 1e-3 * np.abs(X).max()


def test_general_sampled_equals_dense():
    rng = np.random.default_rng(2)
    n, k, h, l, z = 300, 9, 16, 48, 4
    L = rng.standard_normal((n, k))
    R = rng.standard_normal((k, n)) * 0.8 + 0.3
    rs, dense = _tests(n, h, l, z, 20)
    Kd, Yd, Zd = sk.sketch_general_dense(L, R, *dense)
    Ks, Ys, Zs = sk.sketch_general_sampled(L, R, *rs)
    for a, b in ((Kd, Ks), (Yd, Ys), (Zd, Zs)):
        assert metrics.rel_fro(b, a) < 1e-13


def test_general_reduces_to_symmetric():
    # f(L'R') of a graph is symmetric; with C = S and H = O the general pass
    # computes P = Q and the same W as Alg. 4
    rowptr, colidx = synth.sbm([60, 60, 60], 0.15, 0.02, 4)
    A = netmf.adjacency(rowptr, colidx)
    n = A.shape[0]
    from oracle import freigs as fr
    X = netmf.modified_laplacian(A, 0.5)
    U, lam = fr.freigs(X, synth.gaussian_block(n, 40, 5).astype(np.float64), 32, 2)
    Lp, Rp, _ = netmf.eq11_factors(U, lam, netmf.degrees(A), netmf.volume(A), 0.5, 10, 1.0)
    (rS, sS), (rO, sO) = synth.sparse_sign(n, 24, 4, 6), synth.sparse_sign(n, 80, 4, 7)
    S, O = sk.sparse_sign_dense(n, rS, sS), sk.sparse_sign_dense(n, rO, sO)
    K, Y, Z = sk.sketch_general_dense(Lp, Rp, S, S, O, O)
    Ug, sg, Vg, _ = sk.single_pass_svd_general(K, Y, Z, O, O, 8)
    Us, ss, _, _, _ = sk.single_pass_svd(Y, Z, O, 8)
    assert np.allclose(sg, ss, rtol=1e-8)
    assert metrics.rel_fro((Ug * sg) @ Ug.T, (Us * ss) @ Us.T) < 1e-8
