"""Pins for the FP64 oracle: closed forms, exact identities, invariants and
brute force that a plausible mistake in the oracle would fail.

Nothing here re-types the oracle's formula; each check comes from a different
route to the same quantity (a closed form derived from Eq. 1, the full-rank
identity behind Eq. 11, Eq. 2 as the alpha = 1/2 case, the spectral facts the
paper relies on, or exact low-rank inputs for Alg. 4 / Alg. 5).
"""
from fractions import Fraction
from math import comb

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import netmf, freigs as fr, sketch as sk, metrics, pipeline


def A_of(g):
    return netmf.adjacency(*g)


# ---------------------------------------------------------------- Eq. (1)

def test_eq1_cycle_closed_form():
    # Cycle C_n with n > 2T: a random walk cannot wrap, so
    # (D^-1 A)^r_ij = binom(r, (r+delta)/2) / 2^r for r >= |delta|, r = delta mod 2,
    # vol = 2n and D^-1 = I/2, hence M_ij = n/(bT) * sum_r binom(r,(r+delta)/2)/2^r.
    n, T, b = 41, 10, 2.0
    M = netmf.netmf_matrix(A_of(synth.cycle(n)), T, b)
    for i in (0, 7):
        for j in range(n):
            delta = (j - i) % n
            if delta > n // 2:
                delta -= n
            s = Fraction(0)
            for r in range(1, T + 1):
                if r >= abs(delta) and (r - delta) % 2 == 0:
                    s += Fraction(comb(r, (r + delta) // 2), 2 ** r)
            expect = float(Fraction(n) / Fraction(b).limit_denominator() / T * s)
            assert M[i, j] == pytest.approx(expect, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("n,T", [(2, 1), (3, 2), (7, 5), (12, 10)])
def test_eq1_complete_graph_closed_form(n, T):
    # K_n: D^-1 A = (J - I)/(n-1) has eigenvalue 1 on the all-ones vector and
    # mu = -1/(n-1) elsewhere, so (D^-1A)^r = J/n + mu^r (I - J/n).  With
    # D^-1 = I/(n-1) and vol = n(n-1):  off-diagonal M = (T - s)/(bT) and
    # diagonal M = (T + (n-1) s)/(bT), s = sum_{r=1..T} mu^r.
    b = 1.0
    M = netmf.netmf_matrix(A_of(synth.complete(n)), T, b)
    mu = Fraction(-1, n - 1)
    s = sum(mu ** r for r in range(1, T + 1))
    off = float((T - s) / T)
    diag = float((T + (n - 1) * s) / T)
    assert np.allclose(M[~np.eye(n, dtype=bool)], off, rtol=1e-13, atol=0)
    assert np.allclose(np.diag(M), diag, rtol=1e-13, atol=1e-15)
    if n == 2 and T == 1:
        assert M[0, 1] == pytest.approx(2.0) and M[0, 0] == pytest.approx(0.0, abs=1e-15)


def test_eq1_disjoint_union_blocks_zero():
    g = synth.disjoint_union(synth.complete(5), synth.cycle(9))
    F = netmf.trunc_log(netmf.netmf_matrix(A_of(g), 5, 1.0))
    assert np.all(F[:5, 5:] == 0) and np.all(F[5:, :5] == 0)
    assert np.abs(F - F.T).max() < 1e-12  # symmetric


# ---------------------------------------------------------------- Eq. (11)

def _small_graph(seed=3, n=60, isolated=True):
    rowptr, colidx = synth.sbm([20, 20, 20], 0.3, 0.05, seed)
    if isolated:  # append an isolated vertex
        rowptr = np.concatenate([rowptr, [rowptr[-1]]])
    return netmf.adjacency(rowptr, colidx)


@pytest.mark.parametrize("alpha", [0.3, 0.4, 0.5])
def test_eq11_full_rank_equals_eq1(alpha):
    # With the full eigendecomposition D^-a A D^-a = U Lambda U^T (k = n),
    # D^-1 A = D^(-1+a) U Lambda U^T D^a, so every term (D^-1A)^r D^-1 equals
    # D^(-1+a) U Lambda K^(r-1) U^T D^(-1+a) exactly: Eq. (11) reproduces Eq. (1).
    A = _small_graph()
    T, b = 10, 1.0
    X = netmf.modified_laplacian(A, alpha).toarray()
    lam, U = np.linalg.eigh(X)
    Lp, Rp, _ = netmf.eq11_factors(U, lam, netmf.degrees(A), netmf.volume(A), alpha, T, b)
    M = netmf.netmf_matrix(A, T, b)
    assert metrics.rel_fro(Lp @ Rp, M) < 1e-11


def test_eq11_alpha_half_is_eq2():
    # alpha = 1/2: K = U^T U Lambda = Lambda for orthonormal U, so
    # Lambda sum K^(r-1) = sum Lambda^r and Eq. (11) is Eq. (2).
    A = _small_graph(isolated=False)
    X = netmf.modified_laplacian(A, 0.5).toarray()
    lam, U = np.linalg.eigh(X)
    order = fr.sort_by_abs_desc(lam)[:12]
    lam, U = lam[order], U[:, order]
    Lp, Rp, Kmat = netmf.eq11_factors(U, lam, netmf.degrees(A), netmf.volume(A), 0.5, 7, 1.5)
    assert np.abs(Kmat - np.diag(lam)).max() < 1e-12
    assert metrics.rel_fro(Lp @ Rp, netmf.eq2_matrix(A, U, lam, 7, 1.5)) < 1e-12


def test_eq11_core_symmetric():
    # Lambda (sum K^(r-1)) is symmetric: Lambda (G Lambda)^j is a palindrome in
    # the symmetric matrices G = U^T D^(-1+2a) U and Lambda, so L'R' is symmetric.
    A = _small_graph()
    rng = np.random.default_rng(0)
    U = np.linalg.qr(rng.standard_normal((A.shape[0], 9)))[0]
    lam = rng.uniform(-1, 1, 9)
    Lp, Rp, Kmat = netmf.eq11_factors(U, lam, netmf.degrees(A), netmf.volume(A), 0.35, 10, 1.0)
    C = netmf.core_matrix(lam, Kmat, 10)
    assert np.abs(C - C.T).max() <= 1e-12 * np.abs(C).max()
    X = Lp @ Rp
    assert np.abs(X - X.T).max() <= 1e-12 * np.abs(X).max()


# ---------------------------------------------------------------- spectra

def test_lambda_max_is_one_and_bipartite_min():
    A = _small_graph(isolated=False)
    lam = np.linalg.eigvalsh(netmf.modified_laplacian(A, 0.5).toarray())
    assert lam[-1] == pytest.approx(1.0, abs=1e-12)
    # eigenvector of eigenvalue 1 is proportional to D^(1/2) 1
    lam2, V = np.linalg.eigh(netmf.modified_laplacian(A, 0.5).toarray())
    v = np.sqrt(netmf.degrees(A))
    v /= np.linalg.norm(v)
    assert abs(abs(V[:, -1] @ v) - 1) < 1e-12
    lam_c = np.linalg.eigvalsh(netmf.modified_laplacian(A_of(synth.cycle(16)), 0.5).toarray())
    assert lam_c[0] == pytest.approx(-1.0, abs=1e-12)
    lam_o = np.linalg.eigvalsh(netmf.modified_laplacian(A_of(synth.cycle(15)), 0.5).toarray())
    assert lam_o[0] > -1.0 + 1e-3


def test_freigs_exact_on_low_rank():
    # Union of 3 complete bipartite graphs: D^-1/2 A D^-1/2 has rank 6 with
    # eigenvalues +1 (x3) and -1 (x3).  With k + s = 6 the range of X Omega
    # is the whole range of X, so Alg. 5 is exact for any q.  (k + s > rank
    # would make X Omega rank deficient, which eigSVD cannot orthonormalise.)
    gs = []
    for a, bb in [(3, 5), (4, 4), (2, 7)]:
        iu, ju = np.meshgrid(np.arange(a), np.arange(a, a + bb), indexing="ij")
        gs.append(synth.csr_from_edges(a + bb, iu.ravel(), ju.ravel()))
    g = gs[0]
    for h in gs[1:]:
        g = synth.disjoint_union(g, h)
    A = A_of(g)
    X = netmf.modified_laplacian(A, 0.5)
    Om = synth.gaussian_block(A.shape[0], 6, 5).astype(np.float64)
    for q in (0, 2):
        U, lam = fr.freigs(X, Om, 6, q)
        assert np.allclose(np.sort(lam), [-1, -1, -1, 1, 1, 1], atol=1e-12)
        assert np.abs(U @ np.diag(lam) @ U.T - X.toarray()).max() < 1e-12


def test_freigs_converges_to_dense_eigh():
    # On an SBM with 8 planted blocks the top 8 eigenvalues are separated from
    # the bulk; enough power iterations reproduce the dense eigensolver.
    A = A_of(synth.sbm([64] * 8, 0.3, 0.01, 11))
    X = netmf.modified_laplacian(A, 0.5)
    lam_ref = np.linalg.eigvalsh(X.toarray())
    top = lam_ref[np.argsort(-np.abs(lam_ref))][:8]
    Om = synth.gaussian_block(A.shape[0], 24, 7).astype(np.float64)
    U, lam = fr.freigs(X, Om, 8, 12)
    assert lam[0] == pytest.approx(1.0, abs=1e-10)
    assert np.allclose(lam, top, atol=1e-8)


def test_freigs_basis_invariance():
    # eigSVD and Householder QR give the same Ritz pairs (only span(Q) matters).
    A = A_of(synth.sbm([50] * 4, 0.2, 0.02, 2))
    X = netmf.modified_laplacian(A, 0.4)
    Om = synth.gaussian_block(A.shape[0], 30, 9).astype(np.float64)
    U1, l1 = fr.freigs(X, Om, 20, 2, orth=fr.orth_eigsvd)
    U2, l2 = fr.freigs(X, Om, 20, 2, orth=fr.orth_qr)
    assert np.abs(l1 - l2).max() < 1e-11
    assert metrics.sin_theta_fro(U1, U2) < 1e-9


def test_lemma4_with_exact_eigenpairs():
    # Lemma 4 with the exact top-k pairs (epsilon = 0):
    # ||D^-1/2 A D^-1/2 - D^(-1/2+a) U L U^T D^(-1/2+a)||_F <= d_min^(-1+2a) sqrt(tail)
    A = _small_graph(isolated=False)
    deg = netmf.degrees(A)
    Xh = netmf.modified_laplacian(A, 0.5).toarray()
    for alpha in (0.3, 0.4, 0.5):
        Xa = netmf.modified_laplacian(A, alpha).toarray()
        lam, V = np.linalg.eigh(Xa)
        order = fr.sort_by_abs_desc(lam)
        lam, V = lam[order], V[:, order]
        k = 15
        Dk = netmf.deg_power(deg, -0.5 + alpha)
        approx = (Dk[:, None] * V[:, :k]) @ np.diag(lam[:k]) @ (V[:, :k].T * Dk[None, :])
        lhs = np.linalg.norm(Xh - approx)
        rhs = deg.min() ** (-1 + 2 * alpha) * np.sqrt(np.sum(lam[k:] ** 2))
        assert lhs <= rhs * (1 + 1e-12)


# ---------------------------------------------------------------- truncated log

def test_trunc_log_properties():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-5, 5, 10000), rng.lognormal(0, 3, 10000)])
    f = netmf.trunc_log(x)
    assert np.all(f >= 0)
    assert np.all(f[x <= 1] == 0)
    assert netmf.trunc_log(np.e) == pytest.approx(1.0)
    y = x + rng.normal(0, 0.5, len(x))
    assert np.all(np.abs(netmf.trunc_log(y) - f) <= np.abs(y - x) + 1e-15)  # 1-Lipschitz


# ---------------------------------------------------------------- sketch (Alg. 3/4, Eq. 4)

def _factors(n=300, k=24, seed=4):
    A = A_of(synth.sbm([n // 3] * 3, 0.1, 0.01, seed))
    X = netmf.modified_laplacian(A, 0.5)
    Om = synth.gaussian_block(A.shape[0], k + 8, seed).astype(np.float64)
    U, lam = fr.freigs(X, Om, k, 2)
    Lp, Rp, _ = netmf.eq11_factors(U, lam, netmf.degrees(A), netmf.volume(A), 0.5, 10, 1.0)
    return A, Lp, Rp


def test_sketch_two_ways_agree():
    # Eq. (4): column sampling is exactly f(L'R') S.
    A, Lp, Rp = _factors()
    n = A.shape[0]
    rS, sS = synth.sparse_sign(n, 20, 8, 1)
    rO, sO = synth.sparse_sign(n, 40, 8, 2)
    S = sk.sparse_sign_dense(n, rS, sS)
    O = sk.sparse_sign_dense(n, rO, sO)
    Yd, Zd = sk.sketch_dense(Lp, Rp, S, O)
    Ys = sk.sketch_y_sampled(Lp, Rp, rS, sS)
    Zs = sk.sketch_z_sampled(Lp, Rp, rO, sO)
    assert metrics.rel_fro(Ys, Yd) < 1e-13
    assert metrics.rel_fro(Zs, Zd) < 1e-13
    assert np.abs(Zs - Zs.T).max() <= 1e-12 * np.abs(Zs).max()  # symmetric
    sub = np.array([0, 5, 17, 299])
    assert metrics.rel_fro(sk.sketch_y_sampled(Lp, Rp, rS, sS, row_subset=sub), Yd[sub]) < 1e-13


def test_sketch_selection_and_linearity():
    A, Lp, Rp = _factors()
    n = A.shape[0]
    F = netmf.trunc_log(Lp @ Rp)
    cols = np.array([[3], [77], [150], [299]], dtype=np.int32)
    Ysel = sk.sketch_y_sampled(Lp, Rp, cols, np.ones_like(cols, dtype=np.int8))
    assert np.abs(Ysel - F[:, cols.ravel()]).max() < 1e-12  # z = 1 selects columns
    r1, s1 = synth.sparse_sign(n, 6, 8, 8)
    r2, s2 = synth.sparse_sign(n, 6, 8, 9)
    y1 = sk.sketch_y_sampled(Lp, Rp, r1, s1)
    y2 = sk.sketch_y_sampled(Lp, Rp, r2, s2)
    Ssum = sk.sparse_sign_dense(n, r1, s1) + sk.sparse_sign_dense(n, r2, s2)
    assert metrics.rel_fro(y1 + y2, F @ Ssum) < 1e-13
    # O = S: Z = S^T Y
    Z = sk.sketch_z_sampled(Lp, Rp, r1, s1)
    assert metrics.rel_fro(Z, sk.sparse_sign_dense(n, r1, s1).T @ y1) < 1e-13


def test_single_pass_svd_exact_low_rank():
    # Alg. 4 lines 5, 8-10 with a symmetric X of exact rank r <= h and full
    # column rank O^T Q: Q W Q^T = X and the singular values are exact (Eqs. 7-10).
    rng = np.random.default_rng(3)
    n, r, h, l, d = 400, 12, 20, 60, 8
    V = np.linalg.qr(rng.standard_normal((n, r)))[0]
    mu = np.concatenate([np.linspace(5, 1, r // 2), -np.linspace(4.5, 0.5, r // 2)])
    X = V @ np.diag(mu) @ V.T
    rS, sS = synth.sparse_sign(n, h, 8, 1)
    rO, sO = synth.sparse_sign(n, l, 8, 2)
    S = sk.sparse_sign_dense(n, rS, sS)
    O = sk.sparse_sign_dense(n, rO, sO)
    Ud, sig, Vd, W, Q = sk.single_pass_svd(X @ S, O.T @ X @ O, O, d)
    assert np.abs(Q @ W @ Q.T - X).max() < 1e-10
    assert np.allclose(sig, np.sort(np.abs(mu))[::-1][:d], rtol=1e-10)


def test_pipeline_small_against_exact_netmf():
    # Method error context (not parity): on an SBM with q = 2 the SketchNE
    # embedding spans nearly the same subspace as exact NetMF (Alg. 1).
    A = A_of(synth.sbm([128] * 4, 0.1, 0.005, 21))
    n = A.shape[0]
    p = pipeline.Params(alpha=0.5, T=10, b=1.0, k=32, s_eig=16, q=2, d=8, h=32, l=200, z=8)
    Om = synth.gaussian_block(n, p.k + p.s_eig, 1).astype(np.float64)
    rS, sS = synth.sparse_sign(n, p.h, p.z, 2)
    rO, sO = synth.sparse_sign(n, p.l, p.z, 3)
    out = pipeline.sketchne(A, p, Om, rS, sS, rO, sO)
    E_ref, _ = pipeline.netmf_exact(A, p.k, p.d, p.T, p.b)
    # the 4 planted-block directions dominate both embeddings
    assert metrics.sin_theta_fro(out["E"][:, :4], E_ref[:, :4]) < 0.3
    # q = 2 at alpha = 1/2 is not converged (the paper's worst case for freigs),
    # so the top Ritz value is only close to the true eigenvalue 1.
    assert 1.0 - 1e-3 < out["lam"][0] <= 1.0 + 1e-12


def test_sparse_sign_matrix_structure():
    # Alg. 3: each column has exactly z nonzeros, at the drawn rows, equal to
    # sign/sqrt(z); so every column has unit 2-norm.
    n, h, z = 50, 7, 8
    rows, signs = synth.sparse_sign(n, h, z, 4)
    S = sk.sparse_sign_dense(n, rows, signs)
    assert np.all((S != 0).sum(axis=0) == z)
    for c in range(h):
        assert np.allclose(S[rows[c], c], signs[c] / np.sqrt(z))
    assert np.allclose(np.linalg.norm(S, axis=0), 1.0)


def test_principal_angle_metric():
    n = 10
    e = np.eye(n)
    for th in (0.0, 0.3, 1.2):
        b = np.cos(th) * e[:, 0] + np.sin(th) * e[:, 1]
        s = metrics.sin_principal_angles(e[:, [0, 5]], np.stack([b, e[:, 5]], 1))
        assert np.allclose(np.sort(s), np.sort([np.sin(th), 0.0]), atol=1e-12)


def test_eq11_row_subset_forms_match_full_factors():
    """The row-subset forms used at large n agree with the full factors."""
    rowptr, colidx = synth.chung_lu(3000, 2.2, 8, 1, 55)
    A = netmf.adjacency(rowptr, colidx)
    deg = netmf.degrees(A)
    rng = np.random.default_rng(2)
    U = np.linalg.qr(rng.standard_normal((3000, 12)))[0]
    lam = np.sort(rng.uniform(-1, 1, 12))[::-1]
    for alpha in (0.5, 0.4):
        Lp, Rp, K = netmf.eq11_factors(U, lam, deg, netmf.volume(A), alpha, 10, 1.0)
        K2 = netmf.eq11_kmat(U, lam, deg, alpha, block=700)
        assert np.allclose(K2, K, rtol=1e-12, atol=1e-14)
        idx = np.array([0, 5, 17, 2999])
        Lr, Rc = netmf.eq11_rows(U[idx], deg[idx], lam, K2, netmf.volume(A), alpha, 10, 1.0)
        assert np.allclose(Lr, Lp[idx], rtol=1e-12) and np.allclose(Rc, Rp[:, idx], rtol=1e-11, atol=1e-14)
    rows, signs = synth.sparse_sign(3000, 16, 4, 9)
    p = sk.unique_rows(rows)
    Lp, Rp, K = netmf.eq11_factors(U, lam, deg, netmf.volume(A), 0.5, 10, 1.0)
    sub = np.array([1, 2, 100, 2500])
    Y1 = sk.sketch_y_sampled(Lp, Rp, rows, signs, row_subset=sub)
    Y2 = sk.sketch_y_rows(Lp[sub], Rp[:, p], 3000, rows, signs)
    assert np.allclose(Y1, Y2, rtol=1e-13, atol=1e-15)
    Z1 = sk.sketch_z_sampled(Lp, Rp, rows, signs)
    Z2 = sk.sketch_z_parts(Lp[p], Rp[:, p], 3000, rows, signs)
    assert np.allclose(Z1, Z2, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- eigenpair order (Alg. 5, Lemma 4)

def test_sort_by_abs_desc_hand_permutation():
    # |lambda| descending (the order of Lemma 4), ties by lambda descending,
    # then by index; the expected permutation is written out by hand
    lam = np.array([0.5, -2.0, 2.0, -0.5, 1.0, -1.0, 0.0, 1.0])
    assert list(fr.sort_by_abs_desc(lam)) == [2, 1, 4, 7, 5, 0, 3, 6]
    # a spectrum dominated by negative values: signed order would differ everywhere
    lam = np.array([-0.9, 0.1, -0.7, 0.3, -0.99])
    assert list(fr.sort_by_abs_desc(lam)) == [4, 0, 2, 3, 1]


def test_freigs_orders_bipartite_spectrum_by_magnitude():
    # Even cycle C_10 at alpha = 1/2: D^-1/2 A D^-1/2 = A/2 has the eigenvalues
    # cos(2 pi j / 10): 1, -1 and +-cos(pi/5), +-cos(2 pi/5) twice each, none
    # zero.  With k + s = n the start block spans everything, so Alg. 5
    # returns the exact pairs; by magnitude the order is +-1, then the four
    # of modulus cos(pi/5), then the four of cos(2 pi/5) (a signed order
    # would put every negative value last).
    A = A_of(synth.cycle(10))
    X = netmf.modified_laplacian(A, 0.5)
    Om = synth.gaussian_block(10, 10, 3).astype(np.float64)
    U, lam = fr.freigs(X, Om, 10, 1)
    a, b = np.cos(np.pi / 5), np.cos(2 * np.pi / 5)
    # equal moduli are equal only up to rounding, so the tie rule (lambda
    # descending) is not checked here: each group of equal modulus must hold
    # exactly its signed values
    assert np.allclose(np.abs(lam), [1, 1, a, a, a, a, b, b, b, b], atol=1e-12)
    for lo, hi, vals in [(0, 2, [-1, 1]), (2, 6, [-a, -a, a, a]), (6, 10, [-b, -b, b, b])]:
        assert np.allclose(np.sort(lam[lo:hi]), vals, atol=1e-12)
    # the pair of eigenvalue -1 (one of the first two) is the alternating vector
    alt = np.array([1, -1] * 5) / np.sqrt(10)
    j = int(np.argmin(lam[:2]))
    assert abs(abs(U[:, j] @ alt) - 1) < 1e-12


# ---------------------------------------------------------------- Alg. 6 line 5 through embed_step

def test_embed_step_scales_by_sqrt_sigma():
    # Alg. 4 on a symmetric X = V diag(mu) V^T of exact rank r: its SVD is
    # U = V (columns sorted by |mu|), Sigma = |mu|.  Alg. 6 line 5 gives
    # E = U_d Sigma_d^(1/2), so E E^T = V_d |mu_d| V_d^T whatever the signs
    # of the singular vectors (E = U_d Sigma_d would give V_d mu_d^2 V_d^T).
    rng = np.random.default_rng(12)
    n, r, h, l, d = 300, 10, 24, 80, 6
    V = np.linalg.qr(rng.standard_normal((n, r)))[0]
    mu = np.array([6.0, -5.0, 4.0, -3.5, 3.0, 2.5, -2.0, 1.5, 1.0, 0.5])
    X = V @ np.diag(mu) @ V.T
    rS, sS = synth.sparse_sign(n, h, 8, 5)
    rO, sO = synth.sparse_sign(n, l, 8, 6)
    S = sk.sparse_sign_dense(n, rS, sS)
    O = sk.sparse_sign_dense(n, rO, sO)
    E, sig = pipeline.embed_step(X @ S, O.T @ X @ O, rO, sO, d)
    order = np.argsort(-np.abs(mu))[:d]
    expect = V[:, order] @ np.diag(np.abs(mu[order])) @ V[:, order].T
    assert np.allclose(sig, np.abs(mu[order]), rtol=1e-10)
    assert np.abs(E @ E.T - expect).max() < 1e-10
