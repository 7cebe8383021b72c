"""Pins for the spectral-propagation oracle (Alg. 6 line 6): Chebyshev
coefficients against closed forms (polynomials, the Bessel series of exp),
the three-term recurrence against an eigendecomposition of L, and the
complete graph's closed form.  CPU only."""
import numpy as np
import pytest
from scipy.special import iv

import synth
from oracle import netmf, propagation as pg


def test_coeffs_reproduce_polynomials():
    # an interpolant of degree p reproduces every polynomial of degree <= p:
    # T_3(x) has coefficients e_3, and x^2 = (T_0 + T_2) / 2   (x = lambda - 1)
    c = pg.chebyshev_coeffs(lambda lam: 4 * (lam - 1) ** 3 - 3 * (lam - 1), 10)
    assert np.allclose(c, np.eye(11)[3], atol=1e-14)
    c = pg.chebyshev_coeffs(lambda lam: (lam - 1) ** 2, 10)
    assert np.allclose(c, [0.5, 0, 0.5] + [0] * 8, atol=1e-14)


@pytest.mark.parametrize("a", [0.3, 0.7, 1.5])
def test_coeffs_of_exp_are_bessel(a):
    # e^(a cos t) = I_0(a) + 2 sum_r I_r(a) cos(r t), so exp(a x) has the
    # Chebyshev coefficients I_0(a), 2 I_r(a); interpolation at p + 1 points
    # folds each coefficient beyond p onto one below, so they differ by at most
    # the tail sum_{j > p} 2 I_j(a)
    p = 10
    c = pg.chebyshev_coeffs(lambda lam: np.exp(a * (lam - 1)), p)
    exact = np.array([iv(0, a)] + [2 * iv(r, a) for r in range(1, p + 1)])
    tail = sum(2 * iv(j, a) for j in range(p + 1, 60))
    assert np.abs(c - exact).max() <= tail + 1e-15


def test_interpolant_matches_filter_at_nodes():
    g = pg.band_pass(0.5, 0.2)
    p = 10
    c = pg.chebyshev_coeffs(g, p)
    x = np.cos(np.pi * (np.arange(p + 1) + 0.5) / (p + 1))
    assert np.allclose(pg.chebyshev_eval(c, x), g(1 + x), rtol=1e-13, atol=0)
    # the band-pass at its quoted settings: peak e^(theta/2) at lambda = mu
    assert g(0.2) == pytest.approx(np.exp(0.25))


def _graph_with_isolated():
    rowptr, colidx = synth.sbm([30, 25, 20], 0.25, 0.03, 5)
    rowptr = np.concatenate([rowptr, [rowptr[-1]] * 2])  # two isolated vertices
    return netmf.adjacency(rowptr, colidx)


def test_recurrence_equals_eigendecomposition():
    # the same polynomial of L evaluated two ways: the recurrence on the sparse
    # L - I, and p(lambda) applied to the eigenvalues of L (through the
    # symmetric D^-1/2 A D^-1/2); isolated vertices get p(1)
    A = _graph_with_isolated()
    E = np.random.default_rng(0).standard_normal((A.shape[0], 6))
    c = pg.chebyshev_coeffs(pg.band_pass(0.5, 0.2), 10)
    fast = pg.propagate(A, E, c)
    ref = pg.propagate_dense_eig(A, E, lambda lam: pg.chebyshev_eval(c, lam - 1))
    assert np.abs(fast - ref).max() <= 1e-11 * np.abs(ref).max()
    assert np.allclose(fast[-2:], pg.chebyshev_eval(c, 0.0) * E[-2:], rtol=1e-14)


def test_complete_graph_closed_form():
    # K_n: L = I - (J - I)/(n - 1) has eigenvalue 0 on the constant vector and
    # n/(n - 1) on its complement, so p(L) E = p(0) P E + p(n/(n-1)) (E - P E)
    # with P the projector onto constants
    n = 9
    A = netmf.adjacency(*synth.complete(n))
    E = np.random.default_rng(1).standard_normal((n, 4))
    c = pg.chebyshev_coeffs(pg.band_pass(0.5, 0.2), 10)
    PE = np.repeat(E.mean(axis=0, keepdims=True), n, axis=0)
    expect = pg.chebyshev_eval(c, -1.0) * PE + pg.chebyshev_eval(c, n / (n - 1) - 1) * (E - PE)
    assert np.allclose(pg.propagate(A, E, c), expect, rtol=1e-12, atol=1e-14)


def test_high_degree_converges_to_filter():
    # the interpolant of the smooth band-pass converges fast: at p = 40 the
    # propagated block equals g(L) E from the eigendecomposition
    A = _graph_with_isolated()
    E = np.random.default_rng(2).standard_normal((A.shape[0], 3))
    g = pg.band_pass(0.5, 0.2)
    ref = pg.propagate_dense_eig(A, E, g)
    assert np.abs(pg.propagate(A, E, pg.chebyshev_coeffs(g, 40)) - ref).max() <= 1e-10 * np.abs(ref).max()
    # and p = 10 is already close (max |p - g| on [0, 2] is small)
    lam = np.linspace(0, 2, 2001)
    err10 = np.abs(pg.chebyshev_eval(pg.chebyshev_coeffs(g, 10), lam - 1) - g(lam)).max()
    assert err10 < 1e-6
