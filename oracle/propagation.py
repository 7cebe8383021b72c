"""Spectral propagation, Alg. 6 line 6: E <- sum_{r=0..p} c_r T_r(...) E.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper states the step as a degree-p polynomial in the random-walk
Laplacian L = I - D^-1 A with "Chebyshev coefficients" c_r and p = 10, and
takes the technique from ProNE, whose settings it quotes as theta = 0.5 and
mu = 0.2.  The coefficients themselves are not given.  Reading used here:

* the filter is ProNE's band-pass on the Laplacian spectrum lambda in [0, 2],
      g(lambda) = exp(-theta/2 * ((lambda - mu)^2 - 1));
* the polynomial is g's Chebyshev interpolant of degree p on [0, 2]: with
  x = lambda - 1 in [-1, 1], p(lambda) = sum_r c_r T_r(lambda - 1), where T_r
  is the Chebyshev polynomial of the first kind and c_r interpolates g at the
  p + 1 Chebyshev points x_j = cos(pi (j + 1/2) / (p + 1));
* E_out = sum_r c_r T_r(L - I) E, evaluated by the three-term recurrence
  T_0 E = E, T_1 E = (L - I) E, T_{r+1} E = 2 (L - I) T_r E - T_{r-1} E.
  L - I = -D^-1 A has its spectrum in [-1, 1], where the recurrence is stable.
* An isolated vertex has D^-1 taken as 0 (as everywhere in this oracle), so
  its row of L - I is zero and its output row is p(1) E_i (T_r(0) = cos(r pi/2)).

Each function names the passage it follows; parity of the coefficients and of
the propagation is pinned in tests/test_oracle_propagation.py.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .netmf import degrees, deg_power


def band_pass(theta: float = 0.5, mu: float = 0.2):
    """ProNE's band-pass filter g(lambda) (the reading above)."""
    return lambda lam: np.exp(-0.5 * theta * ((np.asarray(lam, np.float64) - mu) ** 2 - 1.0))


def chebyshev_coeffs(g, p: int) -> np.ndarray:
    """c_0..c_p of the degree-p Chebyshev interpolant of g on lambda in [0, 2]
    (nodes x_j = cos(pi (j + 1/2) / (p + 1)), lambda_j = 1 + x_j):
        c_r = (2 - [r == 0]) / (p + 1) * sum_j g(lambda_j) cos(r pi (j + 1/2) / (p + 1))."""
    j = np.arange(p + 1)
    ang = np.pi * (j + 0.5) / (p + 1)
    gv = g(1.0 + np.cos(ang))
    c = np.array([np.sum(gv * np.cos(r * ang)) for r in range(p + 1)]) * (2.0 / (p + 1))
    c[0] *= 0.5
    return c


def chebyshev_eval(c, x) -> np.ndarray:
    """sum_r c_r T_r(x) for scalar or array x in [-1, 1] (T_r(cos t) = cos(r t))."""
    x = np.asarray(x, np.float64)
    t = np.arccos(np.clip(x, -1.0, 1.0))
    return sum(cr * np.cos(r * t) for r, cr in enumerate(c))


def walk_laplacian_shifted(A) -> sp.csr_matrix:
    """L - I = -D^-1 A (Alg. 6 line 6, with L = I - D^-1 A), sparse."""
    dinv = deg_power(degrees(A), -1.0)
    return (-(sp.diags(dinv) @ A)).tocsr()


def propagate(A, E, c) -> np.ndarray:
    """Alg. 6 line 6: sum_r c_r T_r(L - I) E by the three-term recurrence."""
    M = walk_laplacian_shifted(A)
    E = np.asarray(E, np.float64)
    t_prev = E
    out = c[0] * t_prev
    if len(c) == 1:
        return out
    t_cur = M @ E
    out = out + c[1] * t_cur
    for r in range(2, len(c)):
        t_prev, t_cur = t_cur, 2.0 * (M @ t_cur) - t_prev
        out = out + c[r] * t_cur
    return out


def propagate_dense_eig(A, E, fn) -> np.ndarray:
    """fn(L) E through the eigendecomposition of L (small graphs only): on the
    non-isolated vertices L = D^-1/2 (I - D^-1/2 A D^-1/2) D^1/2, so
    fn(L) = D^-1/2 V fn(1 - nu) V^T D^1/2 with D^-1/2 A D^-1/2 = V diag(nu) V^T;
    an isolated vertex is an eigenvector of L with eigenvalue 1."""
    deg = degrees(A)
    E = np.asarray(E, np.float64)
    iso = deg == 0
    keep = ~iso
    out = np.zeros_like(E)
    out[iso] = fn(np.ones(1))[0] * E[iso]
    if keep.any():
        Ak = A[keep][:, keep].toarray()
        dk = deg[keep]
        Xs = Ak / np.sqrt(dk)[:, None] / np.sqrt(dk)[None, :]
        nu, V = np.linalg.eigh(Xs)
        F = (V * fn(1.0 - nu)[None, :]) @ V.T
        out[keep] = (F @ (np.sqrt(dk)[:, None] * E[keep])) / np.sqrt(dk)[:, None]
    return out
