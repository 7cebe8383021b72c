"""Learned warm start for Alg. 5: per-vertex features, a 3-layer MLP, its
subspace loss, analytic gradients and the Adam update, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component: Alg. 5 starts from a Gaussian block.
This module defines the learned start used as a replacement for the first k
columns of that block:

* features (per vertex i, before standardisation)
      phi_i = [ log max(deg_i, 1), (X^3 g)_i1 .. (X^3 g)_i4, (X^4 g)_i1 .. (X^4 g)_i3 ]
  with X = D^-a A D^-a (the matrix of Alg. 5) and g an n x 4 block of
  Rademacher vectors: powers of independent probes are random combinations
  of the leading eigenvectors of X.  Each column is then standardised to
  mean 0 and (population) standard deviation 1 over the vertices; a column
  whose standard deviation is at most 1e-6 times its root mean square is
  constant up to rounding and is set to 0.  ``N_RAW`` of the ``FEAT`` columns
  are used (the rest are 0).
* network  F = relu(relu(phi W1 + b1) W2 + b2) W3 + b3   (n x k)
* loss     L(F) = ||(I - U U^T) F||_F^2 / ||F||_F^2
                  + mu * || (k / ||F||_F^2) F^T F - I ||_F^2
  where U (n x k, orthonormal columns) spans the reference eigenvectors.  The
  first term is the squared sine of the angles between span(F) and span(U)
  weighted by F; the second keeps F's columns well conditioned (a start block
  of rank < k would leave directions to the Gaussian columns only).  L is
  invariant to the scale of F; L = 0 exactly when the columns of F are an
  orthogonal basis of span(U) of equal norms.
* Adam (Kingma & Ba 2015) with bias correction.

Parity unpinned against the paper (it has no such component); pinned by
central finite differences of L and by closed forms.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

FEAT = 8  # padded feature width
N_RAW = 8  # features used: log-degree, X^3 G (4 columns), X^4 G (first 3 columns)
N_PROBE = 4  # Rademacher probe vectors
SPREAD_TOL = 1e-6  # a column with std <= SPREAD_TOL * rms is constant: set to 0


def features(rowptr, colidx, alpha: float, g) -> np.ndarray:
    """phi (n x FEAT), FP64: log-degree and random-walk probes of a block g of
    N_PROBE Rademacher vectors (n x N_PROBE): all columns of X^3 g and the
    first three of X^4 g, each column standardised."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    n = len(rowptr) - 1
    deg = np.diff(rowptr).astype(np.float64)
    A = sp.csr_matrix((np.ones(len(colidx)), colidx, rowptr), shape=(n, n))
    with np.errstate(divide="ignore"):
        dp = np.where(deg > 0, deg ** (-alpha), 0.0)
    X = sp.diags(dp) @ A @ sp.diags(dp)
    raw = np.zeros((n, N_RAW))
    raw[:, 0] = np.log(np.maximum(deg, 1.0))
    v = np.asarray(g, dtype=np.float64).reshape(n, N_PROBE)
    for t in range(1, 5):
        v = X @ v
        if t == 3:
            raw[:, 1:1 + N_PROBE] = v
        elif t == 4:
            raw[:, 1 + N_PROBE:N_RAW] = v[:, :N_RAW - 1 - N_PROBE]
    phi = np.zeros((n, FEAT))
    mean = raw.mean(axis=0)
    std = raw.std(axis=0)
    rms = np.sqrt((raw * raw).mean(axis=0))
    for j in range(N_RAW):
        if std[j] > SPREAD_TOL * rms[j]:
            phi[:, j] = (raw[:, j] - mean[j]) / std[j]
    return phi


def param_shapes(width: int, out: int):
    """Parameter blocks in storage order: W1, b1, W2, b2, W3, b3 (row-major)."""
    return [("W1", (FEAT, width)), ("b1", (width,)), ("W2", (width, width)), ("b2", (width,)),
            ("W3", (width, out)), ("b3", (out,))]


def unflatten(theta, width: int, out: int) -> dict:
    theta = np.asarray(theta, dtype=np.float64)
    p, off = {}, 0
    for name, shp in param_shapes(width, out):
        size = int(np.prod(shp))
        p[name] = theta[off:off + size].reshape(shp)
        off += size
    assert off == theta.size
    return p


def flatten(p: dict, width: int, out: int) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in param_shapes(width, out)])


def forward(p: dict, phi):
    """Returns (H1, H2, F)."""
    H1 = np.maximum(phi @ p["W1"] + p["b1"], 0.0)
    H2 = np.maximum(H1 @ p["W2"] + p["b2"], 0.0)
    F = H2 @ p["W3"] + p["b3"]
    return H1, H2, F


def forward_bf16(p: dict, phi):
    """The inference pass with BF16 hidden activations (the start block only
    seeds the power iteration): each hidden layer's output is rounded to the
    nearest bfloat16 before it enters the next product.  Returns F."""
    H1 = bf16_round(np.maximum(phi @ p["W1"] + p["b1"], 0.0))
    H2 = bf16_round(np.maximum(H1 @ p["W2"] + p["b2"], 0.0))
    return H2 @ p["W3"] + p["b3"]


def loss(F, U, mu: float) -> float:
    k = F.shape[1]
    s = float(np.sum(F * F))
    R = F - U @ (U.T @ F)
    M = (k / s) * (F.T @ F) - np.eye(k)
    return float(np.sum(R * R) / s + mu * np.sum(M * M))


def loss_grad(F, U, mu: float):
    """dL/dF (n x k), from the closed form of each term:
    d/dF [1 - ||U^T F||^2 / s] = -(2/s) U P + (2 ||P||^2 / s^2) F,     P = U^T F
    d/dF [mu ||M||^2]          = (4 mu k / s) F M - (4 mu k <M,G> / s^2) F,
    with s = ||F||^2, G = F^T F, M = (k/s) G - I (U orthonormal)."""
    k = F.shape[1]
    s = float(np.sum(F * F))
    P = U.T @ F
    G = F.T @ F
    M = (k / s) * G - np.eye(k)
    pp = float(np.sum(P * P))
    mg = float(np.sum(M * G))
    return (-(2.0 / s) * (U @ P) + (2.0 * pp / s ** 2) * F
            + (4.0 * mu * k / s) * (F @ M) - (4.0 * mu * k * mg / s ** 2) * F)


def backward(p: dict, phi, H1, H2, dF) -> dict:
    """Gradients of the parameters given dL/dF (chain rule through the layers)."""
    g = {}
    g["W3"] = H2.T @ dF
    g["b3"] = dF.sum(axis=0)
    dZ2 = (dF @ p["W3"].T) * (H2 > 0)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"].T) * (H1 > 0)
    g["W1"] = phi.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g


def grad(theta, phi, U, mu: float, width: int, out: int):
    """(L, dL/dtheta) for flat parameters theta."""
    p = unflatten(theta, width, out)
    H1, H2, F = forward(p, phi)
    return loss(F, U, mu), flatten(backward(p, phi, H1, H2, loss_grad(F, U, mu)), width, out)


def adam(theta, gvec, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * gvec
    v = beta2 * v + (1 - beta2) * gvec * gvec
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def bf16_round(x) -> np.ndarray:
    """Round (the FP32 value of) x to the nearest bfloat16, ties to even; returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
