"""Error measures: relative Frobenius error and principal angles between spans."""
from __future__ import annotations

import numpy as np


def rel_fro(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (den if den > 0 else 1.0))


def sin_principal_angles(A, B) -> np.ndarray:
    """Sines of the principal angles between span(A) and span(B), descending."""
    Qa, _ = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="reduced")
    Qb, _ = np.linalg.qr(np.asarray(B, dtype=np.float64), mode="reduced")
    if Qa.shape[1] > Qb.shape[1]:
        Qa, Qb = Qb, Qa
    R = Qa - Qb @ (Qb.T @ Qa)          # residual of projecting span(A) onto span(B)
    s = np.linalg.svd(R, compute_uv=False)
    return np.clip(s, 0.0, 1.0)


def sin_theta_fro(A, B) -> float:
    """||sin Theta||_F / sqrt(p), p = the smaller of the two dimensions."""
    s = sin_principal_angles(A, B)
    return float(np.sqrt(np.sum(s ** 2) / len(s)))
