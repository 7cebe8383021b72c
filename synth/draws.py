"""Seeded random realizations consumed by the method.

The method draws three kinds of random numbers: a Gaussian start block for the
randomized eigendecomposition, and two sparse-sign test matrices for the
single-pass sketch.  For parity between the CPU oracle and the GPU path the
realizations are drawn here once and handed to both sides as data.
"""
from __future__ import annotations

import numpy as np


def gaussian_block(n: int, cols: int, seed: int, dtype=np.float32) -> np.ndarray:
    """Standard normal n x cols block, drawn in float64 and rounded to ``dtype``."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, cols)).astype(dtype)


def rademacher(n: int, seed: int, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 2, size=n) * 2 - 1).astype(dtype)


def sparse_sign(n: int, cols: int, z: int, seed: int):
    """Coordinates and signs of an n x cols sparse-sign matrix.

    Column c has ``z`` distinct row coordinates drawn uniformly from [0, n)
    (rows may repeat across columns) and ``z`` independent fair signs.
    Returns ``rows`` int32 (cols, z) and ``signs`` int8 (cols, z) with
    values in {-1, +1}.  The numeric value of an entry is signs/sqrt(z).
    """
    if not (1 <= z <= n):
        raise ValueError("need 1 <= z <= n")
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, n, size=(cols, z), dtype=np.int64)
    for _ in range(1000):
        s = np.sort(rows, axis=1)
        dup_cols = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0] if z > 1 else []
        if len(dup_cols) == 0:
            break
        for c in dup_cols:
            # redraw a whole column as z distinct rows (randperm(n, z))
            if n <= 4 * z:
                rows[c] = rng.permutation(n)[:z]
            else:
                r = np.unique(rng.integers(0, n, size=2 * z))
                while len(r) < z:
                    r = np.unique(np.concatenate([r, rng.integers(0, n, size=z)]))
                rows[c] = rng.permutation(r)[:z]
    signs = (rng.integers(0, 2, size=(cols, z)) * 2 - 1).astype(np.int8)
    return rows.astype(np.int32), signs


def sparse_sign_rows(n: int, cols: int, z: int, seed: int):
    """Coordinates and signs of an n x cols sparse-sign matrix with z nonzeros
    per ROW (one per vertex): row i has ``z`` distinct column coordinates in
    [0, cols), in random order, and ``z`` fair signs.  Returns ``cols_idx``
    int32 (n, z) and ``signs`` int8 (n, z); the numeric value of an entry is
    signs/sqrt(z)."""
    if not (1 <= z <= cols):
        raise ValueError("need 1 <= z <= cols")
    rng = np.random.default_rng(seed)
    idx = np.empty((n, z), dtype=np.int32)
    for r0 in range(0, n, 16384):
        r1 = min(n, r0 + 16384)
        # the z smallest of cols uniform keys: a uniformly random z-subset,
        # in the random order of their keys
        keys = rng.random((r1 - r0, cols))
        part = np.argpartition(keys, z - 1, axis=1)[:, :z] if z < cols else np.tile(np.arange(cols), (r1 - r0, 1))
        order = np.argsort(np.take_along_axis(keys, part, axis=1), axis=1)
        idx[r0:r1] = np.take_along_axis(part, order, axis=1)
    signs = (rng.integers(0, 2, size=(n, z)) * 2 - 1).astype(np.int8)
    return idx, signs
