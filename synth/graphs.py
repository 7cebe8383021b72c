"""Seeded synthetic graph generators producing undirected, unweighted CSR.

Every generator returns ``(rowptr, colidx)`` with ``rowptr`` int64 of length
n+1 and ``colidx`` int32: the pattern is symmetric, each row is sorted
ascending, there are no self loops and no duplicate edges (the adjacency is
0/1).  These stand in for the paper's real social and web graphs, which are
not available; the shapes (size, mean degree, degree skew) follow the
workloads the method is evaluated on.
"""
from __future__ import annotations

import numpy as np


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray):
    """Symmetrize, drop self loops, deduplicate and sort an edge list into CSR."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    keys = np.concatenate([u * n + v, v * n + u])
    keys = np.unique(keys)
    rows = keys // n
    cols = (keys - rows * n).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr, cols


def degree_exponent_mle(deg: np.ndarray, d_min: int = 10) -> float:
    """Discrete power-law exponent of the degree tail d >= d_min by the
    standard continuous approximation of the maximum-likelihood estimate
    (Clauset, Shalizi and Newman 2009): 1 + N / sum ln(d / (d_min - 1/2))."""
    tail = deg[deg >= d_min].astype(np.float64)
    if len(tail) == 0:
        return float("nan")
    return float(1.0 + len(tail) / np.sum(np.log(tail / (d_min - 0.5))))


def graph_stats(rowptr: np.ndarray, colidx: np.ndarray) -> dict:
    deg = np.diff(rowptr)
    n = len(deg)
    return {
        "n": int(n),
        "nnz": int(rowptr[-1]),
        "m": int(rowptr[-1] // 2),
        "mean_degree": float(deg.mean()) if n else 0.0,
        "max_degree": int(deg.max()) if n else 0,
        "min_degree": int(deg.min()) if n else 0,
        "isolated": int((deg == 0).sum()),
        "gamma_hat_d10": degree_exponent_mle(deg, 10) if n else float("nan"),
    }


def _sample_pairs_between(rng, lo_a, size_a, lo_b, size_b, same, p):
    """Bernoulli(p) edges between two vertex blocks (or inside one block)."""
    if same:
        npairs = size_a * (size_a - 1) // 2
    else:
        npairs = size_a * size_b
    if npairs == 0 or p <= 0:
        return np.empty(0, np.int64), np.empty(0, np.int64)
    cnt = rng.binomial(npairs, p)
    if cnt == 0:
        return np.empty(0, np.int64), np.empty(0, np.int64)
    # Draw distinct pair indices uniformly (exact Bernoulli-graph law).
    if cnt > npairs // 2:
        idx = rng.permutation(npairs)[:cnt]
    else:
        idx = np.unique(rng.integers(0, npairs, size=int(cnt * 1.2) + 16))
        while len(idx) < cnt:
            extra = rng.integers(0, npairs, size=cnt)
            idx = np.unique(np.concatenate([idx, extra]))
        idx = rng.permutation(idx)[:cnt]
    if same:
        # unrank index -> (i, j), i > j, inside a triangle of size_a
        i = np.floor((1.0 + np.sqrt(1.0 + 8.0 * idx.astype(np.float64))) / 2.0).astype(np.int64)
        i = np.where(i * (i - 1) // 2 > idx, i - 1, i)
        i = np.where((i + 1) * i // 2 <= idx, i + 1, i)
        j = idx - i * (i - 1) // 2
        return lo_a + i, lo_a + j
    return lo_a + idx // size_b, lo_b + idx % size_b


def sbm(block_sizes, p_in: float, p_out: float, seed: int):
    """Stochastic block model: edge (i,j) present with p_in inside a block, p_out across."""
    rng = np.random.default_rng(seed)
    block_sizes = [int(s) for s in block_sizes]
    starts = np.concatenate([[0], np.cumsum(block_sizes)])
    n = int(starts[-1])
    us, vs = [], []
    for a in range(len(block_sizes)):
        for b in range(a, len(block_sizes)):
            p = p_in if a == b else p_out
            u, v = _sample_pairs_between(rng, starts[a], block_sizes[a], starts[b],
                                         block_sizes[b], a == b, p)
            us.append(u)
            vs.append(v)
    u = np.concatenate(us) if us else np.empty(0, np.int64)
    v = np.concatenate(vs) if vs else np.empty(0, np.int64)
    return csr_from_edges(n, u, v)


def _chung_lu_weights(n: int, gamma: float, mean_deg: float, min_w: float):
    """Power-law expected degrees w_i = c (i + i0)^(-1/(gamma-1)) with min w =
    min_w, solved for the mean.  Each of eight refinement passes clips the
    weights at the square root of that pass's unclipped sum and rescales the
    target mean; the clip is therefore loose (on the n = 2^20, mean 20 graph
    the largest returned weight is about 19,000 and the mean about 14), and no
    bound w_i w_j / sum(w) <= 1 is claimed: the generator draws edge endpoints
    independently in proportion to w (Norros-Reittu form), which needs no
    such bound, and tops the edge count up to the target mean degree."""
    beta = 1.0 / (gamma - 1.0)
    i = np.arange(n, dtype=np.float64)
    target = mean_deg
    w = None
    for _ in range(8):
        lo, hi = 1e-9, 1e12
        for _ in range(200):
            i0 = np.sqrt(lo * hi)
            c = min_w * (n - 1 + i0) ** beta
            mean = c * np.mean((i + i0) ** (-beta))
            if mean > target:
                lo = i0
            else:
                hi = i0
        w = c * (i + i0) ** (-beta)
        cap = np.sqrt(w.sum())
        w = np.minimum(w, cap)
        target *= mean_deg / w.mean()
    return w


def chung_lu(n: int, gamma: float, mean_deg: float, min_deg: int, seed: int, permute: bool = True):
    """Chung-Lu power-law graph.

    Edge endpoints are drawn independently with probability proportional to
    the expected-degree weights (Norros-Reittu form of the Chung-Lu model),
    then symmetrized and deduplicated.  Vertices left below ``min_deg`` get
    extra edges to weight-proportional partners.  Labels are then permuted
    with a seeded random permutation, so that vertex index carries no degree
    information.
    """
    rng = np.random.default_rng(seed)
    w = _chung_lu_weights(n, gamma, mean_deg, float(min_deg))
    W = w.sum()
    cdf = np.cumsum(w) / W
    m = int(round(W / 2.0))
    u = np.searchsorted(cdf, rng.random(m), side="right").clip(0, n - 1)
    v = np.searchsorted(cdf, rng.random(m), side="right").clip(0, n - 1)
    rowptr, colidx = csr_from_edges(n, u, v)
    # Deduplication removes repeated hub pairs; top the edge count up until
    # the realized mean degree reaches the target.
    for _ in range(12):
        mean = rowptr[-1] / n
        if mean >= 0.995 * mean_deg:
            break
        extra = int((mean_deg - mean) * n / 2 * 1.15) + 1
        u = np.concatenate([u, np.searchsorted(cdf, rng.random(extra), side="right").clip(0, n - 1)])
        v = np.concatenate([v, np.searchsorted(cdf, rng.random(extra), side="right").clip(0, n - 1)])
        rowptr, colidx = csr_from_edges(n, u, v)
    for _ in range(4):
        deg = np.diff(rowptr)
        low = np.nonzero(deg < min_deg)[0]
        if len(low) == 0:
            break
        need = (min_deg - deg[low]).astype(np.int64)
        a = np.repeat(low, need)
        b = np.searchsorted(cdf, rng.random(len(a)), side="right").clip(0, n - 1)
        rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
        u = np.concatenate([rows, a])
        v = np.concatenate([colidx.astype(np.int64), b])
        rowptr, colidx = csr_from_edges(n, u, v)
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
        rowptr, colidx = csr_from_edges(n, perm[rows], perm[colidx.astype(np.int64)])
    return rowptr, colidx


def rmat(scale: int, n_edges: int, a: float, b: float, c: float, d: float, seed: int,
         permute: bool = True, chunk: int = 1 << 22):
    """R-MAT: each edge descends ``scale`` levels of the adjacency quadrants with
    probabilities (a, b, c, d); then seeded label permutation, symmetrize, dedup."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    us, vs = [], []
    ab = a + b
    c_norm = c / (c + d)
    a_norm = a / (a + b)
    left = n_edges
    while left > 0:
        cnt = min(chunk, left)
        left -= cnt
        u = np.zeros(cnt, np.int64)
        v = np.zeros(cnt, np.int64)
        for lvl in range(scale):
            bit = np.int64(1) << np.int64(scale - 1 - lvl)
            r1 = rng.random(cnt)
            r2 = rng.random(cnt)
            down = r1 > ab
            right = np.where(down, r2 > c_norm, r2 > a_norm)
            u += np.where(down, bit, 0)
            v += np.where(right, bit, 0)
        us.append(u)
        vs.append(v)
    u = np.concatenate(us)
    v = np.concatenate(vs)
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        u, v = perm[u], perm[v]
    return csr_from_edges(n, u, v)


def cycle(n: int):
    i = np.arange(n, dtype=np.int64)
    return csr_from_edges(n, i, (i + 1) % n)


def complete(n: int):
    iu, ju = np.triu_indices(n, 1)
    return csr_from_edges(n, iu, ju)


def disjoint_union(g1, g2):
    r1, c1 = g1
    r2, c2 = g2
    n1 = len(r1) - 1
    rowptr = np.concatenate([r1, r2[1:] + r1[-1]]).astype(np.int64)
    colidx = np.concatenate([c1, c2 + n1]).astype(np.int32)
    return rowptr, colidx
