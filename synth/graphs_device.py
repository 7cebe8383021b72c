"""Seeded graph generators that run on the GPU with torch (for sizes where the
NumPy generators are too slow).  They produce the same kind of graph as
``synth.graphs``: undirected, unweighted, no self loops, no duplicates, CSR
with sorted rows, returned as device tensors (rowptr int64, colidx int32).
The draws use torch's seeded device generator, so a graph is reproducible on
the same device type (not bit-identical to the NumPy generators)."""
from __future__ import annotations


def rmat_device(scale: int, n_edges: int, a: float, b: float, c: float, d: float, seed: int,
                device: str = "cuda", permute: bool = True):
    """R-MAT: each edge descends ``scale`` levels of the adjacency quadrants,
    going down with probability c + d and then right with probability
    b / (a + b) (top half) or d / (c + d) (bottom half); then a seeded label
    permutation, symmetrization, removal of self loops and duplicates."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    n = 1 << scale
    ab = a + b
    a_norm = a / (a + b)
    c_norm = c / (c + d)
    u = torch.zeros(n_edges, dtype=torch.int64, device=device)
    v = torch.zeros(n_edges, dtype=torch.int64, device=device)
    for _ in range(scale):
        r1 = torch.rand(n_edges, generator=gen, device=device, dtype=torch.float64)
        r2 = torch.rand(n_edges, generator=gen, device=device, dtype=torch.float64)
        down = r1 > ab
        right = torch.where(down, r2 > c_norm, r2 > a_norm)
        u = (u << 1) | down.to(torch.int64)
        v = (v << 1) | right.to(torch.int64)
        del r1, r2, down, right
    if permute:
        perm = torch.randperm(n, generator=gen, device=device)
        u = perm[u]
        v = perm[v]
        del perm
    keep = u != v
    u = u[keep]
    v = v[keep]
    keys = torch.cat([u * n + v, v * n + u])
    del u, v, keep
    keys = torch.unique(keys, sorted=True)
    rows = torch.div(keys, n, rounding_mode="floor")
    colidx = (keys - rows * n).to(torch.int32)
    del keys
    counts = torch.bincount(rows, minlength=n)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(counts, 0)
    return rowptr, colidx
