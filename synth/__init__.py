"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds graph generators, the CSR builder and the random
realizations (Gaussian start blocks, sparse-sign test matrices) that the
method consumes.  It contains none of the method's arithmetic: no degree
normalisation, no NetMF matrix, no sketch, no eigensolver.  Both the CPU
oracle and the GPU path take their random draws from here as plain data, so
that the two can be compared on identical inputs.
"""
from .graphs import (  # noqa: F401
    csr_from_edges,
    sbm,
    chung_lu,
    rmat,
    cycle,
    complete,
    disjoint_union,
    graph_stats,
)
from .draws import gaussian_block, sparse_sign, sparse_sign_rows, rademacher  # noqa: F401
