"""The seeded generators produce valid undirected CSR graphs with the stated shapes."""
import numpy as np
import pytest

import synth


def check_csr(rowptr, colidx):
    n = len(rowptr) - 1
    assert rowptr[0] == 0 and np.all(np.diff(rowptr) >= 0)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    assert np.all(rows != colidx)                       # no self loops
    for i in range(0, n, max(1, n // 50)):
        seg = colidx[rowptr[i]:rowptr[i + 1]]
        assert np.all(np.diff(seg) > 0)                # sorted, no duplicates
    key = rows.astype(np.int64) * n + colidx
    rkey = colidx.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(key), np.sort(rkey))  # symmetric


def test_sbm_shape():
    rowptr, colidx = synth.sbm([512] * 8, 0.02, 0.001, 1000)
    check_csr(rowptr, colidx)
    st = synth.graph_stats(rowptr, colidx)
    # E[deg] = 511*0.02 + 3584*0.001 = 13.8
    assert 12.5 < st["mean_degree"] < 15.0


def test_chung_lu_shape():
    rowptr, colidx = synth.chung_lu(65536, 2.1, 16, 2, 1001)
    check_csr(rowptr, colidx)
    st = synth.graph_stats(rowptr, colidx)
    assert st["min_degree"] >= 2
    assert 13.5 < st["mean_degree"] < 17.5
    assert st["max_degree"] > 200                       # heavy tail


def test_rmat_small():
    rowptr, colidx = synth.rmat(10, 8192, 0.57, 0.19, 0.19, 0.05, 3)
    check_csr(rowptr, colidx)


def test_sparse_sign_draw():
    rows, signs = synth.sparse_sign(1000, 300, 8, 5)
    assert rows.shape == (300, 8) and signs.shape == (300, 8)
    for c in range(300):
        assert len(np.unique(rows[c])) == 8
    assert set(np.unique(signs)) == {-1, 1}
    r2, s2 = synth.sparse_sign(1000, 300, 8, 5)
    assert np.array_equal(rows, r2) and np.array_equal(signs, s2)
    # n == z: every column is a permutation of all rows
    r3, _ = synth.sparse_sign(8, 20, 8, 6)
    assert all(sorted(r) == list(range(8)) for r in r3)


def test_degree_exponent_mle():
    # integer samples of a power law with exponent 2.4 above d_min = 10 (a
    # Pareto draw rounded to the nearest integer): the estimate recovers it
    rng = np.random.default_rng(3)
    d = np.rint(9.5 * rng.random(200000) ** (-1.0 / 1.4)).astype(np.int64)
    assert abs(synth.graphs.degree_exponent_mle(d, 10) - 2.4) < 0.05
    # the bench-shaped Chung-Lu graph has the exponent it was built for
    rowptr, colidx = synth.chung_lu(1 << 15, 2.1, 16, 2, 9)
    assert abs(synth.graph_stats(rowptr, colidx)["gamma_hat_d10"] - 2.1) < 0.2
