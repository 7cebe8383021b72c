"""GPU parity of spectral propagation (Alg. 6 line 6) through the C ABI:
the fused Chebyshev-recurrence SpMM against the FP64 oracle's three-term
recurrence, the library's coefficients against the oracle's, and at the
benchmark size (n = 2^20, d = 128, p = 10) sampled columns (columns of E
propagate independently) plus the constant-vector invariant."""
import numpy as np
import pytest

import synth
from oracle import netmf, propagation as pg, metrics
from tests.util import say, c1_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def _oracle(rowptr, colidx, E, c):
    A = netmf.adjacency(rowptr, colidx)
    return pg.propagate(A, E.astype(np.float64), c)


def _gpu(lib, torch, rowptr, colidx, E, c):
    from paper_2110_12782_amd.binding import DeviceGraph
    g = DeviceGraph(rowptr, colidx)
    out = lib.propagate(g, torch.from_numpy(np.ascontiguousarray(E)).cuda(), c)
    assert lib.sync() == 0
    return out.cpu().numpy().astype(np.float64)


def _with_isolated(rowptr, colidx, at, count, tail):
    # `count` isolated vertices inserted before vertex `at`, `tail` appended
    rp = np.concatenate([rowptr[:at + 1], np.full(count, rowptr[at]), rowptr[at + 1:], np.full(tail, rowptr[-1])])
    ci = np.where(colidx >= at, colidx + count, colidx).astype(np.int32)
    return rp, ci


@pytest.mark.parametrize("p", [0, 1, 2, 10])
def test_coeffs_match_oracle(lib, torch, p):
    say(f"propagate_coeffs p={p}")
    c = lib.propagate_coeffs(p, 0.5, 0.2)
    ref = pg.chebyshev_coeffs(pg.band_pass(0.5, 0.2), p)
    # each c_r is a sum of p + 1 terms of size up to max g (about 1.3): the two
    # FP64 summations agree to a few units of 1e-16 in absolute terms
    assert np.abs(c - ref).max() <= 1e-14


# d = 4, 12, 32, 64, 128, 256 take 8, 16, 32 and 64 lanes per slot (12: a
# masked quad in each slot)
@pytest.mark.parametrize("d", [4, 12, 32, 64, 128, 256])
def test_propagate_sbm(lib, torch, d):
    say(f"propagate SBM n=4096 d={d} p=10")
    rowptr, colidx = c1_graph()
    E = synth.gaussian_block(len(rowptr) - 1, d, 71)
    c = pg.chebyshev_coeffs(pg.band_pass(0.5, 0.2), 10)
    out = _gpu(lib, torch, rowptr, colidx, E, c)
    ref = _oracle(rowptr, colidx, E, c)
    assert metrics.rel_fro(out, ref) < 1e-5
    rowerr = np.linalg.norm(out - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-30)
    assert rowerr.max() < 1e-4


@pytest.mark.parametrize("p", [0, 1, 2, 3])
@pytest.mark.parametrize("d", [128, 8])
def test_propagate_hubs_isolated_low_degree(lib, torch, p, d):
    # hubs far longer than one slice (split rows through the fixup), isolated
    # vertices in the middle and at the end, and the degree-0..3 recurrences
    say(f"propagate Chung-Lu n=20005 + isolated, d={d}, p={p}")
    rowptr, colidx = synth.chung_lu(20000, 2.1, 16, 2, 5)
    rowptr, colidx = _with_isolated(rowptr, colidx, 5000, 3, 2)
    n = len(rowptr) - 1
    E = synth.gaussian_block(n, d, 72)
    c = pg.chebyshev_coeffs(pg.band_pass(0.5, 0.2), p)
    out = _gpu(lib, torch, rowptr, colidx, E, c)
    ref = _oracle(rowptr, colidx, E, c)
    assert metrics.rel_fro(out, ref) < 1e-5
    iso = np.diff(rowptr) == 0
    # an isolated vertex keeps p(1) E_i (M has a zero row there)
    assert np.allclose(out[iso], ref[iso], rtol=1e-6, atol=1e-6)


def test_propagate_ragged_tiny(lib, torch):
    say("propagate tiny graphs: n=1 isolated, path of 3, ragged 7")
    c = pg.chebyshev_coeffs(pg.band_pass(0.5, 0.2), 10)
    for rowptr, colidx in [(np.array([0, 0]), np.zeros(0, np.int32)),
                           (np.array([0, 1, 3, 4]), np.array([1, 0, 2, 1], np.int32)),
                           synth.cycle(7)]:
        n = len(rowptr) - 1
        E = synth.gaussian_block(n, 4, 73)
        out = _gpu(lib, torch, rowptr, colidx, E, c)
        ref = _oracle(rowptr, colidx, E, c)
        assert metrics.rel_fro(out, ref) < 1e-5


def test_propagate_args(lib, torch):
    from paper_2110_12782_amd.binding import DeviceGraph, SketchneError
    rowptr, colidx = synth.cycle(16)
    g = DeviceGraph(rowptr, colidx)
    E = torch.zeros((16, 6), dtype=torch.float32, device="cuda")  # d % 4 != 0
    with pytest.raises(SketchneError):
        lib.propagate(g, E, np.ones(3))
    E = torch.zeros((16, 260), dtype=torch.float32, device="cuda")  # d > 256
    with pytest.raises(SketchneError):
        lib.propagate(g, E, np.ones(3))
    with pytest.raises(SketchneError):
        lib.propagate_coeffs(65)


def test_propagate_fullsize_sampled_columns(lib, torch):
    # the benchmark configuration: Chung-Lu n = 2^20, mean degree 20, d = 128,
    # p = 10.  Columns propagate independently, so three columns of the GPU
    # result are compared with the oracle run on those columns alone; the
    # constant vector is an eigenvector of D^-1 A (eigenvalue 1, so of M with
    # -1) and must come out scaled by sum_r c_r T_r(-1) on a graph without
    # isolated vertices.
    from paper_2110_12782_amd.binding import DeviceGraph
    say("propagate Chung-Lu n=2^20 d=128 p=10, sampled columns")
    rowptr, colidx = synth.chung_lu(1 << 20, 2.1, 20, 2, 1003)
    n = len(rowptr) - 1
    assert (np.diff(rowptr) > 0).all()
    c = lib.propagate_coeffs(10, 0.5, 0.2)
    E = synth.gaussian_block(n, 128, 74)
    E[:, 5] = 1.0
    g = DeviceGraph(rowptr, colidx)
    out = lib.propagate(g, torch.from_numpy(E).cuda(), c)
    assert lib.sync() == 0
    out = out.cpu().numpy().astype(np.float64)
    cols = [0, 37, 127]
    ref = _oracle(rowptr, colidx, E[:, cols], pg.chebyshev_coeffs(pg.band_pass(0.5, 0.2), 10))
    assert metrics.rel_fro(out[:, cols], ref) < 1e-5
    const = sum(cr * (-1) ** r for r, cr in enumerate(c))
    assert np.abs(out[:, 5] - const).max() <= 1e-5 * abs(const)
