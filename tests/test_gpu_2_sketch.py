"""GPU parity of the fused sketch (Alg. 4 lines 4 and 7, Eq. 4) against the
FP64 oracle on identical inputs: the same U (rounded to FP32), lambda and the
same sparse-sign realizations S and O."""
import numpy as np
import pytest

from tests.util import say, c1_graph, c2_graph, oracle_factors, oracle_eig_inputs, rel, sk, netmf, synth

pytestmark = pytest.mark.gpu


def run_case(lib, rowptr, colidx, *, k, K, d, h, l, z, T=10, b=1.0, alpha=0.5, q=2, precision=0, split_r=0,
             seed=1, row_subset=None, U32=None, lam=None):
    import torch
    from paper_2110_12782_amd.binding import DeviceGraph, SketchParams
    A = netmf.adjacency(rowptr, colidx)
    n = A.shape[0]
    if U32 is None:
        U32, lam, _ = oracle_eig_inputs(A, k, K, q, alpha, 2000 + seed)
    rS, sS = synth.sparse_sign(n, h, z, 3000 + seed)
    rO, sO = synth.sparse_sign(n, l, z, 4000 + seed)
    p = SketchParams(alpha=alpha, T=T, b=b, k=k, s_eig=K - k, q=q, d=d, h=h, l=l, z=z, precision=precision,
                     split_r=split_r)
    g = DeviceGraph(rowptr, colidx)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Yt, Z, _, _ = lib.sketch(g, p, dev(U32), dev(np.asarray(lam, np.float64)), S=(dev(rS), dev(sS)),
                             O=(dev(rO), dev(sO)))
    assert lib.sync() == 0
    Y = Yt.cpu().numpy().T
    Zg = Z.cpu().numpy()
    Lp, Rp, _ = oracle_factors(A, U32, lam, alpha, T, b)
    Yo = sk.sketch_y_sampled(Lp, Rp, rS, sS, row_subset=row_subset)
    Zo = sk.sketch_z_sampled(Lp, Rp, rO, sO)
    Ycmp = Y if row_subset is None else Y[row_subset]
    return rel(Ycmp, Yo), rel(Zg, Zo), (Y, Zg, Yo, Zo)


def local_errors(Y, Yo, Zg, Zo):
    """Errors that one wrong tile or ragged tail cannot hide in an aggregate:
    the worst column of Y (one group of the test matrix, Eq. 4) relative to
    its own norm, the worst column of Z, and the largest entry error of Z
    relative to Z's largest entry.  (Single entries of Z are sums of z^2
    signed terms that may cancel, so they get no relative bound of their
    own.)"""
    Yo = np.asarray(Yo, np.float64)
    Y = np.asarray(Y, np.float64)
    norms = np.linalg.norm(Yo, axis=0)
    live = norms > 0
    col = np.linalg.norm(Y - Yo, axis=0)[live] / norms[live]
    # a column whose sampled entries all sit at or below the kink of
    # trunc_log is zero in FP64; rounding may lift an entry just above it
    assert np.abs(Y[:, ~live]).max(initial=0.0) <= 1e-3 * np.abs(Yo).max()
    zn = np.linalg.norm(Zo, axis=0)
    zlive = zn > 0
    zcol = np.linalg.norm(Zg - Zo, axis=0)[zlive] / zn[zlive]
    zent = np.abs(Zg - Zo).max() / np.abs(Zo).max()
    return float(col.max()), float(zcol.max()), float(zent)


def check_local(Y, Yo, Zg, Zo, tol):
    col, zcol, zent = local_errors(Y, Yo, Zg, Zo)
    say(f"  worst Y column {col:.2e}  worst Z column {zcol:.2e}  worst Z entry {zent:.2e} (of max |Z|)")
    assert col <= 2 * tol and zcol <= 5 * tol and zent <= tol


def test_sketch_fp32_c1(lib):
    say("sketch FP32 C1 SBM n=4096 k=128 h=80 l=1032")
    ey, ez, (Y, Zg, Yo, Zo) = run_case(lib, *c1_graph(), k=128, K=160, d=32, h=80, l=1032, z=8)
    say(f"  rel Y {ey:.3e}  rel Z {ez:.3e}")
    assert ey <= 1e-4 and ez <= 1e-4
    check_local(Y, Yo, Zg, Zo, 1e-4)
    assert np.abs(Zg - Zg.T).max() <= 1e-4 * np.abs(Zg).max()


# h = 2d + 16 (the widths used throughout) and the paper's h = d + 100
@pytest.mark.parametrize("h", [272, 228])
def test_sketch_fp32_c2(lib, h):
    say(f"sketch FP32 C2 Chung-Lu n=65536 k=256 h={h} l=1128")
    ey, ez, (Y, Zg, Yo, Zo) = run_case(lib, *c2_graph(), k=256, K=288, d=128, h=h, l=1128, z=8)
    say(f"  rel Y {ey:.3e}  rel Z {ez:.3e}")
    assert ey <= 1e-4 and ez <= 1e-4
    check_local(Y, Yo, Zg, Zo, 1e-4)


def test_sketch_edge_cases(lib):
    # ragged n, isolated vertices, z < 8, h and l not multiples of 4, small k,
    # T = 1, alpha < 1/2
    rowptr, colidx = synth.chung_lu(3001, 2.3, 10, 2, 9)
    rowptr = np.concatenate([rowptr, [rowptr[-1]] * 3])
    for kw in [dict(k=64, K=96, d=8, h=37, l=101, z=3, T=1, alpha=0.35),
               dict(k=40, K=64, d=16, h=21, l=50, z=8, T=5, alpha=0.5),
               dict(k=64, K=96, d=4, h=5, l=9, z=1, T=3, alpha=0.45)]:
        say(f"sketch FP32 edge n=3004 {kw}")
        ey, ez, (Y, Zg, Yo, Zo) = run_case(lib, rowptr, colidx, **kw)
        say(f"  rel Y {ey:.3e}  rel Z {ez:.3e}")
        assert ey <= 1e-4 and ez <= 1e-4
        check_local(Y, Yo, Zg, Zo, 1e-4)
        assert np.all(Y[-3:] == 0)  # isolated vertices: zero rows of Y


def test_sketch_lowp_edge_cases(lib):
    # k and r off the 16-wide sections (zero padding in every section), r = 0,
    # ragged n with isolated vertices, z < 8, h and l not multiples of 4
    rowptr, colidx = synth.chung_lu(3001, 2.3, 10, 2, 9)
    rowptr = np.concatenate([rowptr, [rowptr[-1]] * 3])
    for prec, kw in [(1, dict(k=40, K=64, d=16, h=21, l=50, z=8, T=5, split_r=10)),
                     (2, dict(k=100, K=128, d=8, h=37, l=101, z=3, T=1, alpha=0.35, split_r=20)),
                     (1, dict(k=64, K=96, d=4, h=5, l=9, z=1, T=3, alpha=0.45, split_r=0)),
                     (2, dict(k=256, K=288, d=16, h=33, l=70, z=5, split_r=32))]:
        say(f"sketch {'BF16' if prec == 1 else 'FP16'} edge n=3004 {kw}")
        ey, ez, (Y, Zg, Yo, Zo) = run_case(lib, rowptr, colidx, precision=prec, **kw)
        say(f"  rel Y {ey:.3e}  rel Z {ez:.3e}")
        assert ey <= 1e-2 and ez <= 1e-2
        check_local(Y, Yo, Zg, Zo, 1e-2)
        assert np.all(Y[-3:] == 0)  # isolated vertices: zero rows of Y


# (1, 16): the form bench.py times; h = 228 is the paper's h = d + 100
@pytest.mark.parametrize("precision,split_r,h,tol", [(1, 16, 272, 1e-2), (1, 32, 272, 1e-2), (1, 0, 272, 1e-2),
                                                     (2, 32, 272, 1e-2), (1, 16, 228, 1e-2)])
def test_sketch_lowp_c2(lib, precision, split_r, h, tol):
    name = {1: "BF16", 2: "FP16"}[precision]
    say(f"sketch {name} split_r={split_r} C2 h={h}")
    ey, ez, (Y, Zg, Yo, Zo) = run_case(lib, *c2_graph(), k=256, K=288, d=128, h=h, l=1128, z=8,
                                       precision=precision, split_r=split_r)
    say(f"  rel Y {ey:.3e}  rel Z {ez:.3e}")
    assert ey <= tol and ez <= tol
    check_local(Y, Yo, Zg, Zo, tol)
