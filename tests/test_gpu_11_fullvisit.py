"""GPU parity of the full-visit variant (z nonzeros per row of S and O, every
entry of f(L'R') formed) through the C ABI, against the oracle's row-blocked
definition on the same U, lambda, S and O: FP32 to 1e-4 and BF16 to 1e-2
(relative Frobenius on Y and Z, per column of Y), on an SBM with ragged n and
the C1 shape, plus the embedding against the oracle's single pass."""
import numpy as np
import pytest

import synth
from oracle import netmf, freigs as fr, sketch as sk, metrics
from tests.util import say, c1_graph

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _case(lib, rowptr, colidx, k, K, h, l, z, prec, seed):
    from paper_2110_12782_amd.binding import DeviceGraph, SketchParams
    A = netmf.adjacency(rowptr, colidx)
    n = A.shape[0]
    X = netmf.modified_laplacian(A, 0.5)
    U, lam = fr.freigs(X, synth.gaussian_block(n, K, seed).astype(np.float64), k, 2)
    U32 = U.astype(np.float32)
    Lp, Rp, _ = netmf.eq11_factors(U32.astype(np.float64), lam, netmf.degrees(A), netmf.volume(A), 0.5, 10, 1.0)
    sc, ss = synth.sparse_sign_rows(n, h, z, seed + 1)
    oc, os_ = synth.sparse_sign_rows(n, l, z, seed + 2)
    p = SketchParams(alpha=0.5, T=10, b=1.0, k=k, s_eig=K - k, q=2, d=min(16, h), h=h, l=l, z=z, precision=prec)
    g = DeviceGraph(rowptr, colidx)
    Yt, Z, S, O = lib.sketch_fullvisit(g, p, dev(U32), dev(lam), S=(dev(sc), dev(ss)), O=(dev(oc), dev(os_)))
    E, sig = lib.embed_fullvisit(n, p, Yt, Z, O)
    assert lib.sync() & ~1 == 0
    Yo, Zo = sk.sketch_fullvisit(Lp, Rp, sc, ss, oc, os_, h, l)
    Y = Yt.cpu().numpy().T.astype(np.float64)
    col = np.linalg.norm(Y - Yo, axis=0) / np.linalg.norm(Yo, axis=0)
    ey, ez = metrics.rel_fro(Y, Yo), metrics.rel_fro(Z.cpu().numpy(), Zo)
    O_sp = sk.sparse_sign_rows_matrix(n, l, oc, os_)
    Ud, so, _, _, _ = sk.single_pass_svd(Yo, Zo, O_sp, p.d)
    E = E.cpu().numpy().astype(np.float64)
    es = np.abs(sig.cpu().numpy() - so).max() / so.max()
    ee = metrics.rel_fro(E @ E.T, (Ud * so) @ Ud.T)
    say(f"  Y {ey:.3e} (worst column {col.max():.3e})  Z {ez:.3e}  sigma {es:.3e}  EE^T {ee:.3e}")
    return ey, col.max(), ez, es, ee


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 1e-2)])
def test_fullvisit_sbm_ragged(lib, prec, tol):
    say(f"full visit SBM n=1000 (ragged) k=32 h=40 l=70 z=4 prec={prec}")
    rowptr, colidx = synth.sbm([250] * 4, 0.05, 0.005, 31)
    ey, cmax, ez, es, ee = _case(lib, rowptr, colidx, 32, 48, 40, 70, 4, prec, 900)
    assert ey <= tol and ez <= tol and cmax <= 3 * tol
    assert es <= 10 * tol and ee <= 10 * tol


@pytest.mark.parametrize("prec,tol", [(0, 1e-4), (1, 1e-2)])
def test_fullvisit_c1(lib, prec, tol):
    say(f"full visit C1 SBM n=4096 k=128 h=80 l=1032 z=8 prec={prec}")
    rowptr, colidx = c1_graph()
    ey, cmax, ez, es, ee = _case(lib, rowptr, colidx, 128, 160, 80, 1032, 8, prec, 2001)
    assert ey <= tol and ez <= tol and cmax <= 3 * tol
    assert es <= 10 * tol and ee <= 10 * tol
