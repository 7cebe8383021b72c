"""GPU parity of the general single pass, Eqs. (5)-(10), through the C ABI:
the three sketches K, Y, Z of a non-symmetric f(LR) against the oracle's
column-sampled sketches (same factors and test matrices), the reduction to
the embedding on sketches of an exactly low-rank non-symmetric matrix, the
whole general path against the oracle, and the symmetric special case
(C = S, H = O) against the path of Alg. 4."""
import numpy as np
import pytest

import synth
from oracle import sketch as sk, netmf, freigs as fr, metrics
from tests.util import say, c1_graph

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _factors(n, k, seed):
    # entries of LR spread around the trunc_log kink at 1 (about half below)
    rng = np.random.default_rng(seed)
    L = (rng.random((n, k)) * 1.2).astype(np.float32)
    R = (rng.standard_normal((k, n)) * 0.45 + 0.12).astype(np.float32)
    return L, R


def _tests(n, h, l, z, seed):
    return [synth.sparse_sign(n, c, z, seed + i) for i, c in enumerate((h, h, l, l))]


@pytest.mark.parametrize("n,k,h,l,z,prec,split,tol", [
    (5003, 32, 24, 80, 8, 0, 0, 1e-4),
    (5003, 20, 18, 61, 3, 0, 0, 1e-4),     # k, h, l off the tile sizes; z < 8
    (5003, 32, 24, 80, 8, 1, 16, 1e-2),
    (4096, 64, 40, 100, 8, 1, 0, 1e-2),
])
def test_sketch_general_parity(lib, n, k, h, l, z, prec, split, tol):
    from paper_2110_12782_amd.binding import SketchParams
    say(f"sketch_general n={n} k={k} h={h} l={l} z={z} prec={prec} split={split}")
    L, R = _factors(n, k, 7)
    rs = _tests(n, h, l, z, 100)
    p = SketchParams(k=k, s_eig=0, d=min(8, h), h=h, l=l, z=z, precision=prec, split_r=split)
    Kt, Yt, Z = lib.sketch_general(dev(L), dev(R.T), p, *[(dev(r), dev(s)) for r, s in rs])
    assert lib.sync() == 0
    Ko, Yo, Zo = sk.sketch_general_sampled(L.astype(np.float64), R.astype(np.float64), *rs)
    ek = metrics.rel_fro(Kt.cpu().numpy().T, Ko)
    ey = metrics.rel_fro(Yt.cpu().numpy().T, Yo)
    ez = metrics.rel_fro(Z.cpu().numpy(), Zo)
    say(f"  K {ek:.3e}  Y {ey:.3e}  Z {ez:.3e}")
    assert ek <= tol and ey <= tol and ez <= tol


def test_embed_general_exact_low_rank(lib):
    # sketches of X = A B of exact rank r <= h, not symmetric: Q W P^T = X, so
    # sigma are its singular values and E Ed^T = U_d Sigma_d V_d^T exactly
    from paper_2110_12782_amd.binding import SketchParams
    say("embed_general exact low rank n=3000 r=10 h=24 l=80 d=6")
    rng = np.random.default_rng(8)
    n, r, h, l, z, d = 3000, 10, 24, 80, 8, 6
    X = rng.standard_normal((n, r)) @ rng.standard_normal((r, n))
    rs = _tests(n, h, l, z, 200)
    Cd, Sd, Hd, Od = [sk.sparse_sign_dense(n, *x) for x in rs]
    K, Y, Z = X.T @ Cd, X @ Sd, Hd.T @ X @ Od
    p = SketchParams(k=8, s_eig=0, d=d, h=h, l=l, z=z)
    E, Ed, sig = lib.embed_general(n, p, dev(K.T.astype(np.float32)), dev(Y.T.astype(np.float32)),
                                   dev(Z.astype(np.float32)), (dev(rs[2][0]), dev(rs[2][1])),
                                   (dev(rs[3][0]), dev(rs[3][1])))
    assert lib.sync() & ~1 == 0  # K, Y of rank r < h: the documented Cholesky shift (bit 0) only
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    sig = sig.cpu().numpy()
    E, Ed = E.cpu().numpy().astype(np.float64), Ed.cpu().numpy().astype(np.float64)
    say(f"  sigma rel err {np.abs(sig - s[:d]).max() / s[0]:.3e}")
    assert np.allclose(sig, s[:d], rtol=2e-5)
    ref = (U[:, :d] * s[:d]) @ Vt[:d]
    assert metrics.rel_fro(E @ Ed.T, ref) < 1e-4


def test_general_pipeline_vs_oracle(lib):
    from paper_2110_12782_amd.binding import SketchParams
    say("general pipeline n=5003 k=32 h=24 l=80 d=8 (FP32) vs oracle")
    n, k, h, l, z, d = 5003, 32, 24, 80, 8, 8
    L, R = _factors(n, k, 9)
    rs = _tests(n, h, l, z, 300)
    p = SketchParams(k=k, s_eig=0, d=d, h=h, l=l, z=z)
    Kt, Yt, Z = lib.sketch_general(dev(L), dev(R.T), p, *[(dev(r), dev(s)) for r, s in rs])
    E, Ed, sig = lib.embed_general(n, p, Kt, Yt, Z, (dev(rs[2][0]), dev(rs[2][1])), (dev(rs[3][0]), dev(rs[3][1])))
    assert lib.sync() == 0
    Ko, Yo, Zo = sk.sketch_general_sampled(L.astype(np.float64), R.astype(np.float64), *rs)
    H = sk.sparse_sign_matrix(n, *rs[2])
    O = sk.sparse_sign_matrix(n, *rs[3])
    Uo, so, Vo, _ = sk.single_pass_svd_general(Ko, Yo, Zo, H, O, d)
    sig = sig.cpu().numpy()
    E, Ed = E.cpu().numpy().astype(np.float64), Ed.cpu().numpy().astype(np.float64)
    es = np.abs(sig - so).max() / so.max()
    ee = metrics.rel_fro(E @ Ed.T, (Uo * so) @ Vo.T)
    et = metrics.sin_theta_fro(E, Uo * np.sqrt(so))
    say(f"  sigma {es:.3e}  E Ed^T {ee:.3e}  sin theta(E) {et:.3e}")
    assert es <= 1e-4 and ee <= 1e-3 and et <= 1e-3


def test_general_symmetric_case_matches_alg4(lib):
    # the NetMF target of an SBM graph with C = S and H = O: the general
    # sketches equal those of Alg. 4 (sketchne_sketch) on the same U, lambda
    from paper_2110_12782_amd.binding import DeviceGraph, SketchParams
    say("general vs Alg. 4 on C1 SBM factors, C = S, H = O")
    rowptr, colidx = c1_graph()
    A = netmf.adjacency(rowptr, colidx)
    n = A.shape[0]
    X = netmf.modified_laplacian(A, 0.5)
    U, lam = fr.freigs(X, synth.gaussian_block(n, 160, 2001).astype(np.float64), 128, 2)
    U32 = U.astype(np.float32)
    Lp, Rp, _ = netmf.eq11_factors(U32.astype(np.float64), lam, netmf.degrees(A), netmf.volume(A), 0.5, 10, 1.0)
    rS, sS = synth.sparse_sign(n, 80, 8, 3001)
    rO, sO = synth.sparse_sign(n, 1032, 8, 4001)
    p = SketchParams(k=128, s_eig=32, d=32, h=80, l=1032, z=8)
    S, O = (dev(rS), dev(sS)), (dev(rO), dev(sO))
    Kt, Yt, Z = lib.sketch_general(dev(Lp.astype(np.float32)), dev(Rp.T.astype(np.float32)), p, S, S, O, O)
    Ys, Zs, _, _ = lib.sketch(DeviceGraph(rowptr, colidx), p, dev(U32), dev(lam), S=S, O=O)
    assert lib.sync() == 0
    ey = metrics.rel_fro(Yt.cpu().numpy(), Ys.cpu().numpy())
    ek = metrics.rel_fro(Kt.cpu().numpy(), Ys.cpu().numpy())  # f(L'R') is symmetric: K = Y when C = S
    ez = metrics.rel_fro(Z.cpu().numpy(), Zs.cpu().numpy())
    say(f"  Y {ey:.3e}  K vs Y {ek:.3e}  Z {ez:.3e}")
    assert ey <= 1e-4 and ek <= 1e-4 and ez <= 1e-4


def test_general_args(lib):
    from paper_2110_12782_amd.binding import SketchParams, SketchneError
    n, k = 300, 8
    L, R = _factors(n, k, 1)
    rs = _tests(n, 16, 40, 4, 1)
    T = [(dev(r), dev(s)) for r, s in rs]
    with pytest.raises(SketchneError):  # FP16 has no range bound for arbitrary factors
        lib.sketch_general(dev(L), dev(R.T), SketchParams(k=k, s_eig=0, d=4, h=16, l=40, z=4, precision=2), *T)
    with pytest.raises(SketchneError):  # h < d
        lib.sketch_general(dev(L), dev(R.T), SketchParams(k=k, s_eig=0, d=20, h=16, l=40, z=4), *T)
