"""Parity at the benchmark's full size (Chung-Lu, n = 2^20, exponent 2.1,
mean degree 20; k = 256, q = 2, d = 128, h = 272, l = 1128, z = 8; device
draws of Omega, S and O), in the launch configuration bench.py times.

Rows of Y are independent (Eq. 4), so the oracle recomputes a random sample
of rows of Y and all of Z from the same U, lambda, S and O; U and E are
checked through properties that hold at any size."""
import numpy as np
import pytest

import synth
from oracle import netmf, sketch as sk
from tests.util import rel, say

pytestmark = pytest.mark.gpu

N_SCALE = 20


@pytest.fixture(scope="module")
def big():
    from paper_2110_12782_amd.binding import DeviceGraph
    rowptr, colidx = synth.chung_lu(1 << N_SCALE, 2.1, 20.0, 2, 1003)
    A = netmf.adjacency(rowptr, colidx)
    return rowptr, colidx, A, DeviceGraph(rowptr, colidx)


def _params(prec, split):
    from paper_2110_12782_amd.binding import SketchParams
    return SketchParams(alpha=0.5, T=10, b=1.0, k=256, s_eig=32, q=2, d=128, h=272, l=1128, z=8, seed=7,
                        precision=prec, split_r=split)


# (1, 16): the form bench.py times
@pytest.mark.parametrize("prec,split,tol", [(1, 16, 1e-2), (1, 32, 1e-2), (2, 32, 1e-2), (0, 0, 1e-4)])
def test_fullsize_sketch_sampled_rows(lib, big, prec, split, tol):
    import torch
    rowptr, colidx, A, G = big
    p = _params(prec, split)
    nb = lib.workspace_size(p, G.n, G.nnz, 7)
    ws = lib.workspace(nb)
    U, lam = lib.eig(G, p, ws=ws)
    Yt, Z, S, O = lib.sketch(G, p, U, lam, ws=ws)
    E, sig = lib.embed(G.n, p, Yt, Z, O, ws=ws)
    flags = lib.sync()
    assert flags & ~1 == 0
    n = G.n
    rows = np.sort(np.random.default_rng(31).choice(n, size=4096, replace=False))
    Lp, Rp, _ = netmf.eq11_factors(U.cpu().numpy().astype(np.float64), lam.cpu().numpy(), netmf.degrees(A),
                                   netmf.volume(A), 0.5, 10, 1.0)
    rS, sS = S[0].cpu().numpy(), S[1].cpu().numpy()
    rO, sO = O[0].cpu().numpy(), O[1].cpu().numpy()
    Yo = sk.sketch_y_sampled(Lp, Rp, rS, sS, row_subset=rows)
    Zo = sk.sketch_z_sampled(Lp, Rp, rO, sO)
    Yg = Yt[:, torch.from_numpy(rows).cuda()].T.cpu().numpy().astype(np.float64)
    Zg = Z.cpu().numpy().astype(np.float64)
    ey = rel(Yg, Yo)
    ez = rel(Zg, Zo)
    # every column of Y (a group of the test matrix), every sampled row (a
    # vertex) and every column of Z on its own: one wrong tile or ragged tail
    # would be a small share of the aggregate but an O(1) error in its own
    # columns / rows.  (Single entries of Z are sums of z^2 terms that cancel,
    # so their relative error has no useful bound in BF16.)
    col = np.linalg.norm(Yg - Yo, axis=0) / np.linalg.norm(Yo, axis=0)
    row = np.linalg.norm(Yg - Yo, axis=1) / np.maximum(np.linalg.norm(Yo, axis=1), 1e-30)
    zcol = np.linalg.norm(Zg - Zo, axis=0) / np.linalg.norm(Zo, axis=0)
    # E = Q U_d Sigma_d^1/2 with Q orthonormal: E^T E = diag(sigma)
    EtE = (E.double().T @ E.double()).cpu().numpy()
    s = sig.cpu().numpy()
    ee = np.abs(EtE - np.diag(s)).max() / s[0]
    say(f"prec={prec} split={split}: Y rows rel {ey:.3e}  Z rel {ez:.3e}  E^T E vs diag(sigma) {ee:.2e}; "
        f"worst column {col.max():.2e}, worst row {row.max():.2e}, worst Z column {zcol.max():.2e}")
    assert ey <= tol and ez <= tol
    assert col.max() <= 2 * tol and row.max() <= 10 * tol and zcol.max() <= 5 * tol
    assert ee <= 1e-4
    assert np.all(np.diff(s) <= 1e-12 * s[0]) and np.all(s > 0)


@pytest.mark.parametrize("split", [0, 32])
def test_fullsize_fp16_range(lib, big, split):
    """FP16 operands hold |x| < 65504, but R' (which carries vol / (bT), Eq. 11)
    exceeds that on this graph; the library balances L' and R' by a power of
    two.  S and O are made to touch the vertex with the largest |R'| entry,
    and that row of Y, sampled rows and all of Z must meet the bar with no
    non-finite flag."""
    import torch
    rowptr, colidx, A, G = big
    p = _params(2, split)
    nb = lib.workspace_size(p, G.n, G.nnz, 7)
    ws = lib.workspace(nb)
    U, lam = lib.eig(G, p, ws=ws)
    assert lib.sync() & ~1 == 0
    deg, vol = netmf.degrees(A), netmf.volume(A)
    Lp, Rp, _ = netmf.eq11_factors(U.cpu().numpy().astype(np.float64), lam.cpu().numpy(), deg, vol, 0.5, 10, 1.0)
    colmax = np.abs(Rp).max(axis=0) * vol / 10.0  # the GPU's R' side carries vol / (bT)
    hub = int(np.argmax(colmax))
    rS, sS = synth.sparse_sign(G.n, p.h, p.z, 3101)
    rO, sO = synth.sparse_sign(G.n, p.l, p.z, 4101)
    for r in (rS, rO):
        if hub not in r[0]:
            r[0, 0] = hub
    say(f"fp16 split={split}: max |R'| {colmax.max():.3e} at vertex {hub}")
    assert colmax.max() > 65504  # the case the balance exists for
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Yt, Z, _, _ = lib.sketch(G, p, U, lam, S=(dev(rS), dev(sS)), O=(dev(rO), dev(sO)), ws=ws)
    flags = lib.sync()
    assert flags & ~1 == 0
    rows = np.unique(np.concatenate([[hub], np.random.default_rng(32).choice(G.n, size=2048, replace=False)]))
    Yo = sk.sketch_y_sampled(Lp, Rp, rS, sS, row_subset=rows)
    Zo = sk.sketch_z_sampled(Lp, Rp, rO, sO)
    Yg = Yt[:, torch.from_numpy(rows).cuda()].T.cpu().numpy().astype(np.float64)
    ey, ez = rel(Yg, Yo), rel(Z.cpu().numpy().astype(np.float64), Zo)
    hub_row = rel(Yg[rows == hub], Yo[rows == hub])
    say(f"  Y rows rel {ey:.3e}  hub row {hub_row:.3e}  Z rel {ez:.3e}")
    assert np.isfinite(Yg).all() and np.isfinite(Z.cpu().numpy()).all()
    assert ey <= 1e-2 and ez <= 1e-2 and hub_row <= 1e-2


def test_fullsize_calls_only_enqueue(lib, big):
    """sketchne_eig, sketchne_sketch and sketchne_embed enqueue their work and
    return without waiting for the device: right after the three calls the
    stream still has work in flight (the step takes tens of milliseconds), and
    the results equal those of a run that waits after each call."""
    import torch
    rowptr, colidx, A, G = big
    p = _params(1, 16)
    nb = lib.workspace_size(p, G.n, G.nnz, 7)
    ws = lib.workspace(nb)

    def run(wait):
        U, lam = lib.eig(G, p, ws=ws)
        if wait:
            torch.cuda.synchronize()
        Yt, Z, S, O = lib.sketch(G, p, U, lam, ws=ws)
        if wait:
            torch.cuda.synchronize()
        E, sig = lib.embed(G.n, p, Yt, Z, O, ws=ws)
        return E, sig

    run(True)
    torch.cuda.synchronize()
    E, sig = run(False)
    busy = not torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    assert lib.sync() & ~1 == 0
    E2, sig2 = run(True)
    assert lib.sync() & ~1 == 0
    say(f"stream busy right after the three calls: {busy}")
    assert busy
    assert torch.equal(E, E2) and torch.equal(sig, sig2)


def test_fullsize_eig_properties(lib, big):
    """U orthonormal; lambda equal to the Rayleigh quotients diag(U^T X U) and
    inside the spectrum [-1, 1] of D^-1/2 A D^-1/2; the Ritz residuals of the
    library equal ||X U_j - lambda_j U_j|| formed here.  (At this size and
    q = 2 the top Ritz value is not 1: the spectrum has a dense cluster near
    1 that two power iterations do not resolve -- method error, not parity.)"""
    import torch
    rowptr, colidx, A, G = big
    p = _params(1, 32)
    U, lam_d = lib.eig(G, p)
    XU = lib.spmm(G, 0.5, U)
    res = lib.ritz_residual(G, 0.5, U, lam_d)
    assert lib.sync() & ~1 == 0
    Ud = U.double()
    orth = float((Ud.T @ Ud - torch.eye(p.k, dtype=torch.float64, device="cuda")).abs().max())
    rq = (Ud * XU.double()).sum(dim=0).cpu().numpy()
    lam = lam_d.cpu().numpy()
    e_rq = np.abs(rq - lam).max()
    res_ref = torch.linalg.vector_norm(XU.double() - Ud * lam_d[None, :], dim=0).cpu().numpy()
    e_res = np.abs(res.cpu().numpy() - res_ref).max() / res_ref.max()
    say(f"orth {orth:.2e}  |diag(U^T X U) - lambda| {e_rq:.2e}  lambda_1 {lam[0]:.6f}  lambda_k {lam[-1]:.6f}  "
        f"max Ritz residual {res_ref.max():.3e} (library vs here {e_res:.1e})")
    assert orth <= 1e-5
    assert e_rq <= 1e-5
    assert np.all(np.abs(lam) <= 1 + 1e-6)
    assert np.all(np.diff(np.abs(lam)) <= 1e-12)
    assert e_res <= 1e-9
