"""The scale case: R-MAT with 2^28 edges over 2^24 vertices, (a, b, c, d) =
(0.57, 0.19, 0.19, 0.05), symmetrized and deduplicated; k = 256, q = 2,
d = 128, h = 272, l = 1128, z = 8, BF16 fused sketch with split 32.

The whole path runs at full size; the FP64 oracle recomputes a random sample
of rows of Y and all of Z from the GPU's U and lambda (Eq. 11 in row-subset
form), and E is checked through E^T E = diag(sigma).  SpMM bandwidth and the
fused kernel's MFMA rate are printed."""
import numpy as np
import pytest

from oracle import netmf, sketch as sk
from tests.util import rel, say

pytestmark = pytest.mark.gpu


def test_rmat_scale_sampled_parity(lib):
    import torch
    from synth.graphs_device import rmat_device
    from paper_2110_12782_amd.binding import DeviceGraph, SketchParams
    rowptr_d, colidx_d = rmat_device(24, 1 << 28, 0.57, 0.19, 0.19, 0.05, 1004)
    G = DeviceGraph.from_device(rowptr_d, colidx_d)
    deg = torch.diff(rowptr_d).cpu().numpy()
    n, nnz = G.n, G.nnz
    say(f"R-MAT scale 24: n={n} nnz={nnz} isolated={(deg == 0).sum()} max degree={deg.max()}")
    p = SketchParams(alpha=0.5, T=10, b=1.0, k=256, s_eig=32, q=2, d=128, h=272, l=1128, z=8, seed=11,
                     precision=1, split_r=32)
    nb = lib.workspace_size(p, n, nnz, 7)
    say(f"workspace {nb / 2**30:.1f} GiB")
    ws = lib.workspace(nb)
    lib.profile_enable(True)
    U, lam = lib.eig(G, p, ws=ws)
    Yt, Z, S, O = lib.sketch(G, p, U, lam, ws=ws)
    E, sig = lib.embed(n, p, Yt, Z, O, ws=ws)
    prof = lib.profile_read()
    lib.profile_enable(False)
    assert lib.sync() & ~1 == 0
    sp_ms = prof["spmm"][0] / prof["spmm"][1]
    rS, sS = S[0].cpu().numpy(), S[1].cpu().numpy()
    rO, sO = O[0].cpu().numpy(), O[1].cpu().numpy()
    pS, pO = sk.unique_rows(rS), sk.unique_rows(rO)
    y_ms = prof["sketch_y"][0]
    say(f"SpMM {sp_ms:.1f} ms per launch = {nnz * (4 + 4 * 288) / sp_ms / 1e9:.2f} TB/s (no-reuse model); "
        f"fused Y {y_ms:.2f} ms = {2 * 256 * n * len(pS) / y_ms / 1e9:.0f} TFLOP/s algorithmic; "
        + ", ".join(f"{k} {v[0]:.1f} ms" for k, v in prof.items()))
    # oracle on a row sample (rows of Y are independent, Eq. 4) and all of Z
    U_h = U.cpu().numpy()
    lam_h = lam.cpu().numpy()
    Kmat = netmf.eq11_kmat(U_h, lam_h, deg, 0.5)
    rows = np.sort(np.random.default_rng(41).choice(np.flatnonzero(deg > 0), size=2048, replace=False))
    L_rows, _ = netmf.eq11_rows(U_h[rows], deg[rows], lam_h, Kmat, float(nnz), 0.5, 10, 1.0)
    _, R_p = netmf.eq11_rows(U_h[pS], deg[pS], lam_h, Kmat, float(nnz), 0.5, 10, 1.0)
    Yo = sk.sketch_y_rows(L_rows, R_p, n, rS, sS)
    Lo, Ro = netmf.eq11_rows(U_h[pO], deg[pO], lam_h, Kmat, float(nnz), 0.5, 10, 1.0)
    Zo = sk.sketch_z_parts(Lo, Ro, n, rO, sO)
    ey = rel(Yt[:, torch.from_numpy(rows).cuda()].T.cpu().numpy(), Yo)
    ez = rel(Z.cpu().numpy(), Zo)
    EtE = (E.double().T @ E.double()).cpu().numpy()
    s = sig.cpu().numpy()
    ee = np.abs(EtE - np.diag(s)).max() / s[0]
    # isolated vertices: their rows of U, Y and E are zero
    iso = torch.from_numpy(np.flatnonzero(deg == 0)[:1000]).cuda()
    zero_rows = bool((U[iso] == 0).all() and (Yt[:, iso] == 0).all() and (E[iso] == 0).all())
    say(f"Y rows rel {ey:.3e}  Z rel {ez:.3e}  E^T E vs diag(sigma) {ee:.2e}  isolated rows zero {zero_rows}")
    assert ey <= 1e-2 and ez <= 1e-2
    assert ee <= 1e-4
    assert zero_rows
