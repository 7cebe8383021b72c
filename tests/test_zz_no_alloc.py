"""The workspace-free eigensolver entry point (sketchne_symeig_noalloc)
against sketchne_symeig, through the C ABI: two calls in a row on the
library's device scratch, the second of smaller order, each bit-identical to
the workspace entry point on the same input, plus the size limit."""
import numpy as np
import pytest

from tests.util import say

pytestmark = pytest.mark.gpu


def test_symeig_noalloc_matches_workspace_entry(lib):
    import torch
    from paper_2110_12782_amd.binding import SketchneError
    rng = np.random.default_rng(41)
    for m in (288, 100):  # the second call is smaller: stale scratch from the first must not leak in
        say(f"symeig_noalloc m={m} against symeig")
        M = rng.standard_normal((m, m))
        A = torch.from_numpy(M + M.T).cuda()
        Vn, wn = lib.symeig_noalloc(A)
        V, w = lib.symeig(A)
        assert lib.sync() == 0
        assert torch.equal(Vn, V) and torch.equal(wn, w)
        # and against the definition: A V = V diag(w), V orthonormal
        Vc, wc, Ac = Vn.cpu().numpy(), wn.cpu().numpy(), A.cpu().numpy()
        scale = np.abs(wc).max()
        assert np.abs(Ac @ Vc - Vc * wc).max() < 1e-12 * scale * max(1, m / 16)
        assert np.abs(Vc.T @ Vc - np.eye(m)).max() < 1e-12 * max(1, m / 16)
    A = torch.zeros((289, 289), dtype=torch.float64, device="cuda")
    with pytest.raises(SketchneError):
        lib.symeig_noalloc(A)
