"""Guard bands around every output and the workspace: the sketch and embed
calls, in the shapes whose edges the kernels handle by range checks (a
ragged vertex count, z < 8, h and l off the tile sizes, the Z pass split over
workgroups), must not write a byte outside the buffers they are given."""
import ctypes as C

import numpy as np
import pytest

import synth
from tests.util import say

pytestmark = pytest.mark.gpu

GUARD = 4096          # floats on each side of an output
WS_GUARD = 1 << 16    # bytes after the workspace
SENTINEL = 0x7FC0DEAD  # a NaN payload no kernel writes


def _guarded(torch, count, dtype=np.float32):
    """A device buffer with `count` elements between two sentinel bands;
    returns (whole int32 view, pointer to the payload)."""
    itemsize = np.dtype(dtype).itemsize
    words = (count * itemsize + 3) // 4
    whole = torch.full((GUARD + words + GUARD,), SENTINEL, dtype=torch.int32, device="cuda")
    return whole, whole.data_ptr() + 4 * GUARD, words


def _bands_intact(whole, words):
    w = whole.cpu().numpy()
    return bool(np.all(w[:GUARD] == SENTINEL) and np.all(w[GUARD + words:] == SENTINEL))


@pytest.mark.parametrize("prec,split", [(0, 0), (1, 16), (2, 0)])
def test_outputs_and_workspace_guards(lib, prec, split):
    import torch
    from paper_2110_12782_amd.binding import (DeviceGraph, SketchParams, SparseSign, OP_EIG, OP_SKETCH, OP_EMBED)
    n = 4099  # ragged: not a multiple of the 32-vertex tile
    say(f"guard bands n={n} z=5 h=21 l=70 prec={prec} split={split}")
    rowptr, colidx = synth.chung_lu(n, 2.1, 12, 2, 55)
    g = DeviceGraph(rowptr, colidx)
    p = SketchParams(alpha=0.5, T=10, k=32, s_eig=16, q=1, d=8, h=21, l=70, z=5, seed=4, precision=prec,
                     split_r=split)
    U, lam = lib.eig(g, p)
    assert lib.sync() & ~1 == 0
    # workspace: the size the library asks for, then a sentinel band
    nb = lib.workspace_size(p, g.n, g.nnz, OP_SKETCH | OP_EMBED)
    ws_whole = torch.full(((nb + WS_GUARD + 512) // 4,), SENTINEL, dtype=torch.int32, device="cuda")
    base = ws_whole.data_ptr()
    ws_ptr = base + ((-base) % 256)
    Yw, Yp, Yn = _guarded(torch, p.h * n)
    Zw, Zp, Zn = _guarded(torch, p.l * p.l)
    rows_s = torch.empty((p.h, p.z), dtype=torch.int32, device="cuda")
    signs_s = torch.empty((p.h, p.z), dtype=torch.int8, device="cuda")
    rows_o = torch.empty((p.l, p.z), dtype=torch.int32, device="cuda")
    signs_o = torch.empty((p.l, p.z), dtype=torch.int8, device="cuda")
    Ss = SparseSign(p.h, p.z, rows_s.data_ptr(), signs_s.data_ptr())
    Os = SparseSign(p.l, p.z, rows_o.data_ptr(), signs_o.data_ptr())
    pc, gc = p.c(), g.c()
    lib.check(lib.lib.sketchne_sketch(lib.ctx(), C.byref(gc), C.byref(pc), C.c_void_p(U.data_ptr()),
                                      C.c_void_p(lam.data_ptr()), C.byref(Ss), C.byref(Os), 1, C.c_void_p(Yp),
                                      C.c_void_p(Zp), C.c_void_p(ws_ptr), nb), "sketch")
    Ew, Ep, En = _guarded(torch, n * p.d)
    sw, sp, sn = _guarded(torch, p.d, np.float64)
    lib.check(lib.lib.sketchne_embed(lib.ctx(), C.byref(pc), n, C.c_void_p(Yp), C.c_void_p(Zp), C.byref(Os),
                                     C.c_void_p(Ep), C.c_void_p(sp), C.c_void_p(ws_ptr), nb), "embed")
    assert lib.sync() & ~1 == 0
    for name, (whole, words) in {"Yt": (Yw, Yn), "Z": (Zw, Zn), "E": (Ew, En), "sigma": (sw, sn)}.items():
        assert _bands_intact(whole, words), name
    tail = ws_whole.cpu().numpy().view(np.uint8)[ws_ptr - base + nb:ws_ptr - base + nb + WS_GUARD]
    assert np.all(tail.view(np.int32) == SENTINEL), "workspace"
    # and the payloads were written (no sentinel left inside Y)
    Y = Yw.cpu().numpy()[GUARD:GUARD + Yn]
    assert not np.any(Y == SENTINEL)
