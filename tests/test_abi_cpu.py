"""The C-ABI library loads and exports every symbol the header declares; the
host-only parts of the ABI (workspace sizing, argument validation that runs
before anything is enqueued) behave as documented.  No GPU is used."""
import ctypes as C
import os
import re

import pytest

from paper_2110_12782_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sketchne.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sketchne_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libsketchne.so is not built (run __graft_entry__.build())")
    return B.Library(need_gpu=False)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib.lib, name), f"{name} declared in sketchne.h but not exported"
    assert set(names) == set(B.EXPORTED)


def test_status_strings(lib):
    for st in range(6):
        assert lib.lib.sketchne_status_str(st)
    assert b"invalid" in lib.lib.sketchne_status_str(B.E_ARG)


def test_workspace_sizes_scale(lib):
    p = B.SketchParams(k=256, s_eig=32, d=128, h=272, l=1128, z=8)
    small = lib.workspace_size(p, 65536, 1 << 20, B.OP_EIG | B.OP_SKETCH | B.OP_EMBED)
    big = lib.workspace_size(p, 1 << 20, 21 << 20, B.OP_EIG | B.OP_SKETCH | B.OP_EMBED)
    assert 0 < small < big
    # eig holds three n x K FP32 blocks at least
    assert lib.workspace_size(p, 1 << 20, 21 << 20, B.OP_EIG) >= 3 * (1 << 20) * 288 * 4
    bf = B.SketchParams(k=256, s_eig=32, d=128, h=272, l=1128, z=8, precision=B.BF16, split_r=32)
    assert lib.workspace_size(bf, 1 << 20, 0, B.OP_SKETCH) > 0


@pytest.mark.parametrize("field,value", [
    ("alpha", 0.0), ("alpha", 0.6), ("T", 0), ("b", 0.0), ("k", 0), ("q", -1),
    ("d", 0), ("h", 100), ("l", 200), ("z", 0), ("precision", 3), ("split_r", -1),
])
def test_invalid_params_rejected(lib, field, value):
    p = B.SketchParams(k=128, s_eig=32, d=128, h=272, l=1128, z=8)
    setattr(p, field, value)
    pc = p.c()
    out = C.c_size_t(0)
    st = lib.lib.sketchne_workspace_size(C.byref(pc), 65536, 1 << 20, B.OP_SKETCH, C.byref(out))
    assert st == B.E_ARG


def test_k_larger_than_n_rejected(lib):
    p = B.SketchParams(k=256, s_eig=32, d=8, h=16, l=32, z=8)
    pc = p.c()
    out = C.c_size_t(0)
    assert lib.lib.sketchne_workspace_size(C.byref(pc), 200, 1000, B.OP_EIG, C.byref(out)) == B.E_ARG


def test_null_context_and_pointers_rejected_before_any_work(lib):
    p = B.SketchParams(k=8, s_eig=8, d=4, h=8, l=16, z=4).c()
    g = B.Graph(100, 0, None, None)
    L = lib.lib
    assert L.sketchne_eig(None, C.byref(g), C.byref(p), None, None, None, None, 0) == B.E_ARG
    assert L.sketchne_sketch(None, C.byref(g), C.byref(p), None, None, None, None, 0, None, None, None, 0) == B.E_ARG
    assert L.sketchne_embed(None, C.byref(p), 100, None, None, None, None, None, None, 0) == B.E_ARG
    assert L.sketchne_sync(None, None) == B.E_ARG
    assert L.sketchne_destroy(None) == B.E_ARG
    out = C.c_size_t(0)
    assert L.sketchne_orth_workspace_size(0, 4, C.byref(out)) == B.E_ARG
    assert L.sketchne_symeig_workspace_size(0, C.byref(out)) == B.E_ARG
    # the Jacobi workspace holds G = B V (m x m FP64); V itself is never formed
    assert L.sketchne_symeig_workspace_size(288, C.byref(out)) == B.OK and out.value >= 288 * 288 * 8


def test_warm_start_param_count_and_workspace(lib):
    w, o = 256, 256
    assert lib.ws_param_count(w, o) == 8 * w + w + w * w + w + w * o + o
    L = lib.lib
    cnt = C.c_int64(0)
    assert L.sketchne_ws_param_count(0, 4, C.byref(cnt)) == B.E_ARG
    fwd = lib.ws_workspace_size(w, o, 1 << 20, 0, B.WS_OP_FORWARD)
    grad = lib.ws_workspace_size(w, o, 1 << 20, 0, B.WS_OP_GRAD)
    assert fwd >= 2 * (1 << 20) * w * 4 and grad > fwd
    p = B.SketchParams(k=256, s_eig=32, d=128, h=272, l=1128, z=8)
    eig = lib.ws_workspace_size(w, o, 1 << 20, 21 << 20, B.WS_OP_EIG, p)
    assert eig > lib.workspace_size(p, 1 << 20, 21 << 20, B.OP_EIG)
    out = C.c_size_t(0)
    # the eigensolver ops need the parameters
    assert L.sketchne_ws_workspace_size(None, w, o, 1000, 5000, B.WS_OP_EIG, C.byref(out)) == B.E_ARG


def test_warm_start_null_arguments_rejected(lib):
    L = lib.lib
    net = B.MLPStruct(256, 64, None, None, None, None)
    g = B.Graph(100, 0, None, None)
    p = B.SketchParams(k=8, s_eig=8, d=4, h=8, l=16, z=4).c()
    assert L.sketchne_ws_init(None, C.byref(net), 1) == B.E_ARG
    assert L.sketchne_ws_forward(None, C.byref(net), 10, None, None, 64, None, 0) == B.E_ARG
    assert L.sketchne_ws_infer(None, C.byref(net), 10, None, None, 64, None, 0) == B.E_ARG
    assert L.sketchne_ws_grad(None, C.byref(net), 10, None, None, 64, 0.1, None, None, None, 0) == B.E_ARG
    assert L.sketchne_ws_adam(None, C.byref(net), None, 1e-3, 1) == B.E_ARG
    assert L.sketchne_ritz_residual(None, C.byref(g), 0.5, 8, None, None, None, None, 0) == B.E_ARG
    fb = C.c_int32(0)
    assert L.sketchne_eig_learned(None, C.byref(g), C.byref(p), C.byref(net), 1, 1.0, None, None, C.byref(fb),
                                  None, None, 0) == B.E_ARG


def test_profile_constants_match_header():
    # the binding's class names and selection bit are the header's macros
    text = open(HEADER).read()
    macros = dict(re.findall(r"#define\s+SKETCHNE_PROF_(\w+)\s+(0x[0-9a-fA-F]+|\d+)", text))
    assert int(macros["SELECT"], 0) == B.PROF_SELECT
    assert int(macros["CLASSES"], 0) == len(B.PROF_NAMES)
    for i, name in enumerate(B.PROF_NAMES):
        assert int(macros[name.upper()], 0) == i, name
    assert B.PROF_SELECT >> int(macros["CLASSES"]) != 0  # the selection bit lies above every class bit


def test_profile_calls_without_context_rejected(lib):
    ms = (C.c_double * len(B.PROF_NAMES))()
    n = (C.c_int64 * len(B.PROF_NAMES))()
    assert lib.lib.sketchne_profile_enable(None, 1) == B.E_ARG
    assert lib.lib.sketchne_profile_enable(None, B.PROF_SELECT | 1) == B.E_ARG
    assert lib.lib.sketchne_profile_read(None, ms, n) == B.E_ARG
