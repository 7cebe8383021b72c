"""ctypes binding of libsketchne (argument marshalling only).

PyTorch provides device memory and the stream; every step of the method runs
in the library's HIP kernels.  There is no fallback: if the library or a GPU
is missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsketchne.so")

OK, E_ARG, E_WORKSPACE, E_DEVICE, E_NUMERIC, E_UNSUPPORTED = range(6)
FP32, BF16, FP16 = 0, 1, 2
OP_EIG, OP_SKETCH, OP_EMBED, OP_SPMM = 1, 2, 4, 8
PROF_NAMES = ["spmm", "sketch_y", "sketch_z", "gemm64", "small", "prep", "propagate"]
PROF_SELECT = 0x40000000  # with class bits: time only those classes

EXPORTED = [
    "sketchne_status_str", "sketchne_create", "sketchne_destroy", "sketchne_set_stream",
    "sketchne_workspace_size", "sketchne_eig", "sketchne_sketch", "sketchne_embed", "sketchne_sync",
    "sketchne_spmm", "sketchne_orth_workspace_size", "sketchne_orth", "sketchne_symeig_workspace_size",
    "sketchne_symeig", "sketchne_gen_gauss", "sketchne_gen_sparse_sign", "sketchne_profile_enable",
    "sketchne_profile_read", "sketchne_ws_param_count", "sketchne_ws_workspace_size", "sketchne_ws_init",
    "sketchne_ws_features", "sketchne_ws_forward", "sketchne_ws_grad", "sketchne_ws_adam",
    "sketchne_ritz_residual", "sketchne_eig_learned", "sketchne_ws_train", "sketchne_ws_infer",
    "sketchne_propagate_coeffs", "sketchne_propagate_workspace_size", "sketchne_propagate",
    "sketchne_symeig_noalloc", "sketchne_general_workspace_size", "sketchne_sketch_general",
    "sketchne_embed_general", "sketchne_fullvisit_workspace_size", "sketchne_sketch_fullvisit",
    "sketchne_embed_fullvisit",
]
WS_FEAT = 8
WS_OP_FEATURES, WS_OP_FORWARD, WS_OP_GRAD, WS_OP_RESIDUAL, WS_OP_EIG = 1, 2, 4, 8, 16


class SketchneError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


class Graph(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("colidx", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [
        ("alpha", C.c_double), ("T", C.c_int32), ("b", C.c_double),
        ("k", C.c_int32), ("s_eig", C.c_int32), ("q", C.c_int32),
        ("d", C.c_int32), ("h", C.c_int32), ("l", C.c_int32), ("z", C.c_int32),
        ("seed", C.c_uint64), ("precision", C.c_int32), ("split_r", C.c_int32),
    ]


class MLPStruct(C.Structure):
    _fields_ = [("width", C.c_int32), ("out", C.c_int32), ("master", C.c_void_p), ("bf16", C.c_void_p),
                ("adam_m", C.c_void_p), ("adam_v", C.c_void_p)]


class SparseSign(C.Structure):
    _fields_ = [("cols", C.c_int32), ("z", C.c_int32), ("rows", C.c_void_p), ("signs", C.c_void_p)]


class RowSign(C.Structure):
    _fields_ = [("width", C.c_int32), ("z", C.c_int32), ("cols", C.c_void_p), ("signs", C.c_void_p)]


@dataclass
class SketchParams:
    """Hyper-parameters (Table 1 notation)."""
    alpha: float = 0.5
    T: int = 10
    b: float = 1.0
    k: int = 256
    s_eig: int = 32
    q: int = 2
    d: int = 128
    h: int = 272
    l: int = 1128
    z: int = 8
    seed: int = 1
    precision: int = FP32
    split_r: int = 0

    def c(self) -> Params:
        return Params(self.alpha, self.T, self.b, self.k, self.s_eig, self.q, self.d, self.h, self.l,
                      self.z, self.seed, self.precision, self.split_r)


def _ptr(t) -> int:
    return 0 if t is None else t.data_ptr()


class Library:
    _inst = None

    @classmethod
    def get(cls) -> "Library":
        if cls._inst is None:
            cls._inst = Library()
        return cls._inst

    def __init__(self, path: str = LIB_PATH, need_gpu: bool = True):
        import torch  # noqa: F401  (load torch's HIP runtime first so both share it)
        if not os.path.exists(path):
            raise RuntimeError(f"libsketchne not built: {path} is missing (run __graft_entry__.build())")
        self.lib = C.CDLL(path)
        L = self.lib
        L.sketchne_status_str.restype = C.c_char_p
        L.sketchne_status_str.argtypes = [C.c_int]
        for name in EXPORTED[1:]:
            getattr(L, name).restype = C.c_int
        L.sketchne_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]
        L.sketchne_destroy.argtypes = [C.c_void_p]
        L.sketchne_set_stream.argtypes = [C.c_void_p, C.c_void_p]
        L.sketchne_workspace_size.argtypes = [C.POINTER(Params), C.c_int64, C.c_int64, C.c_int, C.POINTER(C.c_size_t)]
        L.sketchne_eig.argtypes = [C.c_void_p, C.POINTER(Graph), C.POINTER(Params), C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_sketch.argtypes = [C.c_void_p, C.POINTER(Graph), C.POINTER(Params), C.c_void_p, C.c_void_p,
                                      C.POINTER(SparseSign), C.POINTER(SparseSign), C.c_int, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_embed.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p,
                                     C.POINTER(SparseSign), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_sync.argtypes = [C.c_void_p, C.POINTER(C.c_uint32)]
        L.sketchne_spmm.argtypes = [C.c_void_p, C.POINTER(Graph), C.c_double, C.c_void_p, C.c_int64, C.c_int32,
                                    C.c_void_p, C.c_int64, C.c_void_p, C.c_size_t]
        L.sketchne_orth_workspace_size.argtypes = [C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]
        L.sketchne_orth.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                                    C.c_size_t]
        L.sketchne_symeig_workspace_size.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
        L.sketchne_symeig.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_size_t]
        L.sketchne_gen_gauss.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_void_p]
        L.sketchne_gen_sparse_sign.argtypes = [C.c_void_p, C.c_int64, C.c_uint64, C.POINTER(SparseSign)]
        L.sketchne_profile_enable.argtypes = [C.c_void_p, C.c_int]
        L.sketchne_profile_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.sketchne_ws_param_count.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int64)]
        L.sketchne_ws_workspace_size.argtypes = [C.POINTER(Params), C.c_int32, C.c_int32, C.c_int64, C.c_int64,
                                                 C.c_int, C.POINTER(C.c_size_t)]
        L.sketchne_ws_init.argtypes = [C.c_void_p, C.POINTER(MLPStruct), C.c_uint64]
        L.sketchne_ws_features.argtypes = [C.c_void_p, C.POINTER(Graph), C.c_double, C.c_void_p, C.c_uint64,
                                           C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_ws_forward.argtypes = [C.c_void_p, C.POINTER(MLPStruct), C.c_int64, C.c_void_p, C.c_void_p,
                                          C.c_int64, C.c_void_p, C.c_size_t]
        L.sketchne_ws_infer.argtypes = L.sketchne_ws_forward.argtypes
        L.sketchne_ws_grad.argtypes = [C.c_void_p, C.POINTER(MLPStruct), C.c_int64, C.c_void_p, C.c_void_p,
                                       C.c_int64, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_ws_adam.argtypes = [C.c_void_p, C.POINTER(MLPStruct), C.c_void_p, C.c_float, C.c_int32]
        L.sketchne_ws_train.argtypes = [C.c_void_p, C.POINTER(MLPStruct), C.c_int32, C.POINTER(C.c_void_p),
                                        C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_int32, C.c_int32, C.c_float,
                                        C.c_float, C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_ritz_residual.argtypes = [C.c_void_p, C.POINTER(Graph), C.c_double, C.c_int32, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_eig_learned.argtypes = [C.c_void_p, C.POINTER(Graph), C.POINTER(Params), C.POINTER(MLPStruct),
                                           C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32),
                                           C.POINTER(C.c_double), C.c_void_p, C.c_size_t]
        L.sketchne_general_workspace_size.argtypes = [C.POINTER(Params), C.c_int64, C.c_int32, C.c_int,
                                                      C.POINTER(C.c_size_t)]
        L.sketchne_sketch_general.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p,
                                              C.POINTER(Params), C.POINTER(SparseSign), C.POINTER(SparseSign),
                                              C.POINTER(SparseSign), C.POINTER(SparseSign), C.c_void_p, C.c_void_p,
                                              C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_embed_general.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p,
                                             C.c_void_p, C.POINTER(SparseSign), C.POINTER(SparseSign), C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_fullvisit_workspace_size.argtypes = [C.POINTER(Params), C.c_int64, C.c_int, C.POINTER(C.c_size_t)]
        L.sketchne_sketch_fullvisit.argtypes = [C.c_void_p, C.POINTER(Graph), C.POINTER(Params), C.c_void_p,
                                                C.c_void_p, C.POINTER(RowSign), C.POINTER(RowSign), C.c_int,
                                                C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_embed_fullvisit.argtypes = [C.c_void_p, C.POINTER(Params), C.c_int64, C.c_void_p, C.c_void_p,
                                               C.POINTER(RowSign), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]
        L.sketchne_symeig_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.sketchne_propagate_coeffs.argtypes = [C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.sketchne_propagate_workspace_size.argtypes = [C.c_int64, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]
        L.sketchne_propagate.argtypes = [C.c_void_p, C.POINTER(Graph), C.c_int32, C.c_void_p, C.c_int64, C.c_int32,
                                         C.POINTER(C.c_double), C.c_void_p, C.c_int64, C.c_void_p, C.c_size_t]
        self._ctx = None

    # ---------------------------------------------------------------- helpers
    def check(self, st: int, where: str):
        if st != OK:
            raise SketchneError(st, where, self.lib.sketchne_status_str(st).decode())

    def workspace_size(self, p: SketchParams, n: int, nnz: int, ops: int) -> int:
        out = C.c_size_t(0)
        pc = p.c()
        self.check(self.lib.sketchne_workspace_size(C.byref(pc), n, nnz, ops, C.byref(out)), "workspace_size")
        return out.value

    def ctx(self):
        """The library context bound to cuda:0 and torch's current stream."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("sketchne needs a GPU: torch.cuda.is_available() is False")
        if self._ctx is None:
            h = C.c_void_p()
            self.check(self.lib.sketchne_create(C.byref(h), 0, C.c_void_p(torch.cuda.current_stream().cuda_stream)),
                       "create")
            self._ctx = h
        self.lib.sketchne_set_stream(self._ctx, C.c_void_p(torch.cuda.current_stream().cuda_stream))
        return self._ctx

    @staticmethod
    def workspace(nbytes: int):
        import torch
        return torch.empty(max(nbytes, 256) + 256, dtype=torch.uint8, device="cuda")

    @staticmethod
    def _aligned(buf):
        p = buf.data_ptr()
        return p + ((-p) % 256)

    def sync(self) -> int:
        f = C.c_uint32(0)
        st = self.lib.sketchne_sync(self.ctx(), C.byref(f))
        self.check(st, "sync")
        return f.value

    # ---------------------------------------------------------------- the path
    def eig(self, g: "DeviceGraph", p: SketchParams, omega0=None, ws=None):
        """Alg. 5 on D^-a A D^-a; returns U (n x k float32), lambda (k float64)."""
        import torch
        K = p.k + p.s_eig
        U = torch.empty((g.n, p.k), dtype=torch.float32, device="cuda")
        lam = torch.empty(p.k, dtype=torch.float64, device="cuda")
        if omega0 is not None:
            assert omega0.dtype == torch.float32 and omega0.is_contiguous() and tuple(omega0.shape) == (g.n, K)
        nb = self.workspace_size(p, g.n, g.nnz, OP_EIG)
        ws = ws if ws is not None else self.workspace(nb)
        pc = p.c()
        gs = g.c()
        self.check(self.lib.sketchne_eig(self.ctx(), C.byref(gs), C.byref(pc), C.c_void_p(_ptr(omega0)),
                                         C.c_void_p(U.data_ptr()), C.c_void_p(lam.data_ptr()),
                                         C.c_void_p(self._aligned(ws)), nb), "eig")
        return U, lam

    def sketch(self, g: "DeviceGraph", p: SketchParams, U, lam, S=None, O=None, ws=None):
        """Y (returned transposed, h x n) and Z (l x l).  S, O: (rows, signs)
        int32/int8 device tensors of shape (cols, z), or None to draw on the
        device (then they are returned)."""
        import torch
        generate = S is None or O is None
        if generate:
            S = (torch.empty((p.h, p.z), dtype=torch.int32, device="cuda"),
                 torch.empty((p.h, p.z), dtype=torch.int8, device="cuda"))
            O = (torch.empty((p.l, p.z), dtype=torch.int32, device="cuda"),
                 torch.empty((p.l, p.z), dtype=torch.int8, device="cuda"))
        Ss = SparseSign(p.h, p.z, S[0].data_ptr(), S[1].data_ptr())
        Os = SparseSign(p.l, p.z, O[0].data_ptr(), O[1].data_ptr())
        Yt = torch.empty((p.h, g.n), dtype=torch.float32, device="cuda")
        Z = torch.empty((p.l, p.l), dtype=torch.float32, device="cuda")
        nb = self.workspace_size(p, g.n, g.nnz, OP_SKETCH)
        ws = ws if ws is not None else self.workspace(nb)
        pc = p.c()
        gs = g.c()
        self.check(self.lib.sketchne_sketch(self.ctx(), C.byref(gs), C.byref(pc), C.c_void_p(U.data_ptr()),
                                            C.c_void_p(lam.data_ptr()), C.byref(Ss), C.byref(Os), int(generate),
                                            C.c_void_p(Yt.data_ptr()), C.c_void_p(Z.data_ptr()),
                                            C.c_void_p(self._aligned(ws)), nb), "sketch")
        return Yt, Z, S, O

    def embed(self, n: int, p: SketchParams, Yt, Z, O, ws=None):
        """E (n x d float32) and sigma (d float64)."""
        import torch
        E = torch.empty((n, p.d), dtype=torch.float32, device="cuda")
        sig = torch.empty(p.d, dtype=torch.float64, device="cuda")
        Os = SparseSign(p.l, p.z, O[0].data_ptr(), O[1].data_ptr())
        nb = self.workspace_size(p, n, 0, OP_EMBED)
        ws = ws if ws is not None else self.workspace(nb)
        pc = p.c()
        self.check(self.lib.sketchne_embed(self.ctx(), C.byref(pc), n, C.c_void_p(Yt.data_ptr()),
                                           C.c_void_p(Z.data_ptr()), C.byref(Os), C.c_void_p(E.data_ptr()),
                                           C.c_void_p(sig.data_ptr()), C.c_void_p(self._aligned(ws)), nb), "embed")
        return E, sig

    # ---------------------------------------------------------------- general single pass
    def general_workspace_size(self, p: SketchParams, n: int, k: int, ops: int) -> int:
        out = C.c_size_t(0)
        pc = p.c()
        self.check(self.lib.sketchne_general_workspace_size(C.byref(pc), n, k, ops, C.byref(out)),
                   "general_workspace_size")
        return out.value

    def sketch_general(self, L, Rt, p: SketchParams, Cm, S, H, O, ws=None):
        """Eq. (5) for f(L R) with R given transposed (Rt, n x k): returns Kt, Yt
        (h x n) and Z (l x l).  Cm, S, H, O: (rows, signs) device tensors."""
        import torch
        n, k = L.shape
        assert Rt.shape == (n, k) and L.dtype == torch.float32 and Rt.dtype == torch.float32
        assert L.is_contiguous() and Rt.is_contiguous()
        ss = [SparseSign(cols, p.z, t[0].data_ptr(), t[1].data_ptr())
              for cols, t in ((p.h, Cm), (p.h, S), (p.l, H), (p.l, O))]
        Kt = torch.empty((p.h, n), dtype=torch.float32, device="cuda")
        Yt = torch.empty((p.h, n), dtype=torch.float32, device="cuda")
        Z = torch.empty((p.l, p.l), dtype=torch.float32, device="cuda")
        nb = self.general_workspace_size(p, n, k, OP_SKETCH)
        ws = ws if ws is not None else self.workspace(nb)
        pc = p.c()
        self.check(self.lib.sketchne_sketch_general(self.ctx(), n, k, C.c_void_p(L.data_ptr()),
                                                    C.c_void_p(Rt.data_ptr()), C.byref(pc), C.byref(ss[0]),
                                                    C.byref(ss[1]), C.byref(ss[2]), C.byref(ss[3]),
                                                    C.c_void_p(Kt.data_ptr()), C.c_void_p(Yt.data_ptr()),
                                                    C.c_void_p(Z.data_ptr()), C.c_void_p(self._aligned(ws)), nb),
                   "sketch_general")
        return Kt, Yt, Z

    def embed_general(self, n: int, p: SketchParams, Kt, Yt, Z, H, O, ws=None):
        """Eqs. (6)-(10): E (column side), Ed (row side), both n x d, and sigma."""
        import torch
        E = torch.empty((n, p.d), dtype=torch.float32, device="cuda")
        Ed = torch.empty((n, p.d), dtype=torch.float32, device="cuda")
        sig = torch.empty(p.d, dtype=torch.float64, device="cuda")
        Hs = SparseSign(p.l, p.z, H[0].data_ptr(), H[1].data_ptr())
        Os = SparseSign(p.l, p.z, O[0].data_ptr(), O[1].data_ptr())
        nb = self.general_workspace_size(p, n, p.h, OP_EMBED)
        ws = ws if ws is not None else self.workspace(nb)
        pc = p.c()
        self.check(self.lib.sketchne_embed_general(self.ctx(), C.byref(pc), n, C.c_void_p(Kt.data_ptr()),
                                                   C.c_void_p(Yt.data_ptr()), C.c_void_p(Z.data_ptr()), C.byref(Hs),
                                                   C.byref(Os), C.c_void_p(E.data_ptr()), C.c_void_p(Ed.data_ptr()),
                                                   C.c_void_p(sig.data_ptr()), C.c_void_p(self._aligned(ws)), nb),
                   "embed_general")
        return E, Ed, sig

    # ---------------------------------------------------------------- full-visit variant
    def fullvisit_workspace_size(self, p: SketchParams, n: int, ops: int) -> int:
        out = C.c_size_t(0)
        pc = p.c()
        self.check(self.lib.sketchne_fullvisit_workspace_size(C.byref(pc), n, ops, C.byref(out)),
                   "fullvisit_workspace_size")
        return out.value

    def sketch_fullvisit(self, g: "DeviceGraph", p: SketchParams, U, lam, S=None, O=None, ws=None):
        """Y (transposed, h x n) and Z (l x l) with z nonzeros per row of S and O.
        S, O: (cols, signs) device tensors of shape (n, z), or None to draw on
        the device (then returned)."""
        import torch
        generate = S is None or O is None
        if generate:
            S = (torch.empty((g.n, p.z), dtype=torch.int32, device="cuda"),
                 torch.empty((g.n, p.z), dtype=torch.int8, device="cuda"))
            O = (torch.empty((g.n, p.z), dtype=torch.int32, device="cuda"),
                 torch.empty((g.n, p.z), dtype=torch.int8, device="cuda"))
        Ss = RowSign(p.h, p.z, S[0].data_ptr(), S[1].data_ptr())
        Os = RowSign(p.l, p.z, O[0].data_ptr(), O[1].data_ptr())
        Yt = torch.empty((p.h, g.n), dtype=torch.float32, device="cuda")
        Z = torch.empty((p.l, p.l), dtype=torch.float32, device="cuda")
        nb = self.fullvisit_workspace_size(p, g.n, OP_SKETCH)
        ws = ws if ws is not None else self.workspace(nb)
        pc, gs = p.c(), g.c()
        self.check(self.lib.sketchne_sketch_fullvisit(self.ctx(), C.byref(gs), C.byref(pc), C.c_void_p(U.data_ptr()),
                                                      C.c_void_p(lam.data_ptr()), C.byref(Ss), C.byref(Os),
                                                      int(generate), C.c_void_p(Yt.data_ptr()),
                                                      C.c_void_p(Z.data_ptr()), C.c_void_p(self._aligned(ws)), nb),
                   "sketch_fullvisit")
        return Yt, Z, S, O

    def embed_fullvisit(self, n: int, p: SketchParams, Yt, Z, O, ws=None):
        import torch
        E = torch.empty((n, p.d), dtype=torch.float32, device="cuda")
        sig = torch.empty(p.d, dtype=torch.float64, device="cuda")
        Os = RowSign(p.l, p.z, O[0].data_ptr(), O[1].data_ptr())
        nb = self.fullvisit_workspace_size(p, n, OP_EMBED)
        ws = ws if ws is not None else self.workspace(nb)
        pc = p.c()
        self.check(self.lib.sketchne_embed_fullvisit(self.ctx(), C.byref(pc), n, C.c_void_p(Yt.data_ptr()),
                                                     C.c_void_p(Z.data_ptr()), C.byref(Os), C.c_void_p(E.data_ptr()),
                                                     C.c_void_p(sig.data_ptr()), C.c_void_p(self._aligned(ws)), nb),
                   "embed_fullvisit")
        return E, sig

    # ---------------------------------------------------------------- steps
    def spmm(self, g: "DeviceGraph", alpha: float, B, out=None):
        import torch
        n, cols = B.shape
        out = out if out is not None else torch.empty_like(B)
        pp = SketchParams(k=1, s_eig=0, d=1, h=1, l=1, z=1)
        nb = self.workspace_size(pp, g.n, g.nnz, OP_SPMM)
        ws = self.workspace(nb)
        gs = g.c()
        self.check(self.lib.sketchne_spmm(self.ctx(), C.byref(gs), alpha, C.c_void_p(B.data_ptr()), B.stride(0),
                                          cols, C.c_void_p(out.data_ptr()), out.stride(0),
                                          C.c_void_p(self._aligned(ws)), nb), "spmm")
        return out

    def orth(self, B):
        n, cols = B.shape
        nb = C.c_size_t(0)
        self.check(self.lib.sketchne_orth_workspace_size(n, cols, C.byref(nb)), "orth_workspace_size")
        ws = self.workspace(nb.value)
        self.check(self.lib.sketchne_orth(self.ctx(), n, cols, C.c_void_p(B.data_ptr()), B.stride(0),
                                          C.c_void_p(self._aligned(ws)), nb.value), "orth")
        return B

    def symeig(self, A):
        import torch
        m = A.shape[0]
        V = torch.empty((m, m), dtype=torch.float64, device="cuda")
        w = torch.empty(m, dtype=torch.float64, device="cuda")
        nb = C.c_size_t(0)
        self.check(self.lib.sketchne_symeig_workspace_size(m, C.byref(nb)), "symeig_workspace_size")
        ws = self.workspace(nb.value)
        self.check(self.lib.sketchne_symeig(self.ctx(), m, C.c_void_p(A.data_ptr()), C.c_void_p(V.data_ptr()),
                                            C.c_void_p(w.data_ptr()), C.c_void_p(self._aligned(ws)), nb.value),
                   "symeig")
        return V, w

    def symeig_noalloc(self, A, V=None, w=None):
        """sketchne_symeig without a workspace (the library's own device scratch);
        V (m x m float64) and w (m float64) are allocated here unless given."""
        import torch
        m = A.shape[0]
        V = V if V is not None else torch.empty((m, m), dtype=torch.float64, device="cuda")
        w = w if w is not None else torch.empty(m, dtype=torch.float64, device="cuda")
        self.check(self.lib.sketchne_symeig_noalloc(self.ctx(), m, C.c_void_p(A.data_ptr()), C.c_void_p(V.data_ptr()),
                                                    C.c_void_p(w.data_ptr())), "symeig_noalloc")
        return V, w

    def propagate_coeffs(self, p: int = 10, theta: float = 0.5, mu: float = 0.2) -> np.ndarray:
        """Chebyshev coefficients c_0..c_p of the band-pass filter (host)."""
        out = (C.c_double * (p + 1))()
        self.check(self.lib.sketchne_propagate_coeffs(p, theta, mu, out), "propagate_coeffs")
        return np.array(out[:], dtype=np.float64)

    def propagate(self, g: "DeviceGraph", E, coef, out=None, ws=None):
        """Alg. 6 line 6: sum_r coef[r] T_r(L - I) E for an n x d float32 block E."""
        import torch
        assert E.dtype == torch.float32 and E.dim() == 2 and E.is_contiguous()
        n, d = E.shape
        if out is None:
            out = torch.empty_like(E)
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        nb = C.c_size_t(0)
        self.check(self.lib.sketchne_propagate_workspace_size(n, g.nnz, d, C.byref(nb)), "propagate_workspace_size")
        if ws is None or ws.numel() < nb.value + 256:
            ws = self.workspace(nb.value)
        gc = g.c()
        cp = (C.c_double * len(coef))(*coef)
        self.check(self.lib.sketchne_propagate(self.ctx(), C.byref(gc), d, C.c_void_p(E.data_ptr()), d,
                                               len(coef) - 1, cp, C.c_void_p(out.data_ptr()), out.stride(0),
                                               C.c_void_p(self._aligned(ws)), nb.value), "propagate")
        return out

    def gen_gauss(self, n: int, cols: int, seed: int):
        import torch
        out = torch.empty((n, cols), dtype=torch.float32, device="cuda")
        self.check(self.lib.sketchne_gen_gauss(self.ctx(), n, cols, seed, C.c_void_p(out.data_ptr())), "gen_gauss")
        return out

    def gen_sparse_sign(self, n: int, cols: int, z: int, seed: int):
        import torch
        rows = torch.empty((cols, z), dtype=torch.int32, device="cuda")
        signs = torch.empty((cols, z), dtype=torch.int8, device="cuda")
        s = SparseSign(cols, z, rows.data_ptr(), signs.data_ptr())
        self.check(self.lib.sketchne_gen_sparse_sign(self.ctx(), n, seed, C.byref(s)), "gen_sparse_sign")
        return rows, signs

    # ---------------------------------------------------------------- learned warm start
    def ws_param_count(self, width: int, out: int) -> int:
        c = C.c_int64(0)
        self.check(self.lib.sketchne_ws_param_count(width, out, C.byref(c)), "ws_param_count")
        return c.value

    def ws_workspace_size(self, width: int, out: int, n: int, nnz: int, ops: int, p: SketchParams = None) -> int:
        nb = C.c_size_t(0)
        pc = p.c() if p is not None else None
        self.check(self.lib.sketchne_ws_workspace_size(C.byref(pc) if pc is not None else None, width, out, n, nnz,
                                                       ops, C.byref(nb)), "ws_workspace_size")
        return nb.value

    def ws_init(self, net: "MLP", seed: int):
        s = net.c()
        self.check(self.lib.sketchne_ws_init(self.ctx(), C.byref(s), seed), "ws_init")

    def ws_features(self, g: "DeviceGraph", alpha: float, probe=None, seed: int = 0, ws=None):
        """phi (n x 8 float32); probe: n x 4 float32 (+-1, row-major) or None to
        draw it from seed."""
        import torch
        phi = torch.empty((g.n, WS_FEAT), dtype=torch.float32, device="cuda")
        nb = self.ws_workspace_size(1, 1, g.n, g.nnz, WS_OP_FEATURES)
        ws = ws if ws is not None else self.workspace(nb)
        gs = g.c()
        self.check(self.lib.sketchne_ws_features(self.ctx(), C.byref(gs), alpha, C.c_void_p(_ptr(probe)), seed,
                                                 C.c_void_p(phi.data_ptr()), C.c_void_p(self._aligned(ws)), nb),
                   "ws_features")
        return phi

    def ws_forward(self, net: "MLP", phi, out=None):
        import torch
        n = phi.shape[0]
        F = out if out is not None else torch.empty((n, net.out), dtype=torch.float32, device="cuda")
        nb = self.ws_workspace_size(net.width, net.out, n, 0, WS_OP_FORWARD)
        ws = self.workspace(nb)
        s = net.c()
        self.check(self.lib.sketchne_ws_forward(self.ctx(), C.byref(s), n, C.c_void_p(phi.data_ptr()),
                                                C.c_void_p(F.data_ptr()), F.stride(0),
                                                C.c_void_p(self._aligned(ws)), nb), "ws_forward")
        return F

    def ws_infer(self, net: "MLP", phi, out=None):
        """The BF16-activation inference pass of sketchne_eig_learned."""
        import torch
        n = phi.shape[0]
        F = out if out is not None else torch.empty((n, net.out), dtype=torch.float32, device="cuda")
        nb = self.ws_workspace_size(net.width, net.out, n, 0, WS_OP_FORWARD)
        ws = self.workspace(nb)
        s = net.c()
        self.check(self.lib.sketchne_ws_infer(self.ctx(), C.byref(s), n, C.c_void_p(phi.data_ptr()),
                                              C.c_void_p(F.data_ptr()), F.stride(0),
                                              C.c_void_p(self._aligned(ws)), nb), "ws_infer")
        return F

    def ws_grad(self, net: "MLP", phi, U, mu: float, grad=None, loss=None, ws=None):
        import torch
        n = phi.shape[0]
        grad = grad if grad is not None else torch.empty(net.count, dtype=torch.float32, device="cuda")
        loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device="cuda")
        nb = self.ws_workspace_size(net.width, net.out, n, 0, WS_OP_GRAD)
        ws = ws if ws is not None else self.workspace(nb)
        s = net.c()
        self.check(self.lib.sketchne_ws_grad(self.ctx(), C.byref(s), n, C.c_void_p(phi.data_ptr()),
                                             C.c_void_p(U.data_ptr()), U.stride(0), mu, C.c_void_p(grad.data_ptr()),
                                             C.c_void_p(loss.data_ptr()), C.c_void_p(self._aligned(ws)), nb),
                   "ws_grad")
        return grad, loss

    def ws_adam(self, net: "MLP", grad, lr: float, step: int):
        s = net.c()
        self.check(self.lib.sketchne_ws_adam(self.ctx(), C.byref(s), C.c_void_p(grad.data_ptr()), lr, step),
                   "ws_adam")

    def ws_train(self, net: "MLP", sets, steps: int, lr: float, mu: float, step0: int = 0):
        """Adam training on [(phi, U), ...] round-robin; returns the per-step losses."""
        import torch
        ns = len(sets)
        phis = (C.c_void_p * ns)(*[C.c_void_p(ph.data_ptr()) for ph, _ in sets])
        Us = (C.c_void_p * ns)(*[C.c_void_p(u.data_ptr()) for _, u in sets])
        nn = (C.c_int64 * ns)(*[ph.shape[0] for ph, _ in sets])
        for ph, u in sets:
            assert u.shape == (ph.shape[0], net.out) and u.is_contiguous() and ph.is_contiguous()
        nmax = max(ph.shape[0] for ph, _ in sets)
        nb = self.ws_workspace_size(net.width, net.out, nmax, 0, WS_OP_GRAD) + 4 * net.count + 512
        ws = self.workspace(nb)
        losses = torch.empty(max(steps, 1), dtype=torch.float32, device="cuda")
        s = net.c()
        self.check(self.lib.sketchne_ws_train(self.ctx(), C.byref(s), ns, phis, Us, nn, steps, step0, lr, mu,
                                              C.c_void_p(losses.data_ptr()), C.c_void_p(self._aligned(ws)), nb),
                   "ws_train")
        return losses[:steps]

    def ritz_residual(self, g: "DeviceGraph", alpha: float, U, lam):
        import torch
        k = U.shape[1]
        res = torch.empty(k, dtype=torch.float64, device="cuda")
        nb = self.ws_workspace_size(1, 1, g.n, g.nnz, WS_OP_RESIDUAL, SketchParams(k=k, s_eig=0, d=1, h=1, l=1, z=1))
        ws = self.workspace(nb)
        gs = g.c()
        self.check(self.lib.sketchne_ritz_residual(self.ctx(), C.byref(gs), alpha, k, C.c_void_p(U.data_ptr()),
                                                   C.c_void_p(lam.data_ptr()), C.c_void_p(res.data_ptr()),
                                                   C.c_void_p(self._aligned(ws)), nb), "ritz_residual")
        return res

    def eig_learned(self, g: "DeviceGraph", p: SketchParams, net: "MLP", q_warm: int, threshold: float, ws=None,
                    with_residual: bool = False):
        """Alg. 5 from the learned start; returns U, lambda, used_fallback
        (and the largest Ritz residual of the warm run with with_residual)."""
        import torch
        U = torch.empty((g.n, p.k), dtype=torch.float32, device="cuda")
        lam = torch.empty(p.k, dtype=torch.float64, device="cuda")
        nb = self.ws_workspace_size(net.width, net.out, g.n, g.nnz, WS_OP_EIG, p)
        ws = ws if ws is not None else self.workspace(nb)
        fb = C.c_int32(0)
        worst = C.c_double(0.0)
        pc = p.c()
        gs = g.c()
        s = net.c()
        self.check(self.lib.sketchne_eig_learned(self.ctx(), C.byref(gs), C.byref(pc), C.byref(s), q_warm, threshold,
                                                 C.c_void_p(U.data_ptr()), C.c_void_p(lam.data_ptr()), C.byref(fb),
                                                 C.byref(worst), C.c_void_p(self._aligned(ws)), nb), "eig_learned")
        if with_residual:
            return U, lam, bool(fb.value), worst.value
        return U, lam, bool(fb.value)

    def profile_enable(self, on: bool, classes=None):
        """Time every kernel class (or, with `classes`, only those named in
        PROF_NAMES; the rest then run without events)."""
        v = int(on)
        if on and classes is not None:
            v = PROF_SELECT
            for name in classes:
                v |= 1 << PROF_NAMES.index(name)
        self.check(self.lib.sketchne_profile_enable(self.ctx(), v), "profile_enable")

    def profile_read(self) -> dict:
        ms = (C.c_double * len(PROF_NAMES))()
        n = (C.c_int64 * len(PROF_NAMES))()
        self.check(self.lib.sketchne_profile_read(self.ctx(), ms, n), "profile_read")
        return {PROF_NAMES[i]: (ms[i], n[i]) for i in range(len(PROF_NAMES))}


class DeviceGraph:
    """CSR arrays resident on cuda:0 (rowptr int64, colidx int32)."""

    def __init__(self, rowptr: np.ndarray, colidx: np.ndarray):
        import torch
        self.n = len(rowptr) - 1
        self.nnz = int(rowptr[-1])
        self.rowptr = torch.from_numpy(np.ascontiguousarray(rowptr, dtype=np.int64)).cuda()
        cols = np.ascontiguousarray(colidx, dtype=np.int32)
        self.colidx = torch.from_numpy(cols if len(cols) else np.zeros(1, np.int32)).cuda()

    @classmethod
    def from_device(cls, rowptr, colidx) -> "DeviceGraph":
        """Wrap CSR arrays already on cuda:0 (rowptr int64, colidx int32)."""
        import torch
        assert rowptr.dtype == torch.int64 and colidx.dtype == torch.int32 and rowptr.is_cuda and colidx.is_cuda
        g = cls.__new__(cls)
        g.n = rowptr.numel() - 1
        g.nnz = int(rowptr[-1])
        g.rowptr = rowptr.contiguous()
        g.colidx = colidx.contiguous() if colidx.numel() else torch.zeros(1, dtype=torch.int32, device="cuda")
        return g

    def c(self) -> Graph:
        return Graph(self.n, self.nnz, self.rowptr.data_ptr(), self.colidx.data_ptr())


class MLP:
    """Device buffers of the warm-start network (FP32 master, BF16 copy, Adam moments)."""

    def __init__(self, lib: Library, width: int, out: int, train: bool = True):
        import torch
        self.width, self.out = width, out
        self.count = lib.ws_param_count(width, out)
        self.master = torch.zeros(self.count, dtype=torch.float32, device="cuda")
        self.bf16 = torch.zeros(self.count, dtype=torch.int16, device="cuda")
        self.m = torch.zeros(self.count, dtype=torch.float32, device="cuda") if train else None
        self.v = torch.zeros(self.count, dtype=torch.float32, device="cuda") if train else None

    def c(self) -> MLPStruct:
        return MLPStruct(self.width, self.out, self.master.data_ptr(), self.bf16.data_ptr(), _ptr(self.m),
                         _ptr(self.v))

    def bf16_values(self):
        """The BF16 copy as float64 numpy (what the forward pass reads)."""
        b = self.bf16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        return b.view(np.float32).astype(np.float64)
