"""Shared helpers for the GPU tests: build device inputs from synth draws and
compute the oracle's reference on the same realizations."""
import sys

import numpy as np

import synth
from oracle import netmf, freigs as fr, sketch as sk, metrics


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def c1_graph():
    # SBM: 8 equal blocks of 512, p_in = 0.02, p_out = 0.001
    return synth.sbm([512] * 8, 0.02, 0.001, 1001)


def c2_graph():
    # Chung-Lu: n = 65536, exponent 2.1, mean degree 16, min degree 2
    return synth.chung_lu(65536, 2.1, 16, 2, 1002)


def oracle_factors(A, U32, lam, alpha, T, b):
    """Eq. 11 factors computed in FP64 from the FP32-rounded U handed to the GPU."""
    U = np.asarray(U32, dtype=np.float64)
    return netmf.eq11_factors(U, np.asarray(lam, np.float64), netmf.degrees(A), netmf.volume(A), alpha, T, b)


def oracle_eig_inputs(A, k, K, q, alpha, seed):
    X = netmf.modified_laplacian(A, alpha)
    Om = synth.gaussian_block(A.shape[0], K, seed)
    U, lam = fr.freigs(X, Om.astype(np.float64), k, q)
    return U.astype(np.float32), lam, Om


def rel(x, ref):
    return metrics.rel_fro(x, ref)


__all__ = ["say", "c1_graph", "c2_graph", "oracle_factors", "oracle_eig_inputs", "rel", "sk", "netmf", "fr",
           "metrics", "synth"]
