"""Learned warm start on the GPU against the FP64 oracle (oracle/mlp.py):
features, forward pass, loss gradient, Adam, and what the trained network
gains over the Gaussian start (with the fallback)."""
import numpy as np
import pytest

import synth
from oracle import mlp as om
from tests.util import rel, say

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _graph_with_isolated():
    rowptr, colidx = synth.chung_lu(5000, 2.2, 8, 1, 4040)
    rowptr = np.concatenate([rowptr, [rowptr[-1]] * 3])  # n = 5003, last three isolated
    return rowptr, colidx


def test_features_parity(lib):
    torch = _torch()
    from paper_2110_12782_amd.binding import DeviceGraph
    for rowptr, colidx in (synth.sbm([512] * 8, 0.02, 0.001, 1001), _graph_with_isolated()):
        n = len(rowptr) - 1
        g = synth.rademacher(n * om.N_PROBE, 21).reshape(n, om.N_PROBE)
        G = DeviceGraph(rowptr, colidx)
        phi = lib.ws_features(G, 0.5, probe=torch.from_numpy(np.ascontiguousarray(g)).cuda()).cpu().numpy()
        ref = om.features(rowptr, colidx, 0.5, g.astype(np.float64))
        e = rel(phi, ref)
        say(f"n={n} features rel {e:.3e}")
        assert e <= 1e-5
        assert np.all(phi[:, om.N_RAW:] == 0)


def _net_and_inputs(lib, n, width, out, seed):
    torch = _torch()
    from paper_2110_12782_amd.binding import MLP
    net = MLP(lib, width, out)
    lib.ws_init(net, seed)
    rng = np.random.default_rng(seed)
    phi = np.zeros((n, om.FEAT), np.float32)
    phi[:, :om.N_RAW] = rng.standard_normal((n, om.N_RAW))
    U = np.linalg.qr(rng.standard_normal((n, out)))[0].astype(np.float32)
    return net, phi, U, torch.from_numpy(phi).cuda(), torch.from_numpy(U).cuda()


def test_init_distribution(lib):
    torch = _torch()
    from paper_2110_12782_amd.binding import MLP
    net = MLP(lib, 256, 64)
    lib.ws_init(net, 9)
    p = om.unflatten(net.master.cpu().numpy(), 256, 64)
    assert np.all(p["W1"][om.N_RAW:] == 0) and np.all(p["b1"] == 0) and np.all(p["b3"] == 0)
    assert abs(p["W2"].std() - np.sqrt(2 / 256)) < 0.01 * np.sqrt(2 / 256) * 10
    assert abs(p["W1"][:om.N_RAW].std() - np.sqrt(2 / om.N_RAW)) < 0.1 * np.sqrt(2 / om.N_RAW)
    # the BF16 copy is the round-to-nearest-even of the master
    assert np.array_equal(net.bf16_values(), om.bf16_round(net.master.cpu().numpy()))
    assert torch.all(net.m == 0) and torch.all(net.v == 0)


@pytest.mark.parametrize("n,width,out", [(1000, 256, 64), (4099, 256, 256), (70, 64, 12)])
def test_forward_and_gradient_parity(lib, n, width, out):
    net, phi, U, phi_d, U_d = _net_and_inputs(lib, n, width, out, 100 + n)
    theta = net.bf16_values()
    p = om.unflatten(theta, width, out)
    F = lib.ws_forward(net, phi_d).cpu().numpy()
    _, _, Fr = om.forward(p, phi.astype(np.float64))
    ef = rel(F, Fr)
    mu = 0.1
    grad, loss = lib.ws_grad(net, phi_d, U_d, mu)
    L, gref = om.grad(theta, phi.astype(np.float64), U.astype(np.float64), mu, width, out)
    gg = grad.cpu().numpy()
    el = abs(float(loss.cpu()) - L) / abs(L)
    eg = rel(gg, gref)
    blocks = {}
    off = 0
    for name, shp in om.param_shapes(width, out):
        size = int(np.prod(shp))
        if np.linalg.norm(gref[off:off + size]) > 0:
            blocks[name] = rel(gg[off:off + size], gref[off:off + size])
        off += size
    say(f"n={n} width={width} out={out}: F rel {ef:.2e}  loss rel {el:.2e}  grad rel {eg:.2e}  "
        + " ".join(f"{k} {v:.1e}" for k, v in blocks.items()))
    assert ef <= 1e-5
    assert el <= 1e-5
    assert eg <= 1e-5 and max(blocks.values()) <= 1e-4


@pytest.mark.parametrize("n,out", [(1000, 256), (4099, 64), (70, 32)])
def test_bf16_inference_parity(lib, n, out):
    """The inference pass (BF16 hidden activations on the BF16 matrix cores)
    against the oracle's BF16-inference semantics on the same BF16 weights, and
    against the exact forward pass within the activation-rounding bound."""
    net, phi, U, phi_d, U_d = _net_and_inputs(lib, n, 256, out, 300 + n)
    p = om.unflatten(net.bf16_values(), 256, out)
    F = lib.ws_infer(net, phi_d).cpu().numpy().astype(np.float64)
    ref = om.forward_bf16(p, phi.astype(np.float64))
    _, _, exact = om.forward(p, phi.astype(np.float64))
    e_inf, e_exact = rel(F, ref), rel(F, exact)
    say(f"n={n} out={out}: BF16 inference vs oracle BF16 semantics {e_inf:.2e}, vs exact forward {e_exact:.2e}")
    # FP32 sums against FP64 sums can move an activation across a BF16
    # rounding boundary (one BF16 unit, 2^-8 relative) in a few entries
    assert e_inf <= 1e-3
    assert e_exact <= 2e-2


def test_adam_parity_and_bf16_copy(lib):
    net, phi, U, phi_d, U_d = _net_and_inputs(lib, 777, 128, 32, 5)

    def state():
        return (net.master.cpu().numpy().astype(np.float64), net.m.cpu().numpy().astype(np.float64),
                net.v.cpu().numpy().astype(np.float64))

    for step in (1, 2):
        grad, _ = lib.ws_grad(net, phi_d, U_d, 0.1)
        w0, m0, v0 = state()
        ref_w, ref_m, ref_v = om.adam(w0, grad.cpu().numpy().astype(np.float64), m0, v0, step, 1e-3)
        lib.ws_adam(net, grad, 1e-3, step)
        w1, m1, v1 = state()
        eu = rel(w1 - w0, ref_w - w0)
        em = rel(m1, ref_m) + rel(v1, ref_v)
        say(f"adam step {step}: update rel {eu:.2e}, moments rel {em:.2e}")
        assert eu <= 1e-5 and em <= 1e-5 and rel(w1, ref_w) <= 1e-6
        # the BF16 copy is exactly the round-to-nearest-even of the new master
        assert np.array_equal(net.bf16_values(), om.bf16_round(w1))


def _sin_theta(U, V):
    torch = _torch()
    a = U.double()
    b = V.double()
    k = a.shape[1]
    s = torch.linalg.matrix_norm(b.T @ a) ** 2
    return float(torch.sqrt(torch.clamp(k - s, min=0.0) / k))


def test_training_gain_and_fallback(lib):
    """The warm-start protocol at test scale: train on eight SBM and Chung-Lu
    graphs (n = 2^13 and 2^14, exponent 2.0-2.5, mean degree 8-32) against
    their own converged eigenvectors, evaluate on four held-out graphs (two
    SBM, two Chung-Lu, n = 2^14): subspace error of U_k against a q = 24
    reference for the Gaussian and learned starts at q = 0..3.  The learned
    start is never worse at equal q, and on the Chung-Lu graphs it saves a
    power iteration (learned at q - 1 at or below plain at q, q = 2, 3; on
    the SBM graphs it gains less than one iteration, which is reported).
    Then the decision residual equals the SpMM form and the fallback
    reproduces the plain result exactly."""
    import torch
    from paper_2110_12782_amd.binding import DeviceGraph, MLP, SketchParams
    k, s_eig, width = 64, 32, 256
    rng = np.random.default_rng(0)

    def P(q, seed):
        return SketchParams(k=k, s_eig=s_eig, q=q, d=16, h=48, l=128, z=8, seed=seed)

    def graph(i, lg, seed):
        n = 1 << lg
        deg = float(np.exp(rng.uniform(np.log(8), np.log(32))))
        if i % 2 == 0:
            bs = n // 16
            return synth.sbm([bs] * 16, deg * 0.8 / bs, deg * 0.2 / (n - bs), seed)
        return synth.chung_lu(n, float(rng.uniform(2.0, 2.5)), deg, 2, seed)

    sets, calib = [], []
    for i, lg in enumerate((13, 13, 14, 14, 13, 14, 13, 14)):
        rowptr, colidx = graph(i, lg, 10000 + i)
        G = DeviceGraph(rowptr, colidx)
        Uref, _ = lib.eig(G, P(16, 100 + i))
        sets.append((lib.ws_features(G, 0.5, seed=200 + i), Uref.contiguous()))
        U2, l2 = lib.eig(G, P(2, 300 + i))
        calib.append(float(lib.ritz_residual(G, 0.5, U2, l2).max()))
    assert lib.sync() & ~1 == 0
    net = MLP(lib, width, k)
    lib.ws_init(net, 11)
    losses = lib.ws_train(net, sets, 600, 1e-3, 0.1).cpu().numpy()
    first, last = losses[:16].mean(), losses[-16:].mean()
    say(f"training loss {first:.4f} -> {last:.4f}")
    assert np.all(np.isfinite(losses))
    assert last < 0.5 * first
    threshold = 1.1 * max(calib)
    for j in range(4):
        rowptr, colidx = graph(j, 14, 20000 + j)
        G = DeviceGraph(rowptr, colidx)
        Uref, _ = lib.eig(G, P(24, 999))
        plain, learned = [], []
        for q in (0, 1, 2, 3):
            Up, lp = lib.eig(G, P(q, 11))
            Uw, lw, fb, worst = lib.eig_learned(G, P(q, 11), net, q, threshold, with_residual=True)
            # the decision residual (from the Rayleigh-Ritz Gram) equals the
            # largest ||X u_j - lambda_j u_j|| formed with a further SpMM
            direct = float(lib.ritz_residual(G, 0.5, Uw, lw).max())
            assert abs(worst - direct) <= 1e-4 * direct + 1e-6
            assert not fb or q == 0
            plain.append(_sin_theta(Up, Uref))
            learned.append(_sin_theta(Uw, Uref))
        kind = "sbm" if j % 2 == 0 else "chung-lu"
        say(f"held-out {kind}: plain " + " ".join(f"{x:.4f}" for x in plain) + "  learned " +
            " ".join(f"{x:.4f}" for x in learned))
        assert all(l_ <= p_ for l_, p_ in zip(learned, plain))
        if kind == "chung-lu":
            assert learned[1] <= plain[2] and learned[2] <= plain[3]
        # fallback: a zero threshold always rejects, and the plain start with p.q runs
        Uf, lf, fb = lib.eig_learned(G, P(2, 11), net, 0, 0.0)
        Up2, lp2 = lib.eig(G, P(2, 11))
        assert fb
        assert torch.equal(Uf, Up2) and torch.equal(lf, lp2)
    assert lib.sync() & ~1 == 0
