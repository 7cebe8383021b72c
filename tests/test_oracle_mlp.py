"""Pins of the warm-start oracle (oracle/mlp.py): closed forms, invariances and
central finite differences.  CPU only."""
import numpy as np
import pytest

import synth
from oracle import mlp


def _orthonormal(n, k, seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, k)))
    return q


def _small_problem(seed=0, n=96, width=16, out=8):
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((n, mlp.FEAT))
    phi[:, mlp.N_RAW:] = 0.0
    theta = np.concatenate([
        rng.standard_normal(mlp.FEAT * width) * np.sqrt(2 / mlp.FEAT), rng.standard_normal(width) * 0.1,
        rng.standard_normal(width * width) * np.sqrt(2 / width), rng.standard_normal(width) * 0.1,
        rng.standard_normal(width * out) * np.sqrt(2 / width), rng.standard_normal(out) * 0.1])
    U = _orthonormal(n, out, seed + 1)
    return phi, theta, U, width, out


@pytest.mark.parametrize("mu", [0.0, 0.1, 1.0])
def test_gradient_matches_central_differences(mu):
    phi, theta, U, width, out = _small_problem()
    L, gvec = mlp.grad(theta, phi, U, mu, width, out)
    rng = np.random.default_rng(3)
    idx = rng.choice(theta.size, size=60, replace=False)
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.grad(tp, phi, U, mu, width, out)[0] - mlp.grad(tm, phi, U, mu, width, out)[0]) / (2 * h)
        assert abs(fd - gvec[i]) <= 1e-6 * max(1.0, np.abs(gvec).max()), (i, fd, gvec[i])


def test_loss_grad_matches_central_differences_in_F():
    rng = np.random.default_rng(4)
    n, k = 40, 6
    F = rng.standard_normal((n, k))
    U = _orthonormal(n, k, 5)
    G = mlp.loss_grad(F, U, 0.3)
    h = 1e-6
    for (i, j) in [(0, 0), (3, 2), (39, 5), (17, 1)]:
        Fp = F.copy(); Fp[i, j] += h
        Fm = F.copy(); Fm[i, j] -= h
        fd = (mlp.loss(Fp, U, 0.3) - mlp.loss(Fm, U, 0.3)) / (2 * h)
        assert abs(fd - G[i, j]) < 1e-7


def test_loss_closed_forms():
    n, k = 50, 5
    U = _orthonormal(n, k, 6)
    # an orthogonal basis of span(U) with equal column norms: both terms vanish
    Qr = _orthonormal(k, k, 7)
    assert mlp.loss(3.7 * U @ Qr, U, 1.0) < 1e-24
    # scale invariance
    F = np.random.default_rng(8).standard_normal((n, k))
    assert abs(mlp.loss(F, U, 0.5) - mlp.loss(-0.01 * F, U, 0.5)) < 1e-12
    # F orthogonal to span(U): the subspace term is exactly 1
    W = _orthonormal(n, 2 * k, 9)
    P = W[:, k:] - U @ (U.T @ W[:, k:])
    assert abs(mlp.loss(P, U, 0.0) - 1.0) < 1e-12
    # half of each column in span(U): subspace term = 1/2
    V = (np.eye(n) - U @ U.T) @ np.random.default_rng(10).standard_normal((n, k))
    V /= np.linalg.norm(V, axis=0)
    F = U + V
    assert abs(mlp.loss(F, U, 0.0) - 0.5) < 1e-12


def test_adam_first_step_closed_form():
    g = np.array([3.0, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # bias-corrected moments of the first step are g and g^2
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_on_cycle_closed_form():
    n = 64
    rowptr, colidx = synth.cycle(n)
    g = synth.rademacher(n * mlp.N_PROBE, 11).astype(np.float64).reshape(n, mlp.N_PROBE)
    phi = mlp.features(rowptr, colidx, 0.5, g)
    # 2-regular: X = A / 2, so X v is the average of the two ring neighbours
    v = g.copy()
    powers = []
    for t in range(4):
        v = 0.5 * (np.roll(v, 1, axis=0) + np.roll(v, -1, axis=0))
        powers.append(v)
    # columns 1-4: X^3 g (all probes); columns 5-7: X^4 g (first three)
    expect_raw = np.concatenate([powers[2], powers[3][:, :3]], axis=1)
    for j in range(expect_raw.shape[1]):
        c = expect_raw[:, j]
        assert np.allclose(phi[:, 1 + j], (c - c.mean()) / c.std(), atol=1e-12)
    # constant degree: the log-degree column has no spread and is set to 0
    assert np.all(phi[:, 0] == 0.0)
    assert mlp.N_RAW == 1 + mlp.N_PROBE + 3 == mlp.FEAT


def test_features_standardised_and_isolated_vertices():
    rowptr, colidx = synth.chung_lu(3000, 2.3, 6, 1, 77)
    # append three isolated vertices
    rowptr = np.concatenate([rowptr, [rowptr[-1]] * 3])
    n = len(rowptr) - 1
    g = synth.rademacher(n * mlp.N_PROBE, 12).astype(np.float64).reshape(n, mlp.N_PROBE)
    phi = mlp.features(rowptr, colidx, 0.5, g)
    assert np.allclose(phi[:, :mlp.N_RAW].mean(axis=0), 0, atol=1e-12)
    assert np.allclose(phi[:, :mlp.N_RAW].std(axis=0), 1, atol=1e-12)
    # isolated vertices: every raw feature is 0 (log max(0, 1) = 0, no neighbours), so their rows coincide
    assert np.allclose(phi[-1], phi[-2]) and np.allclose(phi[-1], phi[-3])


def test_bf16_round_ties_to_even():
    one = 1.0
    vals = np.array([one, one + 2 ** -8, one + 3 * 2 ** -8, one + 2 ** -7, -2.5, 1e-40])
    r = mlp.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6 and r[3] == 1.0 + 2 ** -7
    assert r[4] == -2.5
    assert abs(mlp.bf16_round(np.pi) - np.pi) <= 2 ** -8 * np.pi


def test_bf16_inference_exact_on_representable_activations():
    # small integer weights and inputs: every pre-activation is an integer of
    # magnitude < 256, exactly representable in bfloat16, so the BF16 inference
    # pass must equal the exact forward pass bit for bit
    rng = np.random.default_rng(7)
    width, out, n = 16, 8, 40
    p = {"W1": rng.integers(-1, 2, (mlp.FEAT, width)).astype(float), "b1": rng.integers(-2, 3, width).astype(float),
         "W2": rng.integers(-1, 2, (width, width)).astype(float), "b2": rng.integers(-2, 3, width).astype(float),
         "W3": rng.integers(-1, 2, (width, out)).astype(float) * 0.5, "b3": rng.integers(-2, 3, out).astype(float)}
    phi = rng.integers(-2, 3, (n, mlp.FEAT)).astype(float)
    _, H2, F = mlp.forward(p, phi)
    assert np.abs(H2).max() < 256
    assert np.array_equal(mlp.forward_bf16(p, phi), F)


def test_bf16_inference_within_rounding_bound():
    # each hidden activation is rounded with relative error <= 2^-9, so F moves
    # by at most the rounding of H1 propagated through |W2|, |W3| plus that of H2
    phi, theta, U, width, out = _small_problem(seed=3)
    p = mlp.unflatten(theta, width, out)
    H1, H2, F = mlp.forward(p, phi)
    Fb = mlp.forward_bf16(p, phi)
    u = 2.0 ** -9
    bound = (u * H1) @ np.abs(p["W2"]) @ np.abs(p["W3"]) + u * (H2 + (u * H1) @ np.abs(p["W2"])) @ np.abs(p["W3"])
    assert np.all(np.abs(Fb - F) <= bound + 1e-12)
    assert np.abs(Fb - F).max() > 0  # the rounding is not vacuous here


def test_adam_two_steps_constant_gradient_closed_form():
    # with the same gradient g at steps 1 and 2 the bias-corrected moments are
    # exactly g and g^2 at both steps (m2 = 0.19 g, 1 - 0.9^2 = 0.19;
    # v2 = 0.001999 g^2, 1 - 0.999^2 = 0.001999), so each step moves every
    # parameter by -lr g / (|g| + eps)
    g = np.array([3.0, -2.0, 0.5, -1e-3])
    lr = 0.01
    th, m, v = mlp.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=lr)
    th, m, v = mlp.adam(th, g, m, v, 2, lr=lr)
    step = lr * g / (np.abs(g) + 1e-8)
    assert np.allclose(th, -2 * step, rtol=1e-12, atol=0)
    assert np.allclose(m, 0.19 * g, rtol=1e-14) and np.allclose(v, 0.001999 * g * g, rtol=1e-12)
