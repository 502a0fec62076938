"""Pins of the FP64 warm-start network oracle (oracle/cnn.py)."""
import math

import numpy as np
import pytest

from oracle import cnn


def test_conv3d_matches_direct_definition():
    rng = np.random.default_rng(1)
    C, O, Z, Y, X = 2, 3, 4, 5, 3
    x = rng.normal(size=(C, Z, Y, X))
    W = rng.normal(size=(O, C, 27))
    b = rng.normal(size=O)
    y = cnn.conv3d(x, W, b)
    ref = np.zeros_like(y)
    for o in range(O):
        for z in range(Z):
            for yy in range(Y):
                for xx in range(X):
                    acc = b[o]
                    for c in range(C):
                        for dz in (-1, 0, 1):
                            for dy in (-1, 0, 1):
                                for dx in (-1, 0, 1):
                                    t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                                    acc += W[o, c, t] * x[c, (z + dz) % Z, (yy + dy) % Y, (xx + dx) % X]
                    ref[o, z, yy, xx] = acc
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_conv3d_is_translation_equivariant():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, 6, 5, 4))
    W = rng.normal(size=(2, 3, 27))
    b = np.zeros(2)
    s = (1, -2, 3)
    np.testing.assert_allclose(cnn.conv3d(cnn.shift(x, s), W, b), cnn.shift(cnn.conv3d(x, W, b), s), atol=1e-12)


def test_bf16_round_matches_torch():
    import torch
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=1000) * 10 ** rng.uniform(-6, 3, size=1000),
                        [0.0, 1.0, -1.0, 1.00390625, 1.01171875, 3.0e-39]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16_round(x), ref)


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    L = 6
    params = cnn.init_params(7, channels=(12, 4, 4, 4, 5))
    params = [(W, rng.normal(size=b.shape) * 0.1) for W, b in params]
    x = rng.normal(size=(12, L, L, L))
    qh = rng.normal(size=(5, L, L, L)) * 0.2
    qt = rng.normal(size=(5, L, L, L)) * 0.2
    fluid = rng.uniform(size=(L, L, L)) > 0.2

    def loss_of(ps):
        out, _ = cnn.forward(ps, x)
        return cnn.loss_and_grad(out, qh, qt, fluid, 0.5)[0]

    out, cache = cnn.forward(params, x)
    _, g = cnn.loss_and_grad(out, qh, qt, fluid, 0.5)
    grads = cnn.backward(params, cache, g)
    eps = 1e-6
    for l in range(4):
        for which in (0, 1):
            arr = params[l][which]
            for _ in range(3):
                idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
                plus = [(W.copy(), b.copy()) for W, b in params]
                minus = [(W.copy(), b.copy()) for W, b in params]
                plus[l][which][idx] += eps
                minus[l][which][idx] -= eps
                num = (loss_of(plus) - loss_of(minus)) / (2 * eps)
                ana = grads[l][which][idx]
                assert num == pytest.approx(ana, rel=1e-6, abs=1e-10), (l, which, idx)


def test_adam_first_step_is_lr_times_sign():
    rng = np.random.default_rng(5)
    params = cnn.init_params(1, channels=(12, 4, 4, 4, 5))
    grads = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in params]
    new, state = cnn.adam_step(params, grads, cnn.adam_init(params), lr=1e-3)
    for (W, b), (W1, b1), (gW, gb) in zip(params, new, grads):
        # first step: m_hat = g, v_hat = g^2, so the step is lr g / (|g| + eps)
        np.testing.assert_allclose(W - W1, 1e-3 * gW / (np.abs(gW) + 1e-8), rtol=1e-9)
    assert state[0] == 1


def test_features():
    L, a, p = 16, 4.0, 32.0
    qh = np.zeros((5, L, L, L))
    f = cnn.features(L, (8.0, 8.0, 8.0), a, p, -1.0, qh)
    assert f[0, 8, 8, 8] == pytest.approx(max(-1.0, -a / 8))
    n = np.sqrt(f[1] ** 2 + f[2] ** 2 + f[3] ** 2)
    n[8, 8, 8] = 1.0
    np.testing.assert_allclose(n, 1.0, atol=1e-12)
    assert np.all(f[9] == a / 16) and np.all(f[10] == 32 / p) and np.all(f[11] == -1.0)
    assert f[0].max() <= 2.0 and f[0].min() >= -1.0
