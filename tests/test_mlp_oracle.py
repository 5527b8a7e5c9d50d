"""Pins of the MLP oracle (CPU): finite-difference gradients, bfloat16 rounding against
an independent implementation, and closed-form features/targets."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp


def test_fp64_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    params = mlp.init_params(3)
    x = rng.normal(size=(16, 8))
    y = rng.normal(size=(16, 2))
    _, grads = mlp.loss_and_grads(params, x, y, "f64")
    h = 1e-6
    for pi, p in enumerate(params):
        flat = p.ravel()
        for q in rng.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[q]
            flat[q] = old + h
            lp, _ = mlp.loss_and_grads(params, x, y, "f64")
            flat[q] = old - h
            lm, _ = mlp.loss_and_grads(params, x, y, "f64")
            flat[q] = old
            fd = (lp - lm) / (2 * h)
            g = grads[pi].ravel()[q]
            assert g == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=5000).astype(np.float32) * 10 ** rng.uniform(-30, 30, 5000).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.4e38], np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = mlp.bf16(x)
    assert np.array_equal(got, want)


def test_features_and_targets_closed_form_at_rest():
    gam = 4.0 / 3.0
    n = 3
    gcov = np.zeros((4, 4, n))
    gcon = np.zeros((4, 4, n))
    for a, s in enumerate([-1.0, 1.0, 1.0, 1.0]):
        gcov[a, a] = s
        gcon[a, a] = s
    rho = np.array([1.0, 0.1, 7.0])
    u = np.array([0.5, 2.0, 0.01])
    U = np.zeros((9, n))
    U[0] = rho
    U[1] = -u            # T^t_t + rho u^t = -(rho + u) + rho at rest, no field
    f = mlp.features(U, gcov, gcon, np.ones(n), np.ones(n), gam)
    assert np.allclose(f[0], np.log(rho))
    assert np.allclose(f[1], np.arcsinh(u / rho))
    assert np.all(f[2:5] == 0.0)
    assert np.all(f[5] == 1.0) and np.all(f[6] == gam) and np.all(f[7] == 1.0)
    P = np.vstack([rho, u, [0.6, 0.0, 0.0], [0.0, 0.8, 0.0], [0.0, 0.0, 0.0]])
    t = mlp.targets(P, gcov, gam)
    G = np.sqrt(1 + np.array([0.36, 0.64, 0.0]))
    assert np.allclose(t[0], np.log(G))
    assert np.allclose(t[1], np.log((rho + gam * u) * G / rho))


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(256, 8))
    y = np.stack([np.tanh(x[:, 0] - 0.5 * x[:, 3]), x[:, 1] * x[:, 2] * 0.3], axis=1)
    params = mlp.init_params(5)
    state = (0, [np.zeros_like(p) for p in params], [np.zeros_like(p) for p in params])
    l0, _ = mlp.loss_and_grads(params, x, y)
    for _ in range(300):
        _, g = mlp.loss_and_grads(params, x, y)
        state = mlp.adam_step(params, g, state, 3e-3)
    l1, _ = mlp.loss_and_grads(params, x, y)
    assert l1 < 0.1 * l0
