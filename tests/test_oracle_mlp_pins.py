"""Pins of the closure network's FP64 reference (CPU)."""
import math

import numpy as np
import pytest

import fixtures
from oracle import mlp


def test_parameter_count_and_layout():
    assert mlp.NPARAMS == 39428
    th = fixtures.mlp_init(1)
    assert th.size == mlp.NPARAMS
    p = mlp.unpack(th)
    assert p["W1"].shape == (128, 45) and p["W4"].shape == (4, 128)
    assert np.abs(p["W1"]).max() <= math.sqrt(6 / 45) and np.all(p["b2"] == 0)
    np.testing.assert_array_equal(mlp.pack(p), th.astype(np.float64))


def test_gelu_closed_forms():
    # GELU(z) = z Phi(z): Phi(1) = 0.841344746..., Phi(0) = 1/2; derivative at 0 is 1/2
    assert mlp.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-14)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu(np.array([-1.0]))[0] == pytest.approx(-1.0 + 0.8413447460685429, rel=1e-13)
    assert mlp.gelu_grad(np.array([0.0]))[0] == 0.5
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), atol=1e-9)


def test_bf16_rounding_rules():
    u = 2.0 ** -7      # bfloat16 keeps 7 fraction bits: one ulp at 1
    vals = np.array([1.0, 1.0 + u / 2, 1.0 + 3 * u / 2, 1.0 + u / 2 + 2 ** -20, -3.0, 0.0])
    got = mlp.bf16(vals)
    # ties go to even: 1 + u/2 -> 1; 1 + 3u/2 -> 1 + 2u; just above the tie rounds up
    np.testing.assert_array_equal(got, [1.0, 1.0, 1.0 + 2 * u, 1.0 + u, -3.0, 0.0])


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    th = fixtures.mlp_init(3).astype(np.float64)
    th += rng.normal(0, 0.01, th.size)         # nonzero biases too
    x = rng.normal(0, 1, (7, 45))
    t = rng.normal(0, 1, (7, 4))
    g = mlp.grad(th, x, t)
    idx = rng.choice(th.size, 60, replace=False)
    idx = np.concatenate([idx, [0, 5759, 5760 + 3, mlp.NPARAMS - 1, mlp.NPARAMS - 5]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss(th + e, x, t) - mlp.loss(th - e, x, t)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_constant_network_closed_form():
    """With the second and third hidden weights zero, the output is the
    constant W4 gelu(b3) + b4 for any input."""
    th = fixtures.mlp_init(5).astype(np.float64)
    p = mlp.unpack(th)
    p["W3"][:] = 0.0
    p["b3"][:] = np.linspace(-1, 1, 128)
    p["b4"][:] = [0.5, -1.0, 2.0, 0.0]
    y = mlp.forward(mlp.pack(p), np.random.default_rng(1).normal(0, 1, (5, 45)))
    ref = p["W4"] @ mlp.gelu(p["b3"]) + p["b4"]
    np.testing.assert_allclose(y, np.tile(ref, (5, 1)), rtol=1e-14, atol=1e-14)


def test_adam_first_step_is_signed_lr():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 5.0])
    th2, m, v = mlp.adam(th, np.zeros(3), np.zeros(3), g, 1, lr=1e-3)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> update lr g / (|g| + eps)
    np.testing.assert_allclose(th2, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-15)
    np.testing.assert_allclose(th - th2, 1e-3 * np.sign(g), rtol=1e-4)


def test_descent_reduces_loss():
    rng = np.random.default_rng(2)
    th = fixtures.mlp_init(7).astype(np.float64)
    x = rng.normal(0, 1, (64, 45))
    t = np.tanh(x[:, :4])
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0 = mlp.loss(th, x, t)
    for k in range(1, 51):
        th, m, v = mlp.adam(th, m, v, mlp.grad(th, x, t), k, lr=1e-3)
    assert mlp.loss(th, x, t) < 0.5 * l0
