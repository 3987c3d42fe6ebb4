"""Pins of the float64 MLP reference (CPU only)."""

import numpy as np

from oracle import mlp


def test_gelu_values_from_the_normal_cdf():
    # gelu(z) = z Phi(z): Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145705.
    assert abs(mlp.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array(-1.0)) + 0.15865525393145705) < 1e-15
    assert mlp.gelu(np.array(0.0)) == 0.0
    assert abs(mlp.gelu_grad(np.array(0.0)) - 0.5) < 1e-16
    z = np.linspace(-4, 4, 17)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(z)).max() < 1e-9


def test_bf16_rounding():
    # bfloat16 keeps 8 significand bits: 1 + 2^-8 rounds to 1 (tie to even), 1 + 3*2^-8 to 1 + 2^-6.
    assert mlp.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert mlp.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
    assert mlp.bf16(np.array([-2.5]))[0] == -2.5
    x = np.random.default_rng(0).normal(size=1000)
    assert np.abs(mlp.bf16(x) - x).max() <= np.abs(x).max() * 2.0 ** -8


def test_backward_is_the_derivative_of_forward():
    rng = np.random.default_rng(1)
    dims = mlp.layer_dims(5, 128, 2, 128)
    n = sum(i * o for i, o in zip(*dims)) + sum(dims[1])
    vec = rng.normal(size=n) * 0.05
    x = rng.uniform(20, 250, (6, 5))
    t = rng.uniform(0, 1, (6, 128))
    g = mlp.backward(vec, x, t, dims, 135.0, 1 / 66.0, round=False)
    # directional derivatives by central differences
    for k in range(4):
        v = rng.normal(size=n)
        h = 1e-6
        fd = (mlp.objective(vec + h * v, x, t, dims, 135.0, 1 / 66.0, round=False)
              - mlp.objective(vec - h * v, x, t, dims, 135.0, 1 / 66.0, round=False)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * abs(g @ v) + 1e-12
    # padded input columns get exactly zero gradient
    W0 = g[:128 * dims[0][0]].reshape(128, dims[0][0])
    assert np.all(W0[:, 5:] == 0)
