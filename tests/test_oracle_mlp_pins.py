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


def test_forward_by_hand_on_a_one_unit_path():
    # Weights that route one input through one hidden unit of each layer:
    # y_0 = w3 gelu(w2 gelu(w1 xn + b1) + b2) + b3, with xn = (x - shift) * scale,
    # written out with math.erf (rounding off).
    import math
    dims = mlp.layer_dims(3, 128, 2, 128)
    n = sum(i * o for i, o in zip(*dims)) + sum(dims[1])
    vec = np.zeros(n)
    Ws, bs = mlp.unpack(vec, dims)   # views into vec
    w1, w2, w3, b1, b2, b3 = 0.7, -1.3, 2.1, 0.2, -0.4, 0.05
    Ws[0][0, 1] = w1
    Ws[1][0, 0] = w2
    Ws[2][0, 0] = w3
    bs[0][0], bs[1][0], bs[2][0] = b1, b2, b3
    x = np.array([[10.0, 200.0, 30.0]])
    g = lambda z: 0.5 * z * (1.0 + math.erf(z / math.sqrt(2.0)))
    xn = (200.0 - 135.0) / 66.4
    want = w3 * g(w2 * g(w1 * xn + b1) + b2) + b3
    y, _ = mlp.forward(vec, x, dims, 135.0, 1 / 66.4, round=False)
    assert abs(y[0, 0] - want) < 1e-15
    assert np.all(y[0, 1:] == 0.0)


def test_forward_equals_torch_float64_composition():
    # The same network through torch's float64 linear layers and exact-erf GELU
    # (an independent implementation of the composition), rounding off.
    import torch
    rng = np.random.default_rng(3)
    dims = mlp.layer_dims(7, 128, 3, 256)
    n = sum(i * o for i, o in zip(*dims)) + sum(dims[1])
    vec = rng.normal(size=n) * 0.1
    x = rng.uniform(20, 250, (9, 7))
    y, _ = mlp.forward(vec, x, dims, 135.0, 1 / 66.4, round=False)
    Ws, bs = mlp.unpack(vec, dims)
    h = torch.zeros((9, dims[0][0]), dtype=torch.float64)
    h[:, :7] = (torch.as_tensor(x) - 135.0) * (1 / 66.4)
    for l, (W, b) in enumerate(zip(Ws, bs)):
        h = torch.nn.functional.linear(h, torch.as_tensor(W), torch.as_tensor(b))
        if l < len(Ws) - 1:
            h = torch.nn.functional.gelu(h, approximate="none")
    assert np.abs(h.numpy() - y).max() <= 1e-12 * max(1.0, np.abs(y).max())
