"""The element-wise tolerances of tests/mlp_envelope.py, checked on the CPU:
an emulation of the GPU kernels' arithmetic (float32 accumulation, bf16 at the
same rounding points as the float64 reference) stays well inside them, and
plausible mistakes (a transposed weight gradient, a sign error, a dropped
layer input) fall far outside."""
import math

import numpy as np
import pytest

from oracle import mlp
from tests import mlp_envelope as env

SHIFT, SCALE = 135.0, 1.0 / 66.4


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def mm32(a, b):
    return (np.asarray(a, np.float32) @ np.asarray(b, np.float32)).astype(np.float64)


def emulate(Wr, bs, x, t, dims):
    """Forward and backward in float32 accumulation with the reference's bf16 points."""
    B = x.shape[0]
    h = np.zeros((B, dims[0][0]))
    h[:, :x.shape[1]] = f32((np.float32(x) - np.float32(SHIFT)) * np.float32(SCALE))
    h = mlp.bf16(h)
    hs, zs = [], []
    for l in range(len(Wr)):
        z = f32(mm32(h, Wr[l].T) + f32(bs[l]))
        hs.append(h)
        zs.append(z)
        if l < len(Wr) - 1:
            h = mlp.bf16(f32(mlp.gelu(z)))
    y = z
    dz = mlp.bf16(f32(2.0 * (y - t) / B))
    gW, gb = [None] * len(Wr), [None] * len(Wr)
    for l in range(len(Wr) - 1, -1, -1):
        gW[l] = mm32(dz.T, hs[l])
        gb[l] = f32(dz.sum(0))
        if l > 0:
            dz = mlp.bf16(f32(mm32(dz, Wr[l]) * mlp.gelu_grad(zs[l - 1])))
    return y, np.concatenate([a.ravel() for a in gW] + gb)


def setup(seed):
    rng = np.random.default_rng(seed)
    dims = mlp.layer_dims(30, 256, 2, 256)
    Ws, bs = [], []
    for i, o in zip(*dims):
        a = math.sqrt(6 / (30 if i == dims[0][0] else i))
        W = rng.uniform(-a, a, (o, i))
        if i == dims[0][0]:
            W[:, 30:] = 0
        Ws.append(W)
        bs.append(rng.normal(size=o) * 0.05)
    vec = np.concatenate([W.ravel() for W in Ws] + bs)
    x = rng.uniform(20, 250, (64, 30))
    t = rng.uniform(0, 1, (64, 256))
    g, y, cache, back = mlp.backward(vec, x, t, dims, SHIFT, SCALE, intermediates=True)
    Wr = [mlp.bf16(W) for W in Ws]
    sg, sy = env.sigmas(Wr, bs, y, cache, back)
    return dims, Wr, bs, x, t, g, y, sg, sy


@pytest.mark.parametrize("seed", [0, 1])
def test_emulated_kernels_stay_inside(seed):
    dims, Wr, bs, x, t, g, y, sg, sy = setup(seed)
    ye, ge = emulate(Wr, bs, x, t, dims)
    assert (np.abs(ye - y) <= 0.25 * env.LAMBDA * sy).all()
    assert (np.abs(ge - g) <= 0.25 * env.LAMBDA * np.maximum(sg, 1e-300)).all()
    # and the tolerance is tight: well under the gradients themselves
    assert np.median(sg / np.maximum(np.abs(g), 1e-300)) < 0.05


def test_plausible_mistakes_fall_outside():
    dims, Wr, bs, x, t, g, y, sg, sy = setup(2)
    _, ge = emulate(Wr, bs, x, t, dims)
    n_last = dims[0][-1] * dims[1][-1]
    o_last = sum(i * o for i, o in zip(*dims)) - n_last
    out = lambda a: (np.abs(a - g) > env.LAMBDA * sg).any()
    # transposed output-layer weight gradient (square 256 x 256 block)
    m = ge.copy()
    blk = m[o_last:o_last + n_last].reshape(dims[1][-1], dims[0][-1])
    m[o_last:o_last + n_last] = blk.T.ravel()
    assert out(m)
    # sign error in the bias gradients
    m = ge.copy()
    m[-sum(dims[1]):] *= -1
    assert out(m)
    # the hidden layers' weight gradients 30 % off (e.g. a wrong derivative factor)
    m = ge.copy()
    m[dims[0][0] * dims[1][0]:o_last] *= 1.3
    assert out(m)
