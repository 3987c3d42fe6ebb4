"""Plain float64 NumPy reference of the surrogate MLP (test infrastructure only).

Forward:  h_0 = bf16((x - shift) * scale) (zero-padded to in_pad features)
          z_l = h_l W_l^T + b_l,  h_{l+1} = bf16(gelu(z_l))       (hidden layers)
          y   = h_L W_L^T + b_L                                   (output, not rounded)
Backward of the objective  l = (1/B) sum_b sum_o (y - t)^2  (summed over the
outputs, averaged over the batch):
          dy = bf16(2 (y - t) / B),  dW_L = dy^T h_L,  db_L = sum_rows dy,
          dz_{l} = bf16((dz_{l+1} W_{l+1}) * gelu'(z_l)), dW_l = dz_l^T h_l, db_l = sum_rows dz_l.
gelu(z) = z Phi(z) (exact, standard normal CDF); gelu'(z) = Phi(z) + z phi(z).
bf16() is round-to-nearest-even to bfloat16 at the points where the GPU kernels
store bfloat16; weights enter as bf16(W).  With round=False every rounding is
skipped and backward() is the exact derivative of forward(), which the pins
check against finite differences.  The layout of a parameter vector is the one
of tmm_surrogate_export: every layer's W [out][in], then every layer's b [out].
"""
from __future__ import annotations

import math

import numpy as np


def bf16(a):
    """Round float values to bfloat16 (round to nearest, ties to even) and widen to float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + _erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def layer_dims(n_in, n_hidden, n_layers, n_out):
    in_pad = ((n_in + 127) // 128) * 128
    din = [in_pad] + [n_hidden] * n_layers
    dout = [n_hidden] * n_layers + [n_out]
    return din, dout


def unpack(vec, dims):
    din, dout = dims
    Ws, bs, o = [], [], 0
    for i, o_ in zip(din, dout):
        Ws.append(vec[o:o + i * o_].reshape(o_, i))
        o += i * o_
    for o_ in dout:
        bs.append(vec[o:o + o_])
        o += o_
    return Ws, bs


def forward(vec, x, dims, shift, scale, round=True):
    """Returns y and the cache of (h_l, z_l) per layer."""
    r = bf16 if round else (lambda a: np.asarray(a, dtype=np.float64))
    Ws, bs = unpack(np.asarray(vec, dtype=np.float64), dims)
    B, n_in = x.shape
    h = np.zeros((B, dims[0][0]))
    h[:, :n_in] = (np.asarray(x, dtype=np.float64) - shift) * scale
    h = r(h)
    cache = []
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = h @ r(W).T + b
        cache.append((h, z))
        if l < len(Ws) - 1:
            h = r(gelu(z))
    return z, cache


def backward(vec, x, t, dims, shift, scale, round=True, intermediates=False):
    """Gradient of the objective w.r.t. the parameter vector (export layout).
    With intermediates=True also returns y, the forward cache and, per layer l,
    (dz_l, dh_l): the layer's output gradient and (l > 0) its input gradient
    before the GELU derivative."""
    r = bf16 if round else (lambda a: np.asarray(a, dtype=np.float64))
    Ws, _ = unpack(np.asarray(vec, dtype=np.float64), dims)
    y, cache = forward(vec, x, dims, shift, scale, round)
    B, n_out = y.shape
    dz = r(2.0 * (y - t) / B)
    gW, gb = [None] * len(Ws), [None] * len(Ws)
    back = [None] * len(Ws)
    for l in range(len(Ws) - 1, -1, -1):
        h, z = cache[l]
        gW[l] = dz.T @ h
        gb[l] = dz.sum(axis=0)
        dh = None
        dz_l = dz
        if l > 0:
            dh = dz @ r(Ws[l])
            dz = r(dh * gelu_grad(cache[l - 1][1]))
        back[l] = (dz_l, dh)
    g = np.concatenate([g.ravel() for g in gW] + [g for g in gb])
    if intermediates:
        return g, y, cache, back
    return g


def objective(vec, x, t, dims, shift, scale, round=True):
    """(1/B) sum_b sum_o (y - t)^2."""
    y, _ = forward(vec, x, dims, shift, scale, round)
    return float(np.sum((y - t) ** 2) / y.shape[0])
