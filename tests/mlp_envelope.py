"""Element-by-element tolerances for the surrogate's GPU kernels against the
float64 MLP reference (oracle/mlp.py).

The GPU rounds to bfloat16 at the same points as the reference but accumulates
in float32 (and evaluates erf with a fitted polynomial), so a value that the
reference rounds to one bf16 neighbour may land on the other: a difference of
at most one bf16 spacing, 2^-7 of the value's magnitude.  The model here gives
every rounded value an error of up to that size, with independent signs (the
probabilistic model of rounding-error analysis, in which a sum of K terms with
independent errors e_k has an error of order sqrt(sum e_k^2) rather than
sum |e_k|), and propagates the standard deviations through every product of
the forward and backward passes:
    y = h W^T + b           s_y^2 = s_h^2 (W^2)^T + (eps32 |h| |W|^T)^2
    h' = bf16(gelu(z))      s_h'^2 = (gelu'(z) s_z)^2 + (u h')^2
    dh = dz W               s_dh^2 = s_dz^2 W^2
    dz' = bf16(dh gelu'(z)) s_dz'^2 = (gelu'(z) s_dh)^2 + (dh gelu''(z) s_z)^2 + (u dz')^2
    gW = dz^T h             s_gW^2 = (s_dz^2)^T h^2 + (dz^2)^T s_h^2
Every parameter gradient (and output) then gets its own standard deviation s;
the tests accept |gpu - reference| <= lam * s (lam = 8: for Gaussian errors a
2e-15 chance per element of a false alarm).  Mistakes in the kernels (a wrong
operand, index, sign or layer) move elements by far more than the rounding
model allows.
"""
import math

import numpy as np

U_BF16 = 2.0 ** -7          # one bf16 spacing relative to the magnitude (8 significant bits)
EPS32 = 2.0 ** -24
ERF_FIT = 1.2e-7            # absolute error of the kernels' fitted erf
LAMBDA = 8.0


def _gelu_d(z):
    cdf = 0.5 * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf, pdf * (2.0 - z * z)


def _acc(a, W):
    # float32 accumulation noise of a @ W^T: eps32 sqrt(K) |a| |W|^T / sqrt(K) ~ eps32 |a||W|^T
    return EPS32 * (np.abs(a) @ np.abs(W).T)


def _forward(Ws, cache):
    nl = len(Ws)
    W2 = [W * W for W in Ws]
    s_h = U_BF16 * np.abs(cache[0][0])
    s_z = []
    s_hs = [s_h]
    for l in range(nl):
        h, z = cache[l]
        v = (s_h ** 2) @ W2[l].T + _acc(h, Ws[l]) ** 2
        s_z.append(np.sqrt(v))
        if l < nl - 1:
            g1, _ = _gelu_d(z)
            hn = cache[l + 1][0]
            s_h = np.sqrt((g1 * s_z[-1]) ** 2 + (0.5 * ERF_FIT * z) ** 2 + (U_BF16 * hn) ** 2)
            s_hs.append(s_h)
    return s_z, s_hs


def output_sigma(Ws, cache):
    """Standard deviation of every output y of oracle.mlp.forward (cache from it;
    Ws the bf16-rounded weights)."""
    return _forward(Ws, cache)[0][-1]


def sigmas(Ws, bs, y, cache, back):
    """Ws, bs: bf16-rounded weights and the biases per layer; y, cache, back
    from oracle.mlp.backward(..., intermediates=True).  Returns the standard
    deviations of the parameter-gradient vector (export layout) and of y."""
    nl = len(Ws)
    B = y.shape[0]
    W2 = [W * W for W in Ws]
    s_z, s_hs = _forward(Ws, cache)
    s_y = s_z[-1]
    # backward
    dz = back[-1][0]
    s_dz = np.sqrt((2.0 * s_y / B) ** 2 + (U_BF16 * dz) ** 2)
    sW, sb = [None] * nl, [None] * nl
    for l in range(nl - 1, -1, -1):
        h = cache[l][0]
        dz = back[l][0]
        sW[l] = np.sqrt((s_dz ** 2).T @ (h * h) + (dz * dz).T @ (s_hs[l] ** 2) + (EPS32 * (np.abs(dz).T @ np.abs(h))) ** 2)
        sb[l] = np.sqrt((s_dz ** 2).sum(axis=0) + (EPS32 * np.abs(dz).sum(axis=0)) ** 2)
        if l > 0:
            dh = back[l][1]
            zp = cache[l - 1][1]
            g1, g2 = _gelu_d(zp)
            s_dh = np.sqrt((s_dz ** 2) @ W2[l] + (EPS32 * (np.abs(dz) @ np.abs(Ws[l]))) ** 2)
            dz_new = back[l - 1][0]
            s_dz = np.sqrt((g1 * s_dh) ** 2 + (dh * g2 * s_z[l - 1]) ** 2 + (dh * ERF_FIT) ** 2
                           + (U_BF16 * dz_new) ** 2)
    return np.concatenate([s.ravel() for s in sW] + [s for s in sb]), s_y
