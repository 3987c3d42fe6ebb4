"""Constants and steps of the layer loop's elementary functions (tmm_math.hpp):
the (cos, sin) table at k/64 half-turns, the residual polynomials on |h| <= 1/128
and the exp2 polynomial.  The constants are parsed from the header and the
kernel's steps are replayed in NumPy (float64 / float32, no FMA), then compared
with 40-digit mpmath values.  A wrong table entry, a wrong coefficient or a
wrong reduction step fails here without a GPU."""
import os
import re

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")
mp.mp.dps = 40

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2111_13667_amd", "csrc", "tmm_math.hpp")


def _const(name, dtype):
    src = open(HDR).read()
    m = re.search(r"constexpr (?:double|float) " + name + r"\[[^\]]*\](?:\[2\])? = \{(.*?)\};", src, re.S)
    assert m, name
    vals = [float(v.rstrip("f")) for v in re.findall(r"[-+]?\d[\d.]*(?:e[-+]?\d+)?f?", m.group(1))]
    return np.array(vals, dtype=dtype)


N = 64


def _horner(c, x):
    acc = c[-1]
    for k in range(len(c) - 2, -1, -1):
        acc = acc * x + c[k]
    return acc


def sincospi_tab(x, tab, S, C, ftype):
    x = np.asarray(x, dtype=np.float64)
    k = np.rint(N * x)
    h = (x - k / N).astype(ftype)
    kk = k - 2 * N * np.rint(k * (0.5 / N))          # k modulo 128, in [-64, 64]
    with np.errstate(invalid="ignore"):
        idx = np.clip(np.nan_to_num(kk).astype(np.int64), -N, N) + N
    t = tab[idx]
    h2 = h * h
    sh = h * _horner(S, h2)
    ch = _horner(C, h2)
    return t[:, 0] * ch - t[:, 1] * sh, t[:, 1] * ch + t[:, 0] * sh


def test_table_entries_are_rounded_cos_sin():
    for name, dtype, eps in (("kScTabD", np.float64, 2.0 ** -53), ("kScTabF", np.float32, 2.0 ** -24)):
        tab = _const(name, dtype).reshape(-1, 2)
        assert tab.shape == (2 * N + 1, 2)
        for k in range(-N, N + 1):
            c, s = mp.cospi(mp.mpf(k) / N), mp.sinpi(mp.mpf(k) / N)
            assert abs(float(tab[k + N, 0]) - c) <= eps * max(abs(c), 2.0 ** -60)
            assert abs(float(tab[k + N, 1]) - s) <= eps * max(abs(s), 2.0 ** -60)


def test_sincospi_double_within_a_few_ulp():
    tab = _const("kScTabD", np.float64).reshape(-1, 2)
    S, C = _const("kSinHD", np.float64), _const("kCosHD", np.float64)
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(-3.0, 3.0, 3000), rng.uniform(-2e4, 2e4, 1000),
                         np.arange(-130, 131) / 64.0, np.arange(-130, 131) / 64.0 + 1.0 / 128,
                         [0.0, 0.5, -0.5, 1.0, 1e6 + 0.25, 7.0 / 128 - 1e-17, 2.0 ** 40 + 0.75, -(2.0 ** 52)]])
    c, s = sincospi_tab(xs, tab, S, C, np.float64)
    err = 0.0
    for x, ci, si in zip(xs, c, s):
        xm = mp.mpf(float(x))
        err = max(err, abs(ci - mp.cospi(xm)), abs(si - mp.sinpi(xm)))
    assert err <= 4 * 2.0 ** -53, err


def test_sincospi_float_within_a_few_float_ulp():
    tab = _const("kScTabF", np.float32).reshape(-1, 2)
    S, C = _const("kSinHF", np.float32), _const("kCosHF", np.float32)
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-3.0, 3.0, 3000), rng.uniform(-2e4, 2e4, 500)])
    c, s = sincospi_tab(xs, tab, S, C, np.float32)
    err = max(max(abs(float(ci) - mp.cospi(mp.mpf(float(x)))), abs(float(si) - mp.sinpi(mp.mpf(float(x)))))
              for x, ci, si in zip(xs, c, s))
    assert err <= 4 * 2.0 ** -24, err


def test_non_finite_argument_gives_nan_and_stays_in_the_table():
    tab = _const("kScTabD", np.float64).reshape(-1, 2)
    S, C = _const("kSinHD", np.float64), _const("kCosHD", np.float64)
    with np.errstate(invalid="ignore"):
        c, s = sincospi_tab(np.array([np.inf, -np.inf, np.nan]), tab, S, C, np.float64)
    assert np.isnan(c).all() and np.isnan(s).all()


def test_exp2_polynomial_double():
    E = _const("kExp2D", np.float64)
    rng = np.random.default_rng(2)
    ys = np.concatenate([rng.uniform(-1100.0, 0.0, 2000), rng.uniform(-1.0, 1.0, 1000), [0.0, -0.5, 0.5]])
    k = np.rint(ys)
    f = ys - k
    v = np.ldexp(_horner(E, f), k.astype(np.int64))
    for y, vi in zip(ys, v):
        ref = mp.power(2, mp.mpf(float(y)))
        if ref > mp.mpf(2) ** -1021:   # normal range; below it ldexp rounds to subnormals
            assert abs(vi - ref) <= 4 * 2.0 ** -53 * ref, (y, vi, ref)


def test_exp2_weak_attenuation_series():
    # 2^y on |y| <= 1/64 without range reduction (the kernels' path when every
    # lane of a wave is weakly attenuated)
    for name, dtype, bound in (("kExp2SD", np.float64, 2 * 2.0 ** -53), ("kExp2SF", np.float32, 2 * 2.0 ** -24)):
        E = _const(name, dtype)
        ys = np.linspace(-1.0 / 64, 1.0 / 64, 2001).astype(dtype)
        v = _horner(E, ys)
        err = max(abs(float(vi) - mp.power(2, mp.mpf(float(y)))) / mp.power(2, mp.mpf(float(y)))
                  for y, vi in zip(ys, v))
        assert err <= bound, (name, err)
