"""Constants and steps of the layer loop's elementary functions (tmm_math.hpp,
tmm_phase_table.hpp): the (cos, sin) table at k/256 half-turns, the reduction
through the 1.5 * 2^52 rounding constant, the residual polynomials on
|g| <= 1/2 (g in units of 1/256 half-turn) and the exp2 polynomials.  The
constants are parsed from the headers and the kernel's steps are replayed in
NumPy (float64 / float32, no FMA), then compared with 40-digit mpmath values.
A wrong table entry, a wrong coefficient or a wrong reduction step fails here
without a GPU."""
import os
import re

import numpy as np
import pytest

mp = pytest.importorskip("mpmath")
mp.mp.dps = 40

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2111_13667_amd", "csrc")


def _const(name, dtype):
    src = open(os.path.join(CSRC, "tmm_math.hpp")).read() + open(os.path.join(CSRC, "tmm_phase_table.hpp")).read()
    m = re.search(r"constexpr (?:double|float) " + name + r"\[[^\]]*\](?:\[2\])? = \{(.*?)\};", src, re.S)
    assert m, name
    vals = [float(v.rstrip("f")) for v in re.findall(r"[-+]?\d[\d.]*(?:e[-+]?\d+)?f?", m.group(1))]
    return np.array(vals, dtype=dtype)


def _scalar(name):
    src = open(os.path.join(CSRC, "tmm_math.hpp")).read()
    m = re.search(r"constexpr (?:int|double) " + name + r" = ([^;]+);", src)
    assert m, name
    return m.group(1)


N = 256                     # table points per half-turn
MAGIC = 1.5 * 2.0 ** 52


def _horner(c, x):
    acc = c[-1]
    for k in range(len(c) - 2, -1, -1):
        acc = acc * x + c[k]
    return acc


def exact_g(x):
    """Exact path: x reduced modulo 2 (x - 2 rint(x/2), exact), scaled by 256."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        return (x - 2.0 * np.rint(0.5 * x)) * N


def reduce(g):
    """t = g + 1.5 * 2^52 (rounds g to the integer k), index = low bits of t's
    encoding, residual r = g - (t - 1.5 * 2^52)."""
    g = np.asarray(g, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        t = g + MAGIC
        idx = (t.view(np.uint64) & np.uint64(2 * N - 1)).astype(np.int64)
        r = g - (t - MAGIC)
    return idx, r


def sincospi_g(g, tab, S, C, ftype):
    idx, r = reduce(g)
    r = r.astype(ftype)
    t = tab[idx]
    r2 = r * r
    sh = r * _horner(S, r2)
    ch = _horner(C, r2)
    return t[:, 0] * ch - t[:, 1] * sh, t[:, 1] * ch + t[:, 0] * sh


def test_header_scalars():
    assert int(_scalar("kScSteps")) == N
    assert _scalar("kExp2WeakRange") == "1.0 / 16"
    assert float(_scalar("kRoundMagic")) == MAGIC
    assert float(_scalar("kScFastRange").split("//")[0]) == 2.0 ** 50


def test_table_entries_are_rounded_cos_sin():
    for name, dtype, eps in (("kScTabD", np.float64, 2.0 ** -53), ("kScTabF", np.float32, 2.0 ** -24)):
        tab = _const(name, dtype).reshape(-1, 2)
        assert tab.shape == (2 * N, 2)
        for k in range(2 * N):
            c, s = mp.cospi(mp.mpf(k) / N), mp.sinpi(mp.mpf(k) / N)
            assert abs(float(tab[k, 0]) - c) <= eps * max(abs(c), 2.0 ** -60)
            assert abs(float(tab[k, 1]) - s) <= eps * max(abs(s), 2.0 ** -60)


def test_reduction_is_exact_round_to_table_point():
    # k = round(g) with |r| <= 1/2, the index is k mod 512, and g = k + r holds
    # exactly (checked in rational arithmetic); the exact path's pre-reduction
    # changes x by an even integer only
    rng = np.random.default_rng(3)
    gs = np.concatenate([rng.uniform(-800.0, 800.0, 2000), rng.uniform(-1e12, 1e12, 500),
                         rng.uniform(-2.0 ** 50, 2.0 ** 50, 200), np.arange(-600, 601) * 1.0,
                         np.arange(-600, 601) + 0.5, [-0.0, 2.0 ** 50 - 0.5, -(2.0 ** 50) + 0.25]])
    idx, r = reduce(gs)
    assert np.all(np.abs(r) <= 0.5)
    for g, i, rr in zip(gs, idx, r):
        k = mp.mpf(float(g)) - mp.mpf(float(rr))
        assert k == mp.nint(k), (g, rr)
        assert int(k) % (2 * N) == i, (g, i)
    xs = np.array([3.7, -5.25, 2.0 ** 45 + 0.5, -(2.0 ** 52), 1e300, 7.0])
    for x, g in zip(xs, exact_g(xs)):
        d = (mp.mpf(float(x)) - mp.mpf(float(g)) / N) / 2
        assert d == mp.nint(d) and abs(g) <= N, (x, g)


def test_sincospi_double_within_a_few_ulp():
    tab = _const("kScTabD", np.float64).reshape(-1, 2)
    S, C = _const("kSinGD", np.float64), _const("kCosGD", np.float64)
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(-3.0, 3.0, 3000), rng.uniform(-2e4, 2e4, 1000),
                         np.arange(-520, 521) / 256.0, np.arange(-520, 521) / 256.0 + 1.0 / 512,
                         [0.0, 0.5, -0.5, 1.0, 1e6 + 0.25, 7.0 / 512 - 1e-17, 2.0 ** 40 + 0.75]])
    huge = np.array([2.0 ** 45 + 0.5, -(2.0 ** 52), 2.0 ** 60, 1e300, -3.0 * 2.0 ** 51 + 0.5])
    # fast path: g = 256 x directly (exact scaling, |g| < 2^50); exact path: any finite x
    for xs_, g in ((xs, xs * N), (xs, exact_g(xs)), (huge, exact_g(huge))):
        c, s = sincospi_g(g, tab, S, C, np.float64)
        err = 0.0
        for x, ci, si in zip(xs_, c, s):
            xm = mp.mpf(float(x))
            err = max(err, abs(ci - mp.cospi(xm)), abs(si - mp.sinpi(xm)))
        assert err <= 4 * 2.0 ** -53, err


def test_sincospi_float_within_a_few_float_ulp():
    tab = _const("kScTabF", np.float32).reshape(-1, 2)
    S, C = _const("kSinGF", np.float32), _const("kCosGF", np.float32)
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-3.0, 3.0, 3000), rng.uniform(-2e4, 2e4, 500)])
    c, s = sincospi_g(xs * N, tab, S, C, np.float32)
    err = max(max(abs(float(ci) - mp.cospi(mp.mpf(float(x)))), abs(float(si) - mp.sinpi(mp.mpf(float(x)))))
              for x, ci, si in zip(xs, c, s))
    assert err <= 4 * 2.0 ** -24, err


def test_non_finite_argument_gives_nan_and_stays_in_the_table():
    tab = _const("kScTabD", np.float64).reshape(-1, 2)
    S, C = _const("kSinGD", np.float64), _const("kCosGD", np.float64)
    bad = np.array([np.inf, -np.inf, np.nan])
    for g in (bad, exact_g(bad)):
        idx, _ = reduce(g)
        assert np.all((idx >= 0) & (idx < 2 * N))
        with np.errstate(invalid="ignore"):
            c, s = sincospi_g(g, tab, S, C, np.float64)
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
    # 2^y on |y| <= 1/16 without range reduction (the kernels' path when every
    # lane of a wave is weakly attenuated)
    for name, dtype, bound in (("kExp2SD", np.float64, 2 * 2.0 ** -53), ("kExp2SF", np.float32, 2 * 2.0 ** -24)):
        E = _const(name, dtype)
        ys = np.linspace(-1.0 / 16, 1.0 / 16, 2001).astype(dtype)
        v = _horner(E, ys)
        err = max(abs(float(vi) - mp.power(2, mp.mpf(float(y)))) / mp.power(2, mp.mpf(float(y)))
                  for y, vi in zip(ys, v))
        assert err <= bound, (name, err)
