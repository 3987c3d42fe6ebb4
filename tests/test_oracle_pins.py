"""Pins of the CPU oracle against facts fixed by the physics and mathematics,
not by the oracle's own formulas (CPU only).

Each test names the property and where it comes from.  Together they are chosen
so that a dropped term, a wrong sign or index, or a transposed operand anywhere
in the oracle fails at least one of them.
"""
import numpy as np
import pytest

import oracle
from paper_2111_13667_amd import workloads

mp = pytest.importorskip("mpmath")


def one_stack(n, d, wl, theta, pol="both", flip=None):
    """Run the oracle on one stack given its media n[0..L+1] and thicknesses d."""
    n = np.asarray(n, dtype=np.complex128)
    d = np.asarray(d, dtype=np.float64).reshape(1, -1)
    wl = np.atleast_1d(np.asarray(wl, dtype=np.float64))
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    return oracle.rt(d, n, wl, np.sin(theta), np.cos(theta), pol=pol, flip=flip)


# --- P1: a single interface (L = 0) -----------------------------------------

def test_normal_incidence_single_interface_textbook():
    # Textbook normal-incidence reflectance ((n1-n2)/(n1+n2))^2 and 4 n1 n2/(n1+n2)^2.
    for n1, n2 in [(1.0, 1.5), (1.52, 1.0), (2.35, 1.46), (1.0, 4.0)]:
        o = one_stack([n1, n2], [], 500.0, 0.0)
        R = ((n1 - n2) / (n1 + n2)) ** 2
        T = 4 * n1 * n2 / (n1 + n2) ** 2
        np.testing.assert_allclose(o["R"][0, :, 0, 0], [R, R], rtol=0, atol=1e-15)
        np.testing.assert_allclose(o["T"][0, :, 0, 0], [T, T], rtol=0, atol=1e-15)


def test_brewster_angle_kills_p_reflection():
    # At tan(theta_B) = n2/n1 the p-reflectance vanishes (Brewster); s does not.
    for n1, n2 in [(1.0, 1.5), (1.33, 2.2), (1.6, 1.1)]:
        th = np.arctan(n2 / n1)
        o = one_stack([n1, n2], [], 633.0, th)
        assert o["R"][0, 1, 0, 0] < 1e-28
        assert o["R"][0, 0, 0, 0] > 1e-3


def test_total_internal_reflection():
    # Beyond the critical angle asin(n2/n1) all light is reflected, for s and p.
    th = np.deg2rad(np.array([42.0, 50.0, 70.0, 89.0]))
    o = one_stack([1.52, 1.0], [], 550.0, th)
    np.testing.assert_allclose(o["R"], 1.0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(o["T"], 0.0, rtol=0, atol=1e-14)
    # ... and still with finite films in front of the exit interface.
    o = one_stack([1.52, 2.0, 1.38, 1.0], [80.0, 120.0], 550.0, th)
    np.testing.assert_allclose(o["R"], 1.0, rtol=0, atol=1e-13)


def test_stokes_relations_interface_reversal():
    # Stokes: r' = -r and t t' = 1 - r^2 for the reversed interface (lossless).
    n1, n2 = 1.0, 1.7
    for th1 in np.deg2rad([0.0, 20.0, 45.0, 70.0]):
        th2 = np.arcsin(n1 * np.sin(th1) / n2)
        a = one_stack([n1, n2], [], 500.0, th1)
        b = one_stack([n2, n1], [], 500.0, th2)
        for p in range(2):
            r, t = a["r"][0, p, 0, 0], a["t"][0, p, 0, 0]
            rb, tb = b["r"][0, p, 0, 0], b["t"][0, p, 0, 0]
            assert abs(rb + r) < 1e-15
            assert abs(t * tb - (1 - r * r)) < 1e-15


# --- P2: one layer against the Airy multiple-beam sum -----------------------

def _fresnel(n1, c1, n2, c2, pol):
    if pol == 0:
        den = n1 * c1 + n2 * c2
        return (n1 * c1 - n2 * c2) / den, 2 * n1 * c1 / den
    den = n2 * c1 + n1 * c2
    return (n2 * c1 - n1 * c2) / den, 2 * n1 * c1 / den


def _fwd_cos(n, kx):
    c = np.sqrt(1 - (kx / n) ** 2 + 0j)
    q = n * c
    fwd = q.imag > 0 if abs(q.imag) > 100 * 2.0 ** -52 else q.real > 0
    return c if fwd else -c


@pytest.mark.parametrize("seed", range(6))
def test_single_layer_airy_sum(seed):
    # Summing the multiply-reflected beams inside one film gives
    # r = (r01 + r12 e^{2i d}) / (1 + r01 r12 e^{2i d}),
    # t = t01 t12 e^{i d} / (1 + r01 r12 e^{2i d}).
    rng = np.random.default_rng(seed)
    n0, n2 = 1.0, complex(rng.uniform(1.3, 2.0))
    n1 = complex(rng.uniform(1.2, 3.5), rng.uniform(0, 0.3))
    d = rng.uniform(10, 400)
    wl = rng.uniform(300, 1200, 5)
    th = np.deg2rad(rng.uniform(0, 85, 4))
    o = one_stack([n0, n1, n2], [d], wl, th)
    for k, t0 in enumerate(th):
        kx = n0 * np.sin(t0)
        c0, c1, c2 = np.cos(t0), _fwd_cos(n1, kx), _fwd_cos(n2, kx)
        for i, lam in enumerate(wl):
            delta = 2 * np.pi * n1 * c1 * d / lam
            for p in range(2):
                r01, t01 = _fresnel(n0, c0, n1, c1, p)
                r12, t12 = _fresnel(n1, c1, n2, c2, p)
                den = 1 + r01 * r12 * np.exp(2j * delta)
                r = (r01 + r12 * np.exp(2j * delta)) / den
                t = t01 * t12 * np.exp(1j * delta) / den
                assert abs(o["r"][0, p, k, i] - r) < 1e-14
                assert abs(o["t"][0, p, k, i] - t) < 1e-14


# --- P3: quarter-wave stacks, closed form -----------------------------------

def test_quarter_wave_mirror_normal_incidence():
    # (HL)^N H on a substrate at its design wavelength: the admittance seen from
    # the ambient is Y = (nH/nL)^(2N) nH^2 / ns, so R = ((n0 - Y)/(n0 + Y))^2.
    nH, nL, ns, n0, lam0 = 2.35, 1.46, 1.52, 1.0, 600.0
    for N in [1, 3, 8]:
        n = [n0] + [nH, nL] * N + [nH] + [ns]
        d = [lam0 / (4 * x) for x in n[1:-1]]
        o = one_stack(n, d, lam0, 0.0)
        Y = (nH / nL) ** (2 * N) * nH ** 2 / ns
        R = ((n0 - Y) / (n0 + Y)) ** 2
        np.testing.assert_allclose(o["R"][0, :, 0, 0], [R, R], rtol=2e-13, atol=1e-15)
        np.testing.assert_allclose(o["T"][0, :, 0, 0], [1 - R, 1 - R], rtol=2e-12, atol=1e-15)


def test_quarter_wave_stack_oblique_tilted_admittances():
    # Quarter-wave at an oblique design angle: n_j d_j cos(theta_j) = lam0/4.
    # Tilted admittances eta_s = n cos(theta), eta_p = n / cos(theta); from the
    # substrate outwards Y <- eta_j^2 / Y; R = |(eta_0 - Y)/(eta_0 + Y)|^2.
    n0, ns, lam0, th0 = 1.0, 1.52, 550.0, np.deg2rad(35.0)
    layers = [2.35, 1.46, 2.1, 1.38, 2.35, 1.46, 1.9]
    kx = n0 * np.sin(th0)
    cos = [np.sqrt(1 - (kx / x) ** 2) for x in layers]
    d = [lam0 / (4 * x * c) for x, c in zip(layers, cos)]
    o = one_stack([n0] + layers + [ns], d, lam0, th0)
    cs = np.sqrt(1 - (kx / ns) ** 2)
    for p in range(2):
        eta = (lambda n, c: n * c) if p == 0 else (lambda n, c: n / c)
        Y = eta(ns, cs)
        for x, c in zip(reversed(layers), reversed(cos)):
            Y = eta(x, c) ** 2 / Y
        e0 = eta(n0, np.cos(th0))
        R = abs((e0 - Y) / (e0 + Y)) ** 2
        assert abs(o["R"][0, p, 0, 0] - R) < 1e-13
        assert abs(o["T"][0, p, 0, 0] - (1 - R)) < 1e-13


# --- P4 / P10: energy -------------------------------------------------------

def test_lossless_energy_conservation():
    # R + T = 1 without absorption, any angle below grazing.
    w = workloads.random_stacks(3, B=6, L=17, n_wl=33, n_theta=9, lossy=False, theta_max_deg=89.5)
    o = oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t)
    np.testing.assert_allclose(o["R"] + o["T"], 1.0, rtol=0, atol=1e-13)


def test_passivity_lossy():
    # With k >= 0 everywhere: 0 <= R, 0 <= T, R + T <= 1.
    for w in [workloads.small_batch(), workloads.random_stacks(4, 5, 23, 40, 7, dispersive=True)]:
        o = oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t, mat=w.mat)
        assert (o["R"] >= 0).all() and (o["T"] >= 0).all()
        assert (o["R"] + o["T"] <= 1 + 1e-14).all()
        assert (o["R"] + o["T"] < 1 - 1e-6).any()  # absorption is really there


# --- P5 / P7: invariances ---------------------------------------------------

def test_zero_thickness_layer_is_invisible():
    rng = np.random.default_rng(11)
    n = [1.0, 2.1 + 0.01j, 1.45, 1.9 + 0.002j, 1.52]
    d = [120.0, 75.0, 200.0]
    wl = np.linspace(400, 800, 9)
    th = np.deg2rad([0, 30, 60, 80])
    base = one_stack(n, d, wl, th)
    for pos in range(1, 5):
        extra = complex(rng.uniform(1.1, 4), rng.uniform(0, 0.5))
        n2 = n[:pos] + [extra] + n[pos:]
        d2 = d[:pos - 1] + [0.0] + d[pos - 1:]
        o = one_stack(n2, d2, wl, th)
        for key in "rt":
            assert np.abs(o[key] - base[key]).max() < 1e-14


def test_split_layer_is_invisible():
    n = [1.0, 2.1 + 0.01j, 1.45, 1.52]
    wl = np.linspace(400, 800, 7)
    th = np.deg2rad([0, 45, 75])
    base = one_stack(n, [130.0, 90.0], wl, th)
    o = one_stack([1.0, 2.1 + 0.01j, 2.1 + 0.01j, 1.45, 1.52], [40.0, 90.0, 90.0], wl, th)
    for key in "rt":
        assert np.abs(o[key] - base[key]).max() < 1e-14


def test_half_wave_absentee_layer():
    # A lossless layer with n d cos(theta) = lam0/2 changes neither R nor T at lam0;
    # more generally d -> d + lam/(2 q) leaves R, T unchanged.
    n0, lam0, th0 = 1.0, 633.0, np.deg2rad(25.0)
    n = [n0, 2.0 + 0.01j, 1.5, 1.52]
    d = [100.0, 150.0]
    base = one_stack(n, d, lam0, th0)
    nA = 1.8
    cA = np.sqrt(1 - (n0 * np.sin(th0) / nA) ** 2)
    o = one_stack([n0, 2.0 + 0.01j, nA, 1.5, 1.52], [100.0, lam0 / (2 * nA * cA), 150.0], lam0, th0)
    for key in "RT":
        assert np.abs(o[key] - base[key]).max() < 1e-13
    c2 = np.sqrt(1 - (n0 * np.sin(th0) / 1.5) ** 2)
    o = one_stack(n, [100.0, 150.0 + lam0 / (2 * 1.5 * c2)], lam0, th0)
    for key in "RT":
        assert np.abs(o[key] - base[key]).max() < 1e-13


def test_inner_branch_flip_invariance():
    # The root chosen for q_j of an inner layer does not matter for r and t.
    w = workloads.random_stacks(5, B=1, L=6, n_wl=11, n_theta=5)
    base = oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t)
    for j in range(1, 7):
        flip = np.zeros(8, np.uint8)
        flip[j] = 1
        o = oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t, flip=flip)
        for key in "rt":
            assert np.abs(o[key] - base[key]).max() < 1e-13


# --- P6: reciprocity ----------------------------------------------------------

def test_reciprocity_of_transmittance():
    # Lorentz reciprocity: T is the same when light enters from the other side,
    # at the Snell-conjugate angle, for s and p, absorbing layers included.
    n0, ns = 1.0, 1.52
    inner = [2.2 + 0.03j, 1.46, 1.9 + 0.1j, 1.38]
    d = [80.0, 140.0, 35.0, 210.0]
    wl = np.linspace(420, 900, 13)
    th = np.deg2rad(np.array([0.0, 20.0, 40.0, 60.0, 80.0]))
    fwd = one_stack([n0] + inner + [ns], d, wl, th)
    th_b = np.arcsin(n0 * np.sin(th) / ns)
    bwd = one_stack([ns] + inner[::-1] + [n0], d[::-1], wl, th_b)
    assert np.abs(fwd["T"] - bwd["T"]).max() < 1e-13
    assert np.abs(fwd["R"] - bwd["R"]).max() > 1e-4  # R differs with absorption


# --- P9: normal incidence -----------------------------------------------------

def test_normal_incidence_polarisation_relations():
    # At theta = 0, Eq. (1)-(2) give r_p = -r_s and t_p = t_s, so R_s = R_p, T_s = T_p.
    w = workloads.small_batch()
    o = oracle.rt(w.d, w.nk, w.wl, w.sin_t[:1], w.cos_t[:1])
    assert np.abs(o["r"][:, 1] + o["r"][:, 0]).max() < 1e-14
    assert np.abs(o["t"][:, 1] - o["t"][:, 0]).max() < 1e-14
    assert np.abs(o["R"][:, 1] - o["R"][:, 0]).max() < 1e-14


# --- P11: an independent formulation at 50 digits ----------------------------

def _abeles_mp(n, d, lam, th0, pol):
    """Abeles characteristic (E-H) matrices [[cos D, -i sin D/eta], [-i eta sin D, cos D]]
    with (B, C) = prod M_j (1, eta_sub), r = (eta0 B - C)/(eta0 B + C),
    T = 4 eta0 Re(eta_sub) / |eta0 B + C|^2, in 50-digit arithmetic."""
    mp.mp.dps = 50
    n = [mp.mpc(complex(x)) for x in n]
    lam = mp.mpf(lam)
    kx = n[0] * mp.sin(mp.mpf(th0))
    cos = [mp.cos(mp.mpf(th0))]
    for x in n[1:]:
        c = mp.sqrt(1 - (kx / x) ** 2)
        q = x * c
        fwd = mp.im(q) > 0 if abs(mp.im(q)) > mp.mpf(2) ** -200 else mp.re(q) > 0
        cos.append(c if fwd else -c)
    eta = [(x * c if pol == 0 else x / c) for x, c in zip(n, cos)]
    Bv, Cv = mp.mpc(1), eta[-1]
    for j in range(len(d), 0, -1):
        D = 2 * mp.pi * n[j] * cos[j] * mp.mpf(d[j - 1]) / lam
        cB = mp.cos(D) * Bv - 1j * mp.sin(D) / eta[j] * Cv
        cC = -1j * eta[j] * mp.sin(D) * Bv + mp.cos(D) * Cv
        Bv, Cv = cB, cC
    e0 = eta[0]
    r = (e0 * Bv - Cv) / (e0 * Bv + Cv)
    T = 4 * mp.re(e0) * mp.re(eta[-1]) / abs(e0 * Bv + Cv) ** 2
    t_s = 2 * e0 / (e0 * Bv + Cv)
    return complex(r), float(abs(r) ** 2), float(T), complex(t_s)


# Exit media per seed: 0-3 lossless glass; 4-5 air behind a dense ambient beyond
# the critical angle (evanescent exit: the phase of r depends on its branch);
# 6-7 weakly absorbing glass and 8-9 a metal-like medium (absorbing exit: the
# flux form of T_p, with conj(cos) in Eq. (3)'s Poynting reading, is what the
# admittance formula Re(eta_sub) fixes here).
_ABELES_MEDIA = {0: (1.0, 1.52), 1: (1.0, 1.52), 2: (1.0, 1.52), 3: (1.0, 1.52),
                 4: (1.52, 1.0), 5: (1.52, 1.0), 6: (1.0, 1.52 + 0.05j), 7: (1.33, 1.52 + 0.05j),
                 8: (1.0, 0.2 + 3.5j), 9: (1.0, 0.2 + 3.5j)}


@pytest.mark.parametrize("seed", range(10))
def test_against_50_digit_abeles_matrices(seed):
    rng = np.random.default_rng(100 + seed)
    L = int(rng.integers(1, 14))
    n_in, n_out = _ABELES_MEDIA[seed]
    n = [n_in] + list(rng.uniform(1.3, 2.6, L) + 1j * rng.uniform(0, 0.05, L)) + [n_out]
    d = rng.uniform(10, 300, L)
    wl = rng.uniform(350, 1100, 3)
    th = np.deg2rad(rng.uniform(45, 88, 3) if seed in (4, 5) else rng.uniform(0, 88, 3))
    o = one_stack(n, d, wl, th)
    for k in range(3):
        for i in range(3):
            for p in range(2):
                r, R, T, ts = _abeles_mp(n, d, wl[i], th[k], p)
                # The paper's r_p has the opposite sign of the admittance form's.
                sign = 1 if p == 0 else -1
                assert abs(o["r"][0, p, k, i] - sign * r) < 1e-13
                assert abs(o["R"][0, p, k, i] - R) < 1e-13
                assert abs(o["T"][0, p, k, i] - T) < 1e-13
                if p == 0:
                    assert abs(o["t"][0, p, k, i] - ts) < 1e-13


# --- edge cases of the definition --------------------------------------------

def test_grazing_incidence_is_finite():
    # theta = 90 deg taken with cos computed in float64 (6.1e-17): R -> 1, r -> -1.
    w = workloads.large_batch(B=2, L=40, n_wl=16, n_theta=91)
    o = oracle.rt(w.d, w.nk, w.wl, w.sin_t[-1:], w.cos_t[-1:], mat=w.mat)
    assert np.isfinite(o["R"]).all() and np.isfinite(o["T"]).all()
    np.testing.assert_allclose(o["R"], 1.0, atol=1e-12)
    np.testing.assert_allclose(o["r"], -1.0, atol=1e-12)


def test_invalid_points_are_nan():
    n = np.array([1.0 + 0.1j, 1.5, 1.52])
    o = one_stack(n, [100.0], 500.0, np.deg2rad([0.0, 30.0]))
    assert np.isfinite(o["R"][0, :, 0]).all()     # absorbing ambient, normal incidence
    assert np.isnan(o["R"][0, :, 1]).all()        # ... oblique: undefined
    o = one_stack([1.0, 1.5, 1.52], [-1.0], 500.0, 0.0)
    assert np.isnan(o["R"]).all()
    w = workloads.large_batch(B=2, L=3, n_wl=4, n_theta=2)
    mat = w.mat.copy()
    mat[1, 2] = 6
    o = oracle.rt(w.d, w.nk, w.wl, w.sin_t, w.cos_t, mat=mat)
    assert np.isfinite(o["R"][0]).all() and np.isnan(o["R"][1]).all()
