"""Pins of the complex-step derivative oracle (CPU only): its directional
derivatives must match central finite differences of the plain oracle, for
thicknesses and for the real and imaginary parts of the layer indices, in s and
p, for R and for T."""
import numpy as np
import pytest

import oracle
from paper_2111_13667_amd import workloads


def weighted(o, gR, gT):
    return (gR * o["R"]).sum(axis=(1, 2, 3)) + (gT * o["T"]).sum(axis=(1, 2, 3))


def perturbed(w, eps, vd, vn):
    d = w.d + eps * vd
    nk = w.nk.copy()
    B, L = w.d.shape
    for b in range(B):
        rows = b * (L + 2) + 1 + np.arange(L)
        if nk.ndim == 2:
            nk[rows] += eps * vn[b][:, None]
        else:
            nk[rows] += eps * vn[b]
    return d, nk


@pytest.mark.parametrize("seed,dispersive", [(0, False), (1, True), (2, False)])
def test_complex_step_matches_central_differences(seed, dispersive):
    w = workloads.random_stacks(seed, B=3, L=6, n_wl=5, n_theta=4, dispersive=dispersive,
                                theta_max_deg=75)
    rng = np.random.default_rng(seed + 50)
    shape = (w.B, 2, w.theta.size, w.wl.size)
    gR = rng.normal(size=shape)
    gT = rng.normal(size=shape)
    for kind, h in (("d", 1e-4), ("n_re", 1e-7), ("n_im", 1e-7)):
        vd = np.zeros(w.d.shape)
        vn = np.zeros(w.d.shape, complex)
        if kind == "d":
            vd = rng.normal(size=w.d.shape)
        elif kind == "n_re":
            vn = rng.normal(size=w.d.shape) + 0j
        else:
            vn = 1j * rng.normal(size=w.d.shape)
        cs = oracle.rt_dir_cs(w.d, w.nk, w.wl, w.sin_t, w.cos_t, gR=gR, gT=gT, vd=vd, vn=vn)
        dp, np_ = perturbed(w, h, vd, vn)
        dm, nm = perturbed(w, -h, vd, vn)
        fp = weighted(oracle.rt(dp, np_, w.wl, w.sin_t, w.cos_t), gR, gT)
        fm = weighted(oracle.rt(dm, nm, w.wl, w.sin_t, w.cos_t), gR, gT)
        fd = (fp - fm) / (2 * h)
        scale = np.abs(cs).max()
        assert np.abs(cs - fd).max() <= 2e-6 * scale, (kind, cs, fd)


def test_complex_step_zero_direction_is_zero():
    w = workloads.small_batch(B=2)
    shape = (w.B, 2, w.theta.size, w.wl.size)
    D = oracle.rt_dir_cs(w.d, w.nk, w.wl, w.sin_t, w.cos_t, gR=np.ones(shape))
    assert np.all(D == 0.0)


def test_thickness_derivative_of_single_layer_airy():
    # d/dd of the Airy reflectance of one lossless film, written out by hand:
    # R = |r|^2 with r = (r01 + r12 e^{2i delta}) / (1 + r01 r12 e^{2i delta}),
    # delta = 2 pi n1 cos(theta1) d / lam; dr/dd follows from the quotient rule.
    n0, n1, n2, d, lam = 1.0, 2.1, 1.52, 137.0, 613.0
    th = 0.0
    r01 = (n0 - n1) / (n0 + n1)
    r12 = (n1 - n2) / (n1 + n2)
    k = 2 * np.pi * n1 / lam
    E = np.exp(2j * k * d)
    r = (r01 + r12 * E) / (1 + r01 * r12 * E)
    dE = 2j * k * E
    dr = (r12 * dE * (1 + r01 * r12 * E) - (r01 + r12 * E) * r01 * r12 * dE) / (1 + r01 * r12 * E) ** 2
    dR = 2 * (np.conj(r) * dr).real
    nk = np.array([n0, n1, n2], complex)
    D = oracle.rt_dir_cs(np.array([[d]]), nk, np.array([lam]), np.array([np.sin(th)]),
                         np.array([np.cos(th)]), gR=np.array([[[[1.0]]]]), vd=np.array([[1.0]]), pol="s")
    assert abs(D[0] - dR) < 1e-15 * max(1.0, abs(dR)) + 1e-16
