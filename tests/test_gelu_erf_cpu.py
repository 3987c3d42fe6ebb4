"""The branch-free erf behind the surrogate's GELU epilogues (tmm_mlp_kernels.hpp):
its coefficients are parsed from the header and its float32 steps replayed in
NumPy (no FMA: each step rounds twice, the kernel's fmaf once), then compared
with math.erf.  The kernel's 2^q is the hardware exp2, within one ulp of the
rounded 2^q used here; near |x| >= 0.875 that changes erf by at most
erfc(0.875) * 2^-23 = 2.6e-8."""
import math
import os
import re

import numpy as np

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2111_13667_amd", "csrc")


def _coeffs(name):
    src = open(os.path.join(CSRC, "tmm_mlp_kernels.hpp")).read()
    m = re.search(r"constexpr float " + name + r"\[(\d+)\] = \{(.*?)\};", src, re.S)
    assert m, name
    vals = [np.float32(v.rstrip("f")) for v in re.findall(r"[-+]?\d[\d.]*e[-+]?\d+f", m.group(2))]
    assert len(vals) == int(m.group(1))
    return vals


P = _coeffs("kErfSmall")
Q = _coeffs("kErfcLog2")
f32 = np.float32


def erf_replay(x):
    x = f32(x)
    a = f32(abs(x))
    s = f32(a * a)
    p = P[-1]
    for c in P[-2::-1]:
        p = f32(f32(p * s) + c)
    t = f32(min(a, f32(4.0)))
    q = Q[-1]
    for c in Q[-2::-1]:
        q = f32(f32(q * t) + c)
    r = f32(a * p) if a < f32(0.875) else f32(f32(1.0) - f32(2.0 ** float(q)))
    return math.copysign(float(r), float(x))


def test_erf_fit_accuracy():
    xs = np.concatenate([np.linspace(-6.0, 6.0, 24001), [0.0, -0.0, 0.875, -0.875, np.nextafter(f32(0.875), f32(0)),
                                                        4.0, -4.0, 1e-30, 30.0, -30.0]])
    err = max(abs(erf_replay(x) - math.erf(float(f32(x)))) for x in xs)
    assert err <= 2.5e-7, err


def test_erf_fit_pieces_meet_and_saturate():
    # the two pieces agree at the split to float precision; large |x| gives exactly +-1
    lo = erf_replay(np.nextafter(f32(0.875), f32(0)))
    hi = erf_replay(f32(0.875))
    assert abs(hi - lo) <= 4e-7
    assert erf_replay(10.0) == 1.0 and erf_replay(-10.0) == -1.0
    assert erf_replay(0.0) == 0.0


def test_gelu_from_fit_matches_exact():
    # GELU and its derivative as the epilogues form them, against exact erf
    zs = np.linspace(-8.0, 8.0, 4001)
    for z in zs:
        cdf = 0.5 * (1.0 + erf_replay(f32(z) * f32(0.70710678118654752)))
        cdf_exact = 0.5 * (1.0 + math.erf(z / math.sqrt(2.0)))
        assert abs(z * cdf - z * cdf_exact) <= 1e-6 * max(1.0, abs(z))
