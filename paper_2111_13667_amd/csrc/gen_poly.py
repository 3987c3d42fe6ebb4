"""Generate the polynomial coefficients of tmm_math.hpp.

Near-minimax (Chebyshev) fits in 60-digit arithmetic with mpmath:
  sin(pi r) = r * S(r^2),  cos(pi r) = C(r^2)   for |r| <= 1/4,
  2^f = E(f)                                     for |f| <= 1/2.
Degrees: double S 6, C 7, E 11; float S 3, C 4, E 6.  The printed fit errors
are the approximation errors before rounding the coefficients.
    python gen_poly.py > coefficients.txt
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 60
sinc_pi = lambda s: mp.sinpi(mp.sqrt(s)) / mp.sqrt(s) if s != 0 else mp.pi
cos_pi = lambda s: mp.cospi(mp.sqrt(s))
exp2 = lambda x: mp.power(2, x)
Q = mp.mpf(1) / 16
FITS = [("kSinPiD", sinc_pi, 0, Q, 6, "double"), ("kCosPiD", cos_pi, 0, Q, 7, "double"),
        ("kExp2D", exp2, -0.5, 0.5, 11, "double"),
        ("kSinPiF", sinc_pi, 0, Q, 3, "float"), ("kCosPiF", cos_pi, 0, Q, 4, "float"),
        ("kExp2F", exp2, -0.5, 0.5, 6, "float")]

for name, f, a, b, deg, ty in FITS:
    c, err = mp.chebyfit(f, [mp.mpf(a), mp.mpf(b)], deg + 1, error=True)
    c = [float(x) for x in c[::-1]]
    if ty == "float":
        body = ", ".join("%.9ef" % np.float32(x) for x in c)
    else:
        body = ", ".join(repr(x) for x in c)
    print(f"// fit error {float(err):.2e}")
    print(f"constexpr {ty} {name}[{len(c)}] = {{{body}}};")
