"""Generate the polynomial coefficients and tables of tmm_math.hpp.

Near-minimax (Chebyshev) fits in 60-digit arithmetic with mpmath:
  2^f = E(f)                                     for |f| <= 1/2,
  2^y = Es(y)                                    for |y| <= 1/64 (weak attenuation),
  sin(pi h) = h * Sh(h^2), cos(pi h) = Ch(h^2)  for |h| <= 1/128 (table residual).
Degrees: double E 11, Es 6, Sh 3, Ch 3; float E 6, Es 3, Sh 1, Ch 2.
The printed fit errors are the approximation errors before rounding the
coefficients.  The tables hold cos(pi k/64), sin(pi k/64) for k = -64..64,
rounded to nearest from 60-digit values.
    python gen_poly.py > coefficients.txt
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 60
sinc_pi = lambda s: mp.sinpi(mp.sqrt(s)) / mp.sqrt(s) if s != 0 else mp.pi
cos_pi = lambda s: mp.cospi(mp.sqrt(s))
exp2 = lambda x: mp.power(2, x)
H = mp.mpf(1) / (128 * 128)
S = mp.mpf(1) / 64
FITS = [("kExp2D", exp2, -0.5, 0.5, 11, "double"), ("kExp2F", exp2, -0.5, 0.5, 6, "float"),
        ("kExp2SD", exp2, -S, S, 6, "double"), ("kExp2SF", exp2, -S, S, 3, "float"),
        ("kSinHD", sinc_pi, 0, H, 3, "double"), ("kCosHD", cos_pi, 0, H, 3, "double"),
        ("kSinHF", sinc_pi, 0, H, 1, "float"), ("kCosHF", cos_pi, 0, H, 2, "float")]


def rounded(x, bits):
    with mp.workprec(bits):
        return float(+x)


for name, f, a, b, deg, ty in FITS:
    c, err = mp.chebyfit(f, [mp.mpf(a), mp.mpf(b)], deg + 1, error=True)
    c = [float(x) for x in c[::-1]]
    if ty == "float":
        body = ", ".join("%.9ef" % np.float32(x) for x in c)
    else:
        body = ", ".join(repr(x) for x in c)
    print(f"// fit error {float(err):.2e}")
    print(f"constexpr {ty} {name}[{len(c)}] = {{{body}}};")

N = 64
for name, ty, bits in (("kScTabD", "double", 53), ("kScTabF", "float", 24)):
    rows = []
    for k in range(-N, N + 1):
        cs, sn = mp.cospi(mp.mpf(k) / N), mp.sinpi(mp.mpf(k) / N)
        cs, sn = rounded(cs, bits), rounded(sn, bits)
        if ty == "float":
            rows.append("{%.9ef, %.9ef}" % (np.float32(cs), np.float32(sn)))
        else:
            rows.append("{%r, %r}" % (cs, sn))
    print(f"constexpr {ty} {name}[{2 * N + 1}][2] = {{")
    for i in range(0, len(rows), 2):
        print("    " + ", ".join(rows[i:i + 2]) + ",")
    print("};")
