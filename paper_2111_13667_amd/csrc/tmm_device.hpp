// Device-side building blocks of the transfer-matrix kernels (gfx950).
//
// The forward recursion used by every kernel here is the column-0 form of the
// characteristic-matrix product of Eq. (4)-(5), rewritten so that no step
// divides:
//
//   Each layer matrix is M_j = (e^{-i delta_j} / t_j) diag(1, e^{2 i delta_j})
//   [[1, r_j], [r_j, 1]], and [[1, r], [r, 1]] / t = [[D, N], [N, D]] / c with
//   (s)  D = q_j + q_{j+1},        N = q_j - q_{j+1},        c = 2 q_j
//   (p)  D = eta_j + eta_{j+1},    N = eta_{j+1} - eta_j,    c = 2 n_j n_{j+1} / q_{j+1}
//   where q = n cos(theta) and eta = n^2 / q = n / cos(theta).  These are the
//   Fresnel coefficients of Eq. (1)-(2) (mu_r = 1) with numerator and
//   denominator scaled by a common factor.
//
//   Applying M_L ... M_0 to (1, 0) from the substrate side, with the scalar
//   factors e^{-i delta_j} / c_j pulled out, and tracking sigma = y0 + y1,
//   tau = y0 - y1 instead of the vector (y0, y1) itself:
//     a = alpha_j sigma + beta_j tau,  b = alpha_j sigma - beta_j tau,
//     sigma <- a + E_j b,  tau <- a - E_j b,  E_j = e^{2 i delta_j},
//   with alpha_j = q_j, beta_j = q_{j+1} (s) and alpha_j = eta_{j+1},
//   beta_j = eta_j (p).  At the ambient (j = 0, no phase) the first column of
//   the characteristic matrix is proportional to (a, b), so r = b / a
//   (Eq. (7)), and t = P e^{i sum delta} / a with P = prod c_j.
//   |P|^2 needs only the products of |q_j|^2 (s) or |eta_j|^2 (p) over the
//   finite layers, and T follows from Eq. (3) in its Poynting-flux form:
//     T_s = 4^{L+1} (|q_0|^2 / Re q_0) Re(q_sub) prod|q_j|^2 e^{-2 Im sum delta} / |a|^2
//     T_p = 4^{L+1} (|n_0|^2 / (Re n_0 cos theta_0)) Re(eta_sub) prod|eta_j|^2 e^{-2 Im sum delta} / |a|^2
//
// The phase is carried in half-turns: phi_j = 4 d_j q_j / lambda, so that
// 2 delta_j = pi phi_j and E_j = e^{-pi Im phi_j} (cos pi Re phi_j + i sin pi Re phi_j);
// the argument reduction of sin/cos is then an exact subtraction of an integer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tmm_math.hpp"

namespace tmm {

constexpr int kWave = 64;
constexpr double kNegPiLog2e = -4.5323601418271938;  // -pi / ln 2
constexpr double kBranchEps = 100.0 * 2.220446049250313e-16;
// Largest modulus of a tabulated ratio q_{j+1}/q_j or eta_{j+1}/eta_j in the
// ratio form of the recursion (a larger one falls back to the division-free form).
constexpr double kPairRatioMax = 256.0;

template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ R cnorm(cx<R> a) { return a.re * a.re + a.im * a.im; }
template <typename R>
__device__ __forceinline__ cx<R> cscale(R s, cx<R> a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cx<double> cdiv(cx<double> a, cx<double> b) {
    double inv = 1.0 / cnorm(b);
    return {(a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv};
}
template <typename R>
__device__ __forceinline__ cx<double> widen(cx<R> a) { return {(double)a.re, (double)a.im}; }

// Exponent e with |x| = m 2^e, 0.5 <= m < 1 (0 for 0, inf, NaN).
__device__ __forceinline__ int frexp_exp(double x) { return __builtin_amdgcn_frexp_exp(x); }
__device__ __forceinline__ int frexp_exp(float x) { return __builtin_amdgcn_frexp_expf(x); }
__device__ __forceinline__ double ldexp_(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }
__device__ __forceinline__ float ldexp_(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }

// Per-(medium, lane) quantities of one medium at one wavelength and angle,
// computed in double precision: q = n cos(theta) on the forward branch,
// eta = n^2 / q, and their squared moduli.
struct Medium {
    double qr, qi, er, ei, q2, e2;
};

// q = sqrt(n^2 - kx^2) with the forward-wave branch: the decaying root
// (Im q > 0) when |Im q| exceeds 100 ulp(1), else the root with Re q > 0.
// kx = n_0 sin(theta_0) is the invariant of Snell's law.
__device__ __forceinline__ Medium make_medium(double nr, double ni, double kx) {
    const double ur = nr * nr - ni * ni, ui = 2.0 * nr * ni;
    const double zr = ur - kx * kx, zi = ui;
    const double az = sqrt(zr * zr + zi * zi);
    double qr, qi;
    if (zr >= 0.0) {
        const double t = sqrt(0.5 * (az + zr));
        qr = t;
        qi = t > 0.0 ? zi / (2.0 * t) : 0.0;
    } else {
        const double t = sqrt(0.5 * (az - zr));
        qr = fabs(zi) / (2.0 * t);
        qi = copysign(t, zi);
    }
    const bool flip = fabs(qi) > kBranchEps ? (qi < 0.0) : (qr < 0.0);
    if (flip) {
        qr = -qr;
        qi = -qi;
    }
    Medium m;
    m.qr = qr;
    m.qi = qi;
    m.q2 = qr * qr + qi * qi;
    const double inv = 1.0 / m.q2;
    m.er = (ur * qr + ui * qi) * inv;
    m.ei = (ui * qr - ur * qi) * inv;
    m.e2 = m.er * m.er + m.ei * m.ei;
    return m;
}

// make_medium for a real index with n^2 > kx^2 (a lossless, propagating
// medium in this lane): the same operations with Im n = 0 and the complex
// square root reduced to a real one (sqrt(z^2) = |z| exactly), so the same
// values, at a third of the cost.
__device__ __forceinline__ Medium make_medium_lossless(double nr, double kx) {
    const double ur = nr * nr;
    const double zr = ur - kx * kx;
    const double qr = sqrt(zr);
    Medium m;
    m.qr = qr;
    m.qi = 0.0;
    m.q2 = qr * qr;
    const double inv = 1.0 / m.q2;
    m.er = (ur * qr) * inv;
    m.ei = 0.0;
    m.e2 = m.er * m.er;
    return m;
}

// Values of one medium as the chain consumes them, in the kernel's real type R,
// plus q in double for the phase.
template <typename R>
struct Layer {
    cx<R> q, e;
    R q2, e2;
    double pr, pi;
};

template <typename R>
__device__ __forceinline__ Layer<R> to_layer(const Medium& m) {
    Layer<R> v;
    v.q = {(R)m.qr, (R)m.qi};
    v.e = {(R)m.er, (R)m.ei};
    v.q2 = (R)m.q2;
    v.e2 = (R)m.e2;
    v.pr = m.qr;
    v.pi = m.qi;
    return v;
}

// E = e^{i pi phi} for phi = phr + i phi_im (half-turns), through an LDS copy
// of the (cos, sin) table of tmm_phase_table.hpp.  Every workgroup fills its
// copy once (fill_phase_tab, then a barrier) before the layer loops use it.
//   cis_g(g) e^{i pi g / 256} for real g, |g| < kScFastRange (no period reduction);
//   atten(y) 2^y for y <= 0, through the short series when every lane of the
//            wave has |y| <= 1/16 (the usual weakly absorbing layer);
//   (phr, phi_im, lossy)  the whole factor for any finite phr; `lossy` is
//            wave-uniform and false only when phi_im == 0 in every lane, where
//            the modulus is exactly 1.
template <typename R>
struct TabPhase;

template <>
struct TabPhase<double> {
    const double2* tab;
    __device__ __forceinline__ cx<double> cis_g(double g) const {
        double s, c;
        sincospi_g<true>(g, tab, s, c);
        return {c, s};
    }
    __device__ __forceinline__ double atten(double y) const {
        return __all(__builtin_fabs(y) <= kExp2WeakRange) ? horner<true>(kExp2SD, y) : exp2_d<true>(y);
    }
    __device__ __forceinline__ cx<double> operator()(double phr, double phi_im, bool lossy) const {
        cx<double> e = cis_g(sc_exact_g(phr));
        if (lossy) {
            const double rho = atten(phi_im * kNegPiLog2e);
            e.re *= rho;
            e.im *= rho;
        }
        return e;
    }
};

template <>
struct TabPhase<float> {
    const float2* tab;
    __device__ __forceinline__ cx<float> cis_g(double g) const {
        float s, c;
        sincospi_g_f(g, tab, s, c);
        return {c, s};
    }
    // e^{i pi g / 256} for g = hi + lo given as a float pair, |hi| < 2^21:
    // the index and residual in float, exactly up to the final addition of lo.
    __device__ __forceinline__ cx<float> cis_ff(float hi, float lo) const {
        float s, c;
        sincospi_ff(hi, lo, tab, s, c);
        return {c, s};
    }
    __device__ __forceinline__ float atten(double yd) const { return atten_f((float)yd); }
    __device__ __forceinline__ float atten_f(float y) const {
        return __all(__builtin_fabsf(y) <= (float)kExp2WeakRange) ? horner<true>(kExp2SF, y) : exp2_f(y);
    }
    __device__ __forceinline__ cx<float> operator()(double phr, double phi_im, bool lossy) const {
        cx<float> e = cis_g(sc_exact_g(phr));
        if (lossy) {
            const float rho = atten(phi_im * kNegPiLog2e);
            e.re *= rho;
            e.im *= rho;
        }
        return e;
    }
};

// LDS bytes of the table copy (a multiple of 16).
template <typename R>
__host__ __device__ constexpr size_t phase_tab_bytes() {
    return ((size_t)kScEntries * 2 * sizeof(R) + 15) / 16 * 16;
}

// Copy the table into LDS at `lds`; threads tid = 0..nthr-1 of the workgroup share the work.
template <typename R>
__device__ __forceinline__ void fill_phase_tab(unsigned char* lds, int tid, int nthr) {
    for (int e = tid; e < kScEntries; e += nthr) {
        if (sizeof(R) == 8)
            reinterpret_cast<double2*>(lds)[e] = make_double2(kScTabD[e][0], kScTabD[e][1]);
        else
            reinterpret_cast<float2*>(lds)[e] = make_float2(kScTabF[e][0], kScTabF[e][1]);
    }
}

template <typename R>
__device__ __forceinline__ TabPhase<R> phase_of(const unsigned char* lds) {
    TabPhase<R> t;
    t.tab = reinterpret_cast<decltype(t.tab)>(lds);
    return t;
}

// x - 4 round(x / 4): exact, keeps a running half-turn phase within [-2, 2].
__device__ __forceinline__ double reduce4(double x) { return x - 4.0 * rint(0.25 * x); }
// The same for a phase in units of 1/256 half-turn (period 1024).
__device__ __forceinline__ double reduce1024(double g) { return g - 1024.0 * rint(g * (1.0 / 1024)); }

// Scale a pair of complex numbers by a power of two so that the largest
// component is in [0.5, 1); the exponent taken out is added to e.
template <typename R>
__device__ __forceinline__ void renorm_pair(cx<R>& a, cx<R>& b, int& e) {
    const R m = fmax(fmax(fabs(a.re), fabs(a.im)), fmax(fabs(b.re), fabs(b.im)));
    const int k = frexp_exp(m);
    a.re = ldexp_(a.re, -k);
    a.im = ldexp_(a.im, -k);
    b.re = ldexp_(b.re, -k);
    b.im = ldexp_(b.im, -k);
    e += k;
}
template <typename R>
__device__ __forceinline__ void renorm_one(R& a, int& e) {
    const int k = frexp_exp(a);
    a = ldexp_(a, -k);
    e += k;
}
template <typename R>
__device__ __forceinline__ void renorm_cx(cx<R>& a, int& e) {
    const int k = frexp_exp(fmax(fabs(a.re), fabs(a.im)));
    a.re = ldexp_(a.re, -k);
    a.im = ldexp_(a.im, -k);
    e += k;
}

// True for a thickness that is negative (other than -0) or not finite; uses only
// integer operations so that uniform values stay on the scalar unit.
__device__ __forceinline__ bool bad_thickness(double d) {
    const uint64_t u = (uint64_t)__double_as_longlong(d);
    const bool neg = (u >> 63) && (u << 1);
    const bool nonfinite = ((u >> 52) & 0x7ffu) == 0x7ffu;
    return neg || nonfinite;
}
__device__ __forceinline__ bool bad_thickness(float d) {
    const uint32_t u = (uint32_t)__float_as_uint(d);
    const bool neg = (u >> 31) && (u << 1);
    const bool nonfinite = ((u >> 23) & 0xffu) == 0xffu;
    return neg || nonfinite;
}

// ---------------------------------------------------------------------------
// Ambient medium (j = 0), per lane: q_0 = n_0 cos(theta_0), eta_0 = n_0 / cos(theta_0)
// from the given cosine (no square root, so grazing incidence keeps its tiny
// cosine), the Snell invariant kx and the flux constants of T_s, T_p.
struct Ambient {
    double n0r, n0i, q0r, q0i, e0r, e0i, kx, Ks, Kp;
    bool ok;
};

__device__ __forceinline__ Ambient make_ambient(double n0r, double n0i, double st, double ct) {
    Ambient a;
    a.n0r = n0r;
    a.n0i = n0i;
    a.ok = (n0i == 0.0) || (st == 0.0);
    a.kx = n0r * st;
    a.q0r = n0r * ct;
    a.q0i = n0i * ct;
    const double ic = 1.0 / ct;
    a.e0r = n0r * ic;
    a.e0i = n0i * ic;
    const double nn = n0r * n0r + n0i * n0i;
    a.Ks = nn * ct / n0r;
    a.Kp = nn * ic / n0r;
    return a;
}

template <typename R>
__device__ __forceinline__ void load_n(const R* nk, int dispersive, int n_wl, int64_t row, int i,
                                       double& nr, double& ni) {
    const int64_t idx = dispersive ? row * (int64_t)n_wl + i : row;
    nr = (double)nk[2 * idx];
    ni = (double)nk[2 * idx + 1];
}

}  // namespace tmm
