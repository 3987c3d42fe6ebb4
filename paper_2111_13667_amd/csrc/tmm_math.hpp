// Elementary functions of the layer loop: sin/cos of pi x and 2^y.
//
// The phase of every layer step needs e^{i pi phi}; the library versions carry
// argument handling this loop does not need, so these are written directly:
// reduction to a table point k/256 and a residual |h| <= 1/512 (sin, cos,
// combined with the table by the angle-sum formulas) or to |f| <= 1/2 (exp2),
// then near-minimax polynomials (Chebyshev fits in 60-digit arithmetic; the
// coefficients and fit errors come from gen_poly.py), evaluated by Horner's
// rule with FMA.  tests/test_phase_math_cpu.py replays these steps on the CPU
// with the constants of this file against 40-digit values (double: within 4
// ulp; float: within 4 float ulp); the compiled kernels are covered by the
// parity tests against the oracle.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tmm_phase_table.hpp"

namespace tmm {

// fit error 3.15e-18
constexpr double kExp2D[12] = {1.0, 0.6931471805599453, 0.24022650695910158, 0.055504108664821625,
                               0.009618129107587256, 0.001333355814640647, 0.00015403530463724353,
                               1.5252733841556773e-05, 1.3215432535912375e-06, 1.0178057087733941e-07,
                               7.074194297288521e-09, 4.4558179083360645e-10};
// fit error 1.95e-09
constexpr float kExp2F[7] = {1.000000000e+00f, 6.931471825e-01f, 2.402265072e-01f, 5.550327152e-02f,
                             9.618056938e-03f, 1.340042800e-03f, 1.546144485e-04f};
// 2^y for weak attenuation, |y| <= 1/16 (no range reduction).
// fit error 2.42e-18
constexpr double kExp2SD[8] = {1.0, 0.6931471805599453, 0.2402265069591204, 0.055504108664823096, 0.00961812908242099, 0.0013333558127014689, 0.00015404562882891175, 1.5253528985683798e-05};
// fit error 8.01e-11
constexpr float kExp2SF[5] = {1.000000000e+00f, 6.931471825e-01f, 2.402265072e-01f, 5.551061779e-02f, 9.618881159e-03f};
constexpr double kExp2WeakRange = 1.0 / 16;

// Table-driven sin/cos of pi x: the table (tmm_phase_table.hpp) holds
// (cos, sin)(pi k / 256) for k = 0..511, one period.  The argument is taken in
// units of 1/256 half-turn, g = 256 x; Sg, Cg are near-minimax fits of
// sin(pi g / 256) = g Sg(g^2), cos(pi g / 256) = Cg(g^2) on |g| <= 1/2, the
// residual after g - round(g).
constexpr int kScSteps = 256;                // table points per half-turn
constexpr int kScEntries = 2 * kScSteps;     // one period, a power of two
// Adding 1.5 * 2^52 rounds a double of magnitude below 2^51 to an integer, and
// the low 32 bits of the sum's encoding are that integer modulo 2^32.
constexpr double kRoundMagic = 6755399441055744.0;
// Largest |g| accepted by sincospi_g (its reduction is exact below 2^51).
constexpr double kScFastRange = 1125899906842624.0;  // 2^50
// fit error 4.06e-21
constexpr double kSinGD[3] = {0.01227184630308513, -3.0801968455583244e-07, 2.319357564247385e-12};
// fit error 2.32e-18
constexpr double kCosGD[3] = {1.0, -7.529910584310532e-05, 9.449907778733635e-10};
// fit error 1.81e-14
constexpr float kSinGF[2] = {1.227184664e-02f, -3.080191107e-07f};
// fit error 7.38e-12
constexpr float kCosGF[2] = {1.000000000e+00f, -7.529887080e-05f};

// One Horner step acc * x + c as a single three-operand FMA with the
// coefficient in scalar registers (it is the same for every lane).  Written as
// an instruction so that the compiler keeps the coefficients out of vector
// registers and does not turn the step into a copy plus a two-operand FMA.
// PIN = false leaves the register choice to the compiler, for kernels whose
// scalar registers are needed elsewhere.
template <bool PIN>
__device__ __forceinline__ double fma3(double a, double x, double c) {
    if (!PIN) return __builtin_fma(a, x, c);
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(x), "s"(c));
    return r;
}
template <bool PIN>
__device__ __forceinline__ float fma3(float a, float x, float c) {
    if (!PIN) return __builtin_fmaf(a, x, c);
    float r;
    asm("v_fma_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(x), "s"(c));
    return r;
}

template <bool PIN, typename T, int N>
__device__ __forceinline__ T horner(const T (&c)[N], T x) {
    T acc = c[N - 1];
#pragma unroll
    for (int k = N - 2; k >= 0; --k) acc = fma3<PIN>(acc, x, c[k]);
    return acc;
}

// Two polynomials in the same variable, Horner steps interleaved so that the
// two dependency chains hide each other's latency (NA >= NB).
template <bool PIN, typename T, int NA, int NB>
__device__ __forceinline__ void horner2(const T (&a)[NA], const T (&b)[NB], T x, T& pa, T& pb) {
    static_assert(NA >= NB, "first polynomial must be the longer one");
    T A = a[NA - 1], Bc = b[NB - 1];
#pragma unroll
    for (int k = NA - 2; k >= 0; --k) {
        A = fma3<PIN>(A, x, a[k]);
        const int kb = k - (NA - NB);
        if (kb >= 0) Bc = fma3<PIN>(Bc, x, b[kb]);
    }
    pa = A;
    pb = Bc;
}

// 2^y; y is clamped to [-1100, 1100] so that the exponent fits an int
// (ldexp then gives 0 or inf, as 2^y itself would).
template <bool PIN = true>
__device__ __forceinline__ double exp2_d(double y) {
    y = __builtin_fmin(__builtin_fmax(y, -1100.0), 1100.0);
    const double k = __builtin_rint(y);
    const double f = y - k;
    return __builtin_amdgcn_ldexp(horner<PIN>(kExp2D, f), (int)k);
}

__device__ __forceinline__ float exp2_f(float y) {
    y = __builtin_fminf(__builtin_fmaxf(y, -200.0f), 200.0f);
    const float k = __builtin_rintf(y);
    const float f = y - k;
    return __builtin_amdgcn_ldexpf(horner<true>(kExp2F, f), (int)k);
}

// Table point and residual of g (units of 1/256 half-turn, |g| < 2^50):
// t = g + 1.5 * 2^52 rounds g to the integer k, the low bits of t's encoding
// give the entry k mod 512, and r = g - k is exact with |r| <= 1/2.
// A non-finite g gives a NaN residual, and the masked index stays in the table.
__device__ __forceinline__ double sc_reduce(double g, uint32_t& idx) {
    const double t = g + kRoundMagic;
    idx = (uint32_t)__double2loint(t) & (uint32_t)(kScEntries - 1);
    return g - (t - kRoundMagic);
}

// e^{i pi g / 256} = (c, s) through the table `tab` (an LDS copy of kScTabD)
// and the angle-sum formulas; |g| < kScFastRange.
template <bool PIN>
__device__ __forceinline__ void sincospi_g(double g, const double2* tab, double& s, double& c) {
    uint32_t idx;
    const double r = sc_reduce(g, idx);
    const double2 t = tab[idx];
    const double r2 = r * r;
    const double sh = r * horner<PIN>(kSinGD, r2);
    const double ch = horner<PIN>(kCosGD, r2);
    c = __builtin_fma(t.x, ch, -(t.y * sh));
    s = __builtin_fma(t.y, ch, t.x * sh);
}

// Same in float: the index and residual in exact double arithmetic, then float
// polynomials and table (`tab` is an LDS copy of kScTabF).
__device__ __forceinline__ void sincospi_g_f(double g, const float2* tab, float& s, float& c) {
    uint32_t idx;
    const float r = (float)sc_reduce(g, idx);
    const float2 t = tab[idx];
    const float r2 = r * r;
    const float sh = r * horner<true>(kSinGF, r2);
    const float ch = horner<true>(kCosGF, r2);
    c = __builtin_fmaf(t.x, ch, -(t.y * sh));
    s = __builtin_fmaf(t.y, ch, t.x * sh);
}

// The same for g = hi + lo held as two floats (hi carries g to 24 bits, lo
// the rest), |hi| < 2^21: adding 1.5 * 2^23 rounds hi to an integer n (exact,
// ulp 1), whose low bits index the table; hi - n is exact (Sterbenz), and lo
// is added to it once.  No double arithmetic.
constexpr float kScRoundF = 12582912.0f;  // 1.5 * 2^23
__device__ __forceinline__ void sincospi_ff(float hi, float lo, const float2* tab, float& s, float& c) {
#pragma clang fp contract(off)  // hi is a rounded product: no FMA may re-form it exactly
    const float t = hi + kScRoundF;
    const uint32_t idx = __float_as_uint(t) & (uint32_t)(kScEntries - 1);
    const float r = (hi - (t - kScRoundF)) + lo;
    const float2 e = tab[idx];
    const float r2 = r * r;
    const float sh = r * horner<true>(kSinGF, r2);
    const float ch = horner<true>(kCosGF, r2);
    c = __builtin_fmaf(e.x, ch, -(e.y * sh));
    s = __builtin_fmaf(e.y, ch, e.x * sh);
}
// Largest |hi| sincospi_ff takes (with room below the 2^22 where the rounding
// constant stops giving integers).
constexpr double kScFastRangeF = 2097152.0;  // 2^21

// Any finite x (half-turns): x is first reduced modulo 2, exactly
// (x - 2 rint(x/2)), then scaled by 256 (exact).
__device__ __forceinline__ double sc_exact_g(double x) {
    return __builtin_fma(-2.0, __builtin_rint(0.5 * x), x) * (double)kScSteps;
}

}  // namespace tmm
