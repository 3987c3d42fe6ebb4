// Elementary functions of the layer loop: sin/cos of pi x and 2^y.
//
// The phase of every layer step needs e^{i pi phi}; the library versions carry
// argument handling this loop does not need, so these are written directly:
// exact reduction to |r| <= 1/4 (sin, cos) or |f| <= 1/2 (exp2), then
// near-minimax polynomials (Chebyshev fits in 60-digit arithmetic; the
// coefficients and fit errors come from gen_poly.py), evaluated by Horner's
// rule with FMA.  Accuracy is checked against 50-digit references by the GPU
// tests (double: a few ulp; float: a few float ulp).
#pragma once

#include <hip/hip_runtime.h>

namespace tmm {

// fit error 9.89e-18
constexpr double kSinPiD[7] = {3.141592653589793, -5.167712780049954, 2.5501640398733763, -0.5992645289396449,
                               0.08214586918000175, -0.007370021586907771, 0.000461531855383581};
// fit error 3.03e-20
constexpr double kCosPiD[8] = {1.0, -4.934802200544679, 4.058712126416747, -1.3352627688519174,
                               0.23533063019088787, -0.025806885652951306, 0.0019294657440800042,
                               -0.00010356747255199479};
// fit error 3.15e-18
constexpr double kExp2D[12] = {1.0, 0.6931471805599453, 0.24022650695910158, 0.055504108664821625,
                               0.009618129107587256, 0.001333355814640647, 0.00015403530463724353,
                               1.5252733841556773e-05, 1.3215432535912375e-06, 1.0178057087733941e-07,
                               7.074194297288521e-09, 4.4558179083360645e-10};
// fit error 9.68e-09
constexpr float kSinPiF[4] = {3.141592741e+00f, -5.167707920e+00f, 2.549767017e+00f, -5.890750885e-01f};
// fit error 4.75e-11
constexpr float kCosPiF[5] = {1.000000000e+00f, -4.934802055e+00f, 4.058707237e+00f, -1.335044503e+00f,
                              2.313287854e-01f};
// fit error 1.95e-09
constexpr float kExp2F[7] = {1.000000000e+00f, 6.931471825e-01f, 2.402265072e-01f, 5.550327152e-02f,
                             9.618056938e-03f, 1.340042800e-03f, 1.546144485e-04f};

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

// Quadrant rotation: x = r + k/2 with k in {-2..2}; returns sin(pi x), cos(pi x)
// from sr = sin(pi r), cr = cos(pi r).
template <typename T>
__device__ __forceinline__ void rotate_quadrant(int k, T sr, T cr, T& s, T& c) {
    T ss = (k & 1) ? cr : sr;
    T cc = (k & 1) ? sr : cr;
    s = (k & 2) ? -ss : ss;
    c = ((k + 1) & 2) ? -cc : cc;
}

// sin(pi x), cos(pi x) for finite x.  x - 2 round(x/2) and x - k/2 are exact.
template <bool PIN = true>
__device__ __forceinline__ void sincospi_d(double x, double& s, double& c) {
    x = __builtin_fma(-2.0, __builtin_rint(0.5 * x), x);
    const double k = __builtin_rint(2.0 * x);
    const double r = __builtin_fma(-0.5, k, x);
    const double r2 = r * r;
    double ps, pc;
    horner2<PIN>(kCosPiD, kSinPiD, r2, pc, ps);
    rotate_quadrant((int)k, r * ps, pc, s, c);
}

// Same for a float argument already reduced to |x| <= 1.
__device__ __forceinline__ void sincospi_f(float x, float& s, float& c) {
    const float k = __builtin_rintf(2.0f * x);
    const float r = __builtin_fmaf(-0.5f, k, x);
    const float r2 = r * r;
    float ps, pc;
    horner2<true>(kCosPiF, kSinPiF, r2, pc, ps);
    rotate_quadrant((int)k, r * ps, pc, s, c);
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

}  // namespace tmm
