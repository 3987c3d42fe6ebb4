// Ragged batches: stacks with different layer counts, wavelength grids and
// angle grids in one persistent launch (gfx950), behind a plan object that
// owns the work lists, the autotuned launch shape and an optional HIP graph.
//
// A stack's points (angle k, wavelength i) are numbered f = k * n_wl + i, the
// order of its output block.  A work unit is one tile of consecutive points of
// one stack: 64 points at one lane per point, or 32 / 16 points when two or
// four lanes share a point (layer split, below).  Units are ordered by
// decreasing layer count (longest chains first) and handed out through an
// atomic counter, so a wave that finishes early takes the next unit.  For
// every unit each lane computes q, eta of the index-table rows the stack uses
// (its layers' materials and the substrate) at its own (wavelength, angle)
// into the wave's LDS slice, then runs the division-free layer recursion of
// the dense kernels (tmm_chain.hpp) on table lookups; the stack's layer data
// are wave-uniform.
//
// Phase of a layer of thickness d in units of 1/256 half-turn:
// g = d (1024 / lambda) Re q, reduced to a table point by the rounding-constant
// add of tmm_math.hpp (exact for |g| < 2^50; a unit whose thickness and
// indices could exceed that first reduces g modulo 512 exactly).
//
// Layer split (LPP = 2 or 4 lanes per point): the stack's layers are cut into
// LPP contiguous segments; lane s of a point's group runs segment s as a 2x2
// operator (the recursion applied to the two unit states, one renormalisation
// exponent for both columns), and the group then composes the operators
// bottom-up across its lanes (substrate side first) and the top lane finishes
// the point.  Twice the arithmetic per layer, a fraction of the latency: for
// batches with few points per stack.
//
// Amplitudes r, t (Eq. (7)): separate instantiations (AMP) of the one-lane-
// per-point kernel keep the complex running products of q and eta and the
// phase sum (modulo 1024 in units of 1/256 half-turn, two turns: half of it is
// the phase of t), and the shared extraction returns r and t with R and T.
//
// The plan keeps one 64-byte record per stack on the device (its offsets,
// sizes and unit range, built from the offsets it was created with), so the
// kernel never reads a caller's offset array and a wave reads a stack's
// description with one scalar load when its units move on to the next stack.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "tmm_chain.hpp"
#include "tmm_host.hpp"
#include "tmm_ragged.h"

namespace tmm {
namespace ragged {

// Every wave works on its own units with its own media table; a workgroup is
// 1-16 such waves plus the shared phase table, sized at launch so that the
// CU's resident waves fit its LDS.  Resident waves per CU that the kernels'
// registers allow: 3 per SIMD in double (up to 168 VGPRs), 4 in float (128).
template <typename R, bool AMP = false> struct Occupancy;
template <> struct Occupancy<double, false> { static constexpr int kWavesPerCU = 12; };
template <> struct Occupancy<float, false> { static constexpr int kWavesPerCU = 16; };
// r and t wanted: the running products of q and eta are complex and the phase
// sum rides along (FP64: two values spill at 168 registers, still 7 % faster
// than 8 waves without spills)
template <> struct Occupancy<double, true> { static constexpr int kWavesPerCU = 12; };
template <> struct Occupancy<float, true> { static constexpr int kWavesPerCU = 16; };
constexpr int kMaxWavesPerCU = 16;
constexpr int kMaxMat = 8;
constexpr size_t kLdsPerCU = 160 * 1024;
constexpr int kLppChoices[3] = {1, 2, 4};
// A unit whose largest phase coefficient is below 2^kPhaseCoefExp (per unit
// thickness, units of 1/256 half-turn) takes the direct reduction for every
// layer thinner than 2^(49 - kPhaseCoefExp).
constexpr int kPhaseCoefExp = 20;

// What a wave needs of a stack, in one 64-byte record (one scalar load),
// per lanes-per-point choice since the unit ranges differ.
struct StackInfo {
    int64_t l0;          // first layer in d, mat
    int64_t w0;          // first wavelength column
    int64_t t0;          // first angle
    int64_t out0;        // first output element
    int64_t first_unit;  // units [first_unit, end_unit) are this stack's tiles
    int64_t end_unit;
    int32_t L, n_wl, n_th, pad;
};
static_assert(sizeof(StackInfo) == 64, "one 64-byte scalar load per stack");

template <typename R>
struct Params {
    int B;
    const StackInfo* info;  // [B]
    const R* d;
    const int32_t* mat;
    const int32_t* ends;
    const R* wl;
    const R* sin_t;
    const R* cos_t;
    const R* nk;
    int n_mat;
    int64_t nk_stride;  // wl_off[B]
    R* R_out;
    R* T_out;
    const int32_t* unit_stack;  // stack of each unit (units of a stack are consecutive)
    int64_t n_units;
    unsigned long long* counter;
    int grain;
    R* r_out;  // complex interleaved, or null (read by the amplitude kernels only)
    R* t_out;
};

// One index-table row at a lane's point, as the layer step consumes it.
//   FP64: q, eta; the step forms the phase from d (1024 / lambda) and q.
//   FP32: q, eta in float and c = 1024 Re(q) / lambda in double for the phase
//         (reduced in double, evaluated in float, as in the dense kernels).
template <typename R> struct Row;
template <> struct Row<double> { cx<double> q, e; };
template <> struct Row<float> { cx<float> q, e; double c; };

// Per-wave media table in LDS, one block per index-table row, structure of arrays:
//   FP64 [q (double2) x 64][eta (double2) x 64]                     32 bytes per (row, lane)
//   FP32 [c (double) x 64][q.re, q.im, eta.re, eta.im (float4) x 64] 24 bytes per (row, lane)
template <typename R> struct WaveTable;

template <>
struct WaveTable<double> {
    static constexpr int kBlockBytes = kWave * 32;
    unsigned char* base;
    __device__ WaveTable(unsigned char* b) : base(b) {}
    __device__ __forceinline__ void put(int m, int lane, double qr, double qi, double er, double ei, double) {
        double2* blk = reinterpret_cast<double2*>(base + m * kBlockBytes);
        blk[lane] = make_double2(qr, qi);
        blk[kWave + lane] = make_double2(er, ei);
    }
    __device__ __forceinline__ Row<double> get(int m, int lane) const {
        const double2* blk = reinterpret_cast<const double2*>(base + m * kBlockBytes) + lane;
        const double2 a = blk[0], b = blk[kWave];
        return {{a.x, a.y}, {b.x, b.y}};
    }
    __device__ __forceinline__ Row<double> get_qe(int m, int lane) const { return get(m, lane); }
    // The row's refractive index parked in its q slot until put() replaces it.
    __device__ __forceinline__ void stage(int m, int lane, double nr, double ni) {
        reinterpret_cast<double2*>(base + m * kBlockBytes)[lane] = make_double2(nr, ni);
    }
    __device__ __forceinline__ void staged(int m, int lane, double& nr, double& ni) const {
        const double2 v = reinterpret_cast<const double2*>(base + m * kBlockBytes)[lane];
        nr = v.x;
        ni = v.y;
    }
};

template <>
struct WaveTable<float> {
    static constexpr int kBlockBytes = kWave * 24;
    unsigned char* base;
    __device__ WaveTable(unsigned char* b) : base(b) {}
    __device__ __forceinline__ void put(int m, int lane, double qr, double qi, double er, double ei, double c) {
        unsigned char* blk = base + m * kBlockBytes;
        reinterpret_cast<double*>(blk)[lane] = c;
        reinterpret_cast<float4*>(blk + kWave * 8)[lane] = make_float4((float)qr, (float)qi, (float)er, (float)ei);
    }
    __device__ __forceinline__ Row<float> get_qe(int m, int lane) const {
        const float4 v = reinterpret_cast<const float4*>(base + m * kBlockBytes + kWave * 8)[lane];
        return {{v.x, v.y}, {v.z, v.w}, 0.0};
    }
    __device__ __forceinline__ Row<float> get(int m, int lane) const {
        Row<float> r = get_qe(m, lane);
        r.c = reinterpret_cast<const double*>(base + m * kBlockBytes)[lane];
        return r;
    }
    // The row's refractive index parked in its c slot until put() replaces it.
    __device__ __forceinline__ void stage(int m, int lane, float nr, float ni) {
        reinterpret_cast<float2*>(base + m * kBlockBytes)[lane] = make_float2(nr, ni);
    }
    __device__ __forceinline__ void staged(int m, int lane, double& nr, double& ni) const {
        const float2 v = reinterpret_cast<const float2*>(base + m * kBlockBytes)[lane];
        nr = (double)v.x;
        ni = (double)v.y;
    }
};

template <typename R>
__host__ __device__ constexpr size_t wave_lds_bytes(int n_mat) {
    return (size_t)n_mat * WaveTable<R>::kBlockBytes;
}

// The Layer view of a row for the extraction (q in double for the s terms).
template <typename R>
__device__ __forceinline__ Layer<R> as_layer(const Row<R>& r) {
    Layer<R> v;
    v.q = r.q;
    v.e = r.e;
    v.q2 = r.q.re * r.q.re + r.q.im * r.q.im;
    v.e2 = r.e.re * r.e.re + r.e.im * r.e.im;
    v.pr = (double)r.q.re;
    v.pi = (double)r.q.im;
    return v;
}

// Per-lane constants of a unit's point.
struct LaneK {
    double c1024;  // 1024 / lambda
    float kim;     // -(pi / ln 2) 4 / lambda: log2 of the attenuation per unit thickness and unit Im q
};

// g modulo 512 (one full turn in units of 1/256 half-turn), exactly, for any finite g.
__device__ __forceinline__ double reduce512(double g) {
    return __builtin_fma(-512.0, __builtin_rint(g * (1.0 / 512)), g);
}

// 1 / x from the hardware reciprocal and two Newton steps (within about an ulp;
// x = 0 gives NaN, as a division's inf times the zero it multiplies would).
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// q and eta of one row (Snell invariant kx) in double; the forward branch as
// make_medium.  Lossless and propagating in every lane: one real square root.
__device__ __forceinline__ void row_lossless(double nr, double kx, double& qr, double& er) {
    const double ur = nr * nr;
    qr = __builtin_sqrt(ur - kx * kx);
    er = ur * rcp_nr(qr);
}

__device__ __forceinline__ void row_general(double nr, double ni, double kx, double& qr, double& qi, double& er,
                                            double& ei) {
    const double ur = nr * nr - ni * ni, ui = 2.0 * nr * ni;
    const double zr = ur - kx * kx, zi = ui;
    const double az = __builtin_sqrt(zr * zr + zi * zi);
    if (zr >= 0.0) {
        const double t = __builtin_sqrt(0.5 * (az + zr));
        qr = t;
        qi = t > 0.0 ? zi * (0.5 * rcp_nr(t)) : 0.0;
    } else {
        const double t = __builtin_sqrt(0.5 * (az - zr));
        qr = __builtin_fabs(zi) * (0.5 * rcp_nr(t));
        qi = __builtin_copysign(t, zi);
    }
    const bool flip = __builtin_fabs(qi) > kBranchEps ? (qi < 0.0) : (qr < 0.0);
    if (flip) {
        qr = -qr;
        qi = -qi;
    }
    const double inv = rcp_nr(qr * qr + qi * qi);
    er = (ur * qr + ui * qi) * inv;
    ei = (ui * qr - ur * qi) * inv;
}

// 2^y on the short series of weak attenuation alone (its coefficients are the
// only exp2 constants resident in the loop): directly when every lane has
// |y| <= 1/16, else 2^y = 2^k (2^(f/8))^8 with k = rint(y), |f| <= 1/2, three
// squarings (relative error within about 10 ulp).  y is clamped as in exp2_d.
__device__ __forceinline__ double exp2_weak_sq(double y) {
    if (__all(__builtin_fabs(y) <= kExp2WeakRange)) return horner<true>(kExp2SD, y);
    y = __builtin_fmin(__builtin_fmax(y, -1100.0), 1100.0);
    const double k = __builtin_rint(y);
    double v = horner<true>(kExp2SD, (y - k) * 0.125);
    v *= v;
    v *= v;
    v *= v;
    return __builtin_amdgcn_ldexp(v, (int)k);
}

// Division-free recursion (tmm_device.hpp) on table rows.  S sums
// d (1024 / lambda) Im q in double (FP64) or the base-2 exponents of the
// attenuation (FP32); kSLog2 turns it into the latter for the extraction.
template <typename R, int POL, bool AMP = false>
struct RChain : Chain<R, POL, AMP> {
    static constexpr double kSLog2 = sizeof(R) == 8 ? kNegPiLog2e / kScSteps : 1.0;
    __device__ __forceinline__ static double exp2_ext(double y) { return exp2_weak_sq(y); }

    // E_j for the current row (dl = d (1024 / lambda), df = d in the kernel's type).
    template <bool CR>
    __device__ __forceinline__ cx<R> phase_of(const Row<R>& cur, double dl, R df, const LaneK& k, bool huge,
                                              const TabPhase<R>& phase) {
        double g;
        if constexpr (sizeof(R) == 8) g = dl * cur.q.re;
        else g = dl * cur.c;
        if (huge) {
            // rare (wave-uniform): an empty side-effecting asm keeps this a branch
            // rather than a select that would run the reduction on every step
            asm volatile("");
            // one turn is enough for E; the phase sum of t needs two (its half
            // enters the extraction)
            g = AMP ? reduce1024(g) : reduce512(g);
        }
        if constexpr (AMP) this->F = reduce1024(this->F + g);  // in 1/256 half-turn until the extraction
        cx<R> E = phase.cis_g(g);
        if (!CR) attenuate(E, cur, dl, df, k);
        return E;
    }

    // Attenuation of a lossy current row: E scaled by 2^y, y added to S.
    __device__ __forceinline__ void attenuate(cx<R>& E, const Row<R>& cur, double dl, R df, const LaneK& k) {
        R att;
        if constexpr (sizeof(R) == 8) {
            const double ph = dl * cur.q.im;
            this->S += ph;
            att = exp2_weak_sq(ph * kSLog2);
        } else {
            const float y = (df * k.kim) * cur.q.im;
            this->S += (double)y;
            att = __all(__builtin_fabsf(y) <= (float)kExp2WeakRange) ? horner<true>(kExp2SF, y) : exp2_f(y);
        }
        E.re *= att;
        E.im *= att;
    }

    // One layer step; CR / NR: the current / next row is lossless and
    // propagating in every lane (real q and eta), wave-uniform.
    template <bool CR, bool NR>
    __device__ __forceinline__ void step(const Row<R>& cur, const Row<R>& nxt, double dl, R df, const LaneK& k,
                                         bool huge, const TabPhase<R>& phase) {
        step_E<CR, NR>(cur, nxt, phase_of<CR>(cur, dl, df, k, huge, phase));
    }

    // The chain update of a step whose phase factor E is known.
    template <bool CR, bool NR>
    __device__ __forceinline__ void step_E(const Row<R>& cur, const Row<R>& nxt, const cx<R>& E) {
        if (POL & 1) {
            const cx<R> A = CR ? cscale(cur.q.re, this->ss) : cmul(cur.q, this->ss);
            const cx<R> Bv = NR ? cscale(nxt.q.re, this->ts) : cmul(nxt.q, this->ts);
            const cx<R> a = cadd(A, Bv), b = csub(A, Bv);
            const cx<R> Eb = cmul(E, b);
            this->ss = cadd(a, Eb);
            this->ts = csub(a, Eb);
        }
        if (POL & 2) {
            const cx<R> A = NR ? cscale(nxt.e.re, this->sp) : cmul(nxt.e, this->sp);
            const cx<R> Bv = CR ? cscale(cur.e.re, this->tp) : cmul(cur.e, this->tp);
            const cx<R> a = cadd(A, Bv), b = csub(A, Bv);
            const cx<R> Eb = cmul(E, b);
            this->sp = cadd(a, Eb);
            this->tp = csub(a, Eb);
        }
        if constexpr (AMP) {
            if (POL & 1) this->Pq = CR ? cscale(cur.q.re, this->Pq) : cmul(this->Pq, cur.q);
            if (POL & 2) this->Pe = CR ? cscale(cur.e.re, this->Pe) : cmul(this->Pe, cur.e);
        } else {
            if (POL & 1) this->pis *= CR ? cur.q.re * cur.q.re : cur.q.re * cur.q.re + cur.q.im * cur.q.im;
            if (POL & 2) this->pip *= CR ? cur.e.re * cur.e.re : cur.e.re * cur.e.re + cur.e.im * cur.e.im;
        }
    }
};

__global__ void reset_counter(unsigned long long* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0ull;
}

// The recursion applied to two states at once (the columns of a segment's
// operator in the (sigma, tau) basis), with one exponent per polarisation for
// both columns.
template <typename R, int POL>
struct Operator {
    RChain<R, POL> c0, c1;  // column 0 from (1, 0), column 1 from (0, 1); c0 holds es, ep, pis, pip, S
    __device__ __forceinline__ void init() {
        c0.init();
        c1.init();
        c0.ts = c0.tp = {(R)0, (R)0};
        c1.ss = c1.sp = {(R)0, (R)0};
    }
    __device__ __forceinline__ void step(const Row<R>& cur, const Row<R>& nxt, double dl, R df, const LaneK& k,
                                         bool huge, bool lossy, const TabPhase<R>& phase) {
        const cx<R> E = lossy ? c0.template phase_of<false>(cur, dl, df, k, huge, phase)
                              : c0.template phase_of<true>(cur, dl, df, k, huge, phase);
        col(c0, cur, nxt, E);
        col(c1, cur, nxt, E);
        if (POL & 1) c0.pis *= cur.q.re * cur.q.re + cur.q.im * cur.q.im;
        if (POL & 2) c0.pip *= cur.e.re * cur.e.re + cur.e.im * cur.e.im;
    }
    __device__ __forceinline__ static void col(RChain<R, POL>& c, const Row<R>& cur, const Row<R>& nxt,
                                               const cx<R>& E) {
        if (POL & 1) {
            const cx<R> A = cmul(cur.q, c.ss), Bv = cmul(nxt.q, c.ts);
            const cx<R> a = cadd(A, Bv), b = csub(A, Bv);
            const cx<R> Eb = cmul(E, b);
            c.ss = cadd(a, Eb);
            c.ts = csub(a, Eb);
        }
        if (POL & 2) {
            const cx<R> A = cmul(nxt.e, c.sp), Bv = cmul(cur.e, c.tp);
            const cx<R> a = cadd(A, Bv), b = csub(A, Bv);
            const cx<R> Eb = cmul(E, b);
            c.sp = cadd(a, Eb);
            c.tp = csub(a, Eb);
        }
    }
    __device__ __forceinline__ void renorm() {
        if (POL & 1) renorm_joint(c0.ss, c0.ts, c1.ss, c1.ts, c0.es);
        if (POL & 2) renorm_joint(c0.sp, c0.tp, c1.sp, c1.tp, c0.ep);
        if (POL & 1) renorm_one(c0.pis, c0.epis);
        if (POL & 2) renorm_one(c0.pip, c0.epip);
    }
    __device__ __forceinline__ static void renorm_joint(cx<R>& a, cx<R>& b, cx<R>& c, cx<R>& d, int& e) {
        const R m = fmax(fmax(fmax(fabs(a.re), fabs(a.im)), fmax(fabs(b.re), fabs(b.im))),
                         fmax(fmax(fabs(c.re), fabs(c.im)), fmax(fabs(d.re), fabs(d.im))));
        const int k = frexp_exp(m);
        a.re = ldexp_(a.re, -k); a.im = ldexp_(a.im, -k);
        b.re = ldexp_(b.re, -k); b.im = ldexp_(b.im, -k);
        c.re = ldexp_(c.re, -k); c.im = ldexp_(c.im, -k);
        d.re = ldexp_(d.re, -k); d.im = ldexp_(d.im, -k);
        e += k;
    }
};

template <typename R>
__device__ __forceinline__ cx<R> shfl_down_cx(cx<R> v, int d) {
    return {__shfl_down(v.re, d, kWave), __shfl_down(v.im, d, kWave)};
}

// Steps between renormalisations for a unit whose rows' q and eta components
// all lie in [2^(emin-1), 2^emax) (wave-uniform): per step the state grows by
// less than 2^(emax + 2.5) and |q|^2, |eta|^2 lie within 2^(+-(2 |e| + 1)), so
// the chosen period keeps the state and the running products far from
// overflow and underflow.  Powers of two, so that the 64-layer chunks hold
// whole blocks.
template <typename R>
__device__ __forceinline__ int renorm_period(bool small, bool medium);
template <>
__device__ __forceinline__ int renorm_period<double>(bool small, bool medium) { return small ? 64 : (medium ? 32 : 16); }
template <>
__device__ __forceinline__ int renorm_period<float>(bool small, bool medium) { return small ? 16 : (medium ? 8 : 4); }
// Exponent bounds (frexp) for the two longer periods: the largest component
// below 2^hi, each row's largest component at least 2^(lo - 1).  FP64: 64 steps
// keep the state below 2^544 and the products within 2^(+-896); 32 steps below
// 2^(32 x 16.5) and within 2^(+-960).  FP32: 16 steps below 2^96 and within
// 2^(+-112); 8 steps below 2^72 and within 2^(+-112) (normal range 2^-126).
template <typename R> struct PeriodBounds;
template <> struct PeriodBounds<double> {
    static constexpr int kSmallHi = 6, kSmallLo = -6, kMediumHi = 14, kMediumLo = -14;
};
template <> struct PeriodBounds<float> {
    static constexpr int kSmallHi = 3, kSmallLo = -2, kMediumHi = 6, kMediumLo = -6;
};

// Read of a plan or input array at a wave-uniform index through the constant
// address space: a scalar load straight into scalar registers (none of these
// arrays is written while the kernel runs).
template <typename T>
__device__ __forceinline__ T uread(const T* a, int64_t i) {
    return ((const __attribute__((address_space(4))) T*)a)[i];
}

// A stack's record, field by field through uread (one 64-byte scalar load).
__device__ __forceinline__ StackInfo uread_info(const StackInfo* a, int64_t b) {
    const int64_t* w = reinterpret_cast<const int64_t*>(a + b);
    const int32_t* v = reinterpret_cast<const int32_t*>(w + 6);
    StackInfo r;
    r.l0 = uread(w, 0);
    r.w0 = uread(w, 1);
    r.t0 = uread(w, 2);
    r.out0 = uread(w, 3);
    r.first_unit = uread(w, 4);
    r.end_unit = uread(w, 5);
    r.L = uread(v, 0);
    r.n_wl = uread(v, 1);
    r.n_th = uread(v, 2);
    r.pad = 0;
    return r;
}

// Claims the next batch of units; the old counter value arrives in lane 0.
__device__ __forceinline__ unsigned long long claim(unsigned long long* counter, int grain, int lane) {
    unsigned long long v = 0;
    if (lane == 0) v = atomicAdd(counter, (unsigned long long)grain);
    return v;
}

__device__ __forceinline__ int64_t first_lane(unsigned long long v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename R, int POL, int LPP, bool AMP = false>
__global__ void __launch_bounds__((Occupancy<R, AMP>::kWavesPerCU * kWave)) ragged_kernel(Params<R> p) {
    static_assert(!AMP || LPP == 1, "r and t come from the one-lane-per-point chain");
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    fill_phase_tab<R>(smem, threadIdx.x, blockDim.x);
    __syncthreads();
    const TabPhase<R> phase = phase_of<R>(smem);
    unsigned char* my = smem + phase_tab_bytes<R>() + (size_t)wave * wave_lds_bytes<R>(p.n_mat);
    WaveTable<R> tab(my);
    constexpr int P = (POL == 3) ? 2 : 1;
    constexpr int PPW = kWave / LPP;  // points per unit (the tile)
    const int pt = lane / LPP;        // this lane's point within the unit
    const int seg = lane % LPP;       // and its layer segment (0 = ambient side)
    // The next batch is claimed while the current one's first unit runs, so
    // the atomic's round trip overlaps that work.
    int64_t next = first_lane(claim(p.counter, p.grain, lane));
    // the current stack's record and end rows, kept while the units stay in it
    StackInfo si;
    si.first_unit = 1;
    si.end_unit = 0;
    int b = 0, a_raw = 0, s_raw = 0;
    for (;;) {
        const int64_t base = next;
        if (base >= p.n_units) break;
        for (int g = 0; g < p.grain; ++g) {
            const int64_t u = base + g;
            if (u >= p.n_units) break;
            // the stack's description (wave-uniform), read when the unit leaves the last one
            if (u < si.first_unit || u >= si.end_unit) {
                b = uread(p.unit_stack, u);
                si = uread_info(p.info, b);
                a_raw = uread(p.ends, 2 * (int64_t)b);
                s_raw = uread(p.ends, 2 * (int64_t)b + 1);
            }
            const int64_t tile = u - si.first_unit;
            const int64_t l0 = si.l0, w0 = si.w0, t0 = si.t0;
            const int L = si.L, nwl = si.n_wl, nth = si.n_th;
            int a_row = a_raw, s_row = s_raw;
            const int64_t npts = (int64_t)nth * nwl;
            const int64_t f_raw = tile * PPW + pt;
            const bool active = f_raw < npts;
            const int64_t f = active ? f_raw : npts - 1;
            int k, i;
            if (npts <= 0x7fffffff) {  // wave-uniform: 32-bit division
                const uint32_t fu = (uint32_t)f, nw = (uint32_t)nwl;
                const uint32_t ku = fu / nw;
                k = (int)ku;
                i = (int)(fu - ku * nw);
            } else {
                k = (int)(f / nwl);
                i = (int)(f - (int64_t)k * nwl);
            }
            const int64_t col = w0 + i;  // column of this lane's wavelength in nk
            bool bad = (uint32_t)a_row >= (uint32_t)p.n_mat || (uint32_t)s_row >= (uint32_t)p.n_mat;
            a_row = min(max(a_row, 0), p.n_mat - 1);
            s_row = min(max(s_row, 0), p.n_mat - 1);
            const R* drow = p.d + l0;
            const int32_t* mrow = p.mat + l0;
            // Every per-lane read of the unit is issued here, before any of them
            // is used, so that they share one memory round trip: the point's
            // wavelength and angle, the ambient's and every table row's index
            // (rows past n_mat repeat the last one), and the layer list of the
            // top 64-layer chunk (lane l: layer lo1 + l).
            const R lam_r = p.wl[col];
            const R st_r = p.sin_t[t0 + k], ct_r = p.cos_t[t0 + k];
            const R* nkc = p.nk + 2 * col;
            const R an_r = nkc[2 * (int64_t)a_row * p.nk_stride], an_i = nkc[2 * (int64_t)a_row * p.nk_stride + 1];
            R raw_r[kMaxMat], raw_i[kMaxMat];
#pragma unroll
            for (int m = 0; m < kMaxMat; ++m) {
                const int64_t e = 2 * (int64_t)min(m, p.n_mat - 1) * p.nk_stride;
                raw_r[m] = nkc[e];
                raw_i[m] = nkc[e + 1];
            }
            R ns_r = (R)0, ns_i = (R)0;  // the substrate's index (t of p)
            if constexpr (AMP) {
                const int64_t e = 2 * (int64_t)s_row * p.nk_stride;
                ns_r = nkc[e];
                ns_i = nkc[e + 1];
            }
            const int lo1 = max(L - kWave + 1, 1);
            const int j1 = lo1 + lane;
            R d1 = (R)0;
            int m1 = 0;
            if (j1 <= L) {
                d1 = drow[j1 - 1];
                m1 = mrow[j1 - 1];
            }
            const double lam = (double)lam_r;
            const bool lam_ok = lam > 0.0 && lam < __builtin_inf();
            LaneK kk;
            kk.c1024 = (double)(4 * kScSteps) * rcp_nr(lam);
            kk.kim = (float)(kk.c1024 * (kNegPiLog2e / kScSteps));
            const Ambient amb = make_ambient((double)an_r, (double)an_i, (double)st_r, (double)ct_r);
            // rows the stack uses: its layers' materials and the substrate
            uint32_t used = 1u << s_row;
            {
                uint32_t lane_used = j1 <= L ? 1u << min(max(m1, 0), p.n_mat - 1) : 0u;
                for (int j = lane; j < lo1 - 1; j += kWave) lane_used |= 1u << min(max(mrow[j], 0), p.n_mat - 1);
                for (int m = 0; m < p.n_mat; ++m)
                    if (__any((lane_used >> m) & 1u)) used |= 1u << m;
            }
            // this unit's media table: the indices staged in each row's block,
            // then q and eta of the used rows at this lane's point
#pragma unroll
            for (int m = 0; m < kMaxMat; ++m)
                if (m < p.n_mat) tab.stage(m, lane, raw_r[m], raw_i[m]);
            uint32_t lossy_mask = 0;
            int ex_max = -1100, ex_min = 1100, ex_c = -1100;
            for (int m = 0; m < p.n_mat; ++m) {
                if (!((used >> m) & 1u)) continue;
                double nr, ni;
                tab.staged(m, lane, nr, ni);
                double qr, qi = 0.0, er, ei = 0.0;
                if (__all(ni == 0.0 && nr * nr - amb.kx * amb.kx > 0.0)) {
                    row_lossless(nr, amb.kx, qr, er);
                } else {
                    row_general(nr, ni, amb.kx, qr, qi, er, ei);
                    if (__any(qi != 0.0)) lossy_mask |= 1u << m;
                }
                tab.put(m, lane, qr, qi, er, ei, kk.c1024 * qr);
                const double qa = fmax(fabs(qr), fabs(qi)), ea = fmax(fabs(er), fabs(ei));
                ex_max = max(ex_max, max(frexp_exp(qa), frexp_exp(ea)));
                ex_min = min(ex_min, min(frexp_exp(qa), frexp_exp(ea)));
                ex_c = max(ex_c, frexp_exp(kk.c1024 * fabs(qr)));
            }
            // The next batch is claimed now that the unit's reads are consumed
            // (vector memory operations complete in order, so an atomic issued
            // before them would hold up their wait) and read back once the
            // unit is done.
            unsigned long long claimed = 0;
            if (g == 0) claimed = claim(p.counter, p.grain, lane);
            // renormalisation period and phase-range check (wave-uniform)
            using PB = PeriodBounds<R>;
            const int RPu = renorm_period<R>(__all(ex_max <= PB::kSmallHi && ex_min >= PB::kSmallLo),
                                             __all(ex_max <= PB::kMediumHi && ex_min >= PB::kMediumLo));
            const bool c_ok = __all(ex_c <= kPhaseCoefExp);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const Row<R> sub = tab.get_qe(s_row, lane);
            RChain<R, POL, AMP> c;
            int first_row = s_row;  // table row of layer 1 (the substrate for L = 0)
            if constexpr (LPP == 1) {
                int nxt_row = s_row;  // the layer below, as its table row (re-read from LDS per step)
                c.init();
                for (int top = L; top >= 1; top -= kWave) {
                    const int lo = top - kWave + 1 > 1 ? top - kWave + 1 : 1;
                    // lane l holds layer lo + l (thickness, table row); the loop broadcasts them
                    const int j = lo + lane;
                    R dj = d1;  // the top chunk was read with the unit's other reads
                    int mj = m1;
                    if (top != L && j <= top) {
                        dj = drow[j - 1];
                        mj = mrow[j - 1];
                    }
                    R my_d = (R)0;
                    int my_m = 0;
                    bool lane_bad = false;
                    if (j <= top) {
                        lane_bad = bad_thickness(dj) || (uint32_t)mj >= (uint32_t)p.n_mat;
                        my_d = dj;
                        my_m = min(max(mj, 0), p.n_mat - 1);
                    }
                    bad = bad || __any(lane_bad);
                    const bool huge = !c_ok || __any(my_d >= (R)0x1p29);
                    auto step = [&](int jj) {
                        const int sl = jj - lo;
                        const int m = __builtin_amdgcn_readlane(my_m, sl);
                        R df;
                        double dl;
                        if constexpr (sizeof(R) == 8) {
                            df = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(my_d), sl),
                                                  __builtin_amdgcn_readlane(__double2loint(my_d), sl));
                            dl = df * kk.c1024;
                        } else {
                            df = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_d), sl));
                            dl = (double)df;
                        }
                        const Row<R> cur = tab.get(m, lane), nx = tab.get_qe(nxt_row, lane);
                        // lossless rows (bit clear) step with real q and eta
                        if (((lossy_mask >> m) & 1u) == 0) {
                            if (((lossy_mask >> nxt_row) & 1u) == 0)
                                c.template step<true, true>(cur, nx, dl, df, kk, huge, phase);
                            else
                                c.template step<true, false>(cur, nx, dl, df, kk, huge, phase);
                        } else {
                            if (((lossy_mask >> nxt_row) & 1u) == 0)
                                c.template step<false, true>(cur, nx, dl, df, kk, huge, phase);
                            else
                                c.template step<false, false>(cur, nx, dl, df, kk, huge, phase);
                        }
                        nxt_row = m;
                    };
                    // renormalisation blocks of RPu steps (a power of two <= 64:
                    // whole blocks in every chunk but the last)
                    for (int bt = top; bt >= lo; bt -= RPu) {
                        if (bt - lo >= RPu - 1) {
#pragma unroll 2
                            for (int uu = 0; uu < RPu; ++uu) step(bt - uu);
                            c.renorm();
                        } else {
                            for (int jj = bt; jj >= lo; --jj) step(jj);
                        }
                    }
                }
                c.renorm();
                first_row = nxt_row;
            } else {
                // segment seg of the layers: [lo_s, hi_s], equal lengths from the top
                constexpr int RP = RenormPeriod<R>::value;
                const int ns = (L + LPP - 1) / LPP;
                const int lo_s = 1 + seg * ns;
                const int hi_s = min(L, lo_s + ns - 1);
                Operator<R, POL> op;
                op.init();
                int nxt_row = s_row;
                if (hi_s < L) {
                    const int m = mrow[hi_s];  // layer hi_s + 1
                    bad = bad || (uint32_t)m >= (uint32_t)p.n_mat;
                    nxt_row = min(max(m, 0), p.n_mat - 1);
                }
                int cnt = 0;
                for (int uu = 0; uu < ns; ++uu) {
                    const int j = hi_s - uu;
                    if (j >= lo_s) {
                        const R dj = drow[j - 1];
                        const int m_raw = mrow[j - 1];
                        bad = bad || bad_thickness(dj) || (uint32_t)m_raw >= (uint32_t)p.n_mat;
                        const int m = min(max(m_raw, 0), p.n_mat - 1);
                        const bool huge = !c_ok || dj >= (R)0x1p29;
                        const double dl = sizeof(R) == 8 ? (double)dj * kk.c1024 : (double)dj;
                        op.step(tab.get(m, lane), tab.get_qe(nxt_row, lane), dl, dj, kk, huge,
                                (lossy_mask >> m) & 1u, phase);
                        nxt_row = m;
                        if (++cnt == RP) {
                            op.renorm();
                            cnt = 0;
                        }
                    }
                }
                op.renorm();
                bad = __any(bad);
                // state at the top of this segment for the substrate-side input (1, 1)
                // of the bottom segment: compose bottom-up across the group
                c = op.c0;  // exponents, products and phase sums of this segment
                if (POL & 1) {
                    c.ss = cadd(op.c0.ss, op.c1.ss);
                    c.ts = cadd(op.c0.ts, op.c1.ts);
                }
                if (POL & 2) {
                    c.sp = cadd(op.c0.sp, op.c1.sp);
                    c.tp = cadd(op.c0.tp, op.c1.tp);
                }
                for (int r = LPP - 2; r >= 0; --r) {
                    // lane seg = r takes the state reached below it (lane seg + 1) through its operator
                    RChain<R, POL> v = c;
                    if (POL & 1) {
                        v.ss = shfl_down_cx(c.ss, 1);
                        v.ts = shfl_down_cx(c.ts, 1);
                        v.es = __shfl_down(c.es, 1, kWave);
                        v.pis = __shfl_down(c.pis, 1, kWave);
                        v.epis = __shfl_down(c.epis, 1, kWave);
                    }
                    if (POL & 2) {
                        v.sp = shfl_down_cx(c.sp, 1);
                        v.tp = shfl_down_cx(c.tp, 1);
                        v.ep = __shfl_down(c.ep, 1, kWave);
                        v.pip = __shfl_down(c.pip, 1, kWave);
                        v.epip = __shfl_down(c.epip, 1, kWave);
                    }
                    v.S = __shfl_down(c.S, 1, kWave);
                    if (seg == r) {
                        if (POL & 1) {
                            c.ss = cadd(cmul(op.c0.ss, v.ss), cmul(op.c1.ss, v.ts));
                            c.ts = cadd(cmul(op.c0.ts, v.ss), cmul(op.c1.ts, v.ts));
                            c.es = op.c0.es + v.es;
                            c.pis = op.c0.pis * v.pis;
                            c.epis = op.c0.epis + v.epis;
                        }
                        if (POL & 2) {
                            c.sp = cadd(cmul(op.c0.sp, v.sp), cmul(op.c1.sp, v.tp));
                            c.tp = cadd(cmul(op.c0.tp, v.sp), cmul(op.c1.tp, v.tp));
                            c.ep = op.c0.ep + v.ep;
                            c.pip = op.c0.pip * v.pip;
                            c.epip = op.c0.epip + v.epip;
                        }
                        c.S = op.c0.S + v.S;
                        c.renorm();
                    }
                }
                if (L >= 1) {
                    const int m = mrow[0];
                    first_row = min(max(m, 0), p.n_mat - 1);
                }
            }
            PointOut out[2];
            if constexpr (AMP) c.F *= 1.0 / kScSteps;  // half-turns, as the extraction takes them
            finish<R, POL, AMP>(c, amb, as_layer(tab.get_qe(first_row, lane)), as_layer(sub), (double)ns_r,
                                (double)ns_i, L, out, phase);
            if (active && seg == 0) {
                const bool valid = lam_ok && amb.ok && !bad;
                const double nan = __builtin_nan("");
                for (int q = 0; q < P; ++q) {
                    const int64_t o = si.out0 + (int64_t)q * npts + f;
                    if (p.R_out) p.R_out[o] = (R)(valid ? out[q].R : nan);
                    if (p.T_out) p.T_out[o] = (R)(valid ? out[q].T : nan);
                    if constexpr (AMP) {
                        if (p.r_out) {
                            p.r_out[2 * o] = (R)(valid ? out[q].r.re : nan);
                            p.r_out[2 * o + 1] = (R)(valid ? out[q].r.im : nan);
                        }
                        if (p.t_out) {
                            p.t_out[2 * o] = (R)(valid ? out[q].t.re : nan);
                            p.t_out[2 * o + 1] = (R)(valid ? out[q].t.im : nan);
                        }
                    }
                }
            }
            if (g == 0) {
                asm volatile("" : "+v"(claimed));  // keeps the read here, after the unit
                next = first_lane(claimed);
            }
            // the next unit rewrites this wave's table slice
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Launch shape chosen by the autotuner: workgroups per CU, units taken per
// counter update, waves per workgroup, lanes per point (1, 2 or 4; the unit
// then covers 64, 32 or 16 points).
struct Shape {
    int blocks_per_cu;
    int grain;
    int waves;
    int lpp;
};

inline int lpp_index(int lpp) { return lpp == 1 ? 0 : (lpp == 2 ? 1 : 2); }

template <typename R>
size_t shape_lds(int n_mat, int waves) {
    return phase_tab_bytes<R>() + (size_t)waves * wave_lds_bytes<R>(n_mat);
}

// Workgroup shapes that hold the most resident waves per CU (at most the
// kernel's register limit, Occupancy<R>) within the CU's LDS; the three with
// the largest workgroups.
template <typename R, bool AMP>
std::vector<Shape> candidate_shapes(int n_mat) {
    const size_t granule = 2048;
    constexpr int kMax = Occupancy<R, AMP>::kWavesPerCU;
    int best = 0;
    std::vector<Shape> out;
    for (int waves = kMax; waves >= 1; --waves) {
        const size_t lds = (shape_lds<R>(n_mat, waves) + granule - 1) / granule * granule;
        int per_cu = (int)(kLdsPerCU / lds);
        if (per_cu > kMax / waves) per_cu = kMax / waves;
        if (per_cu < 1) continue;
        const int total = per_cu * waves;
        if (total > best) {
            best = total;
            out.clear();
        }
        if (total == best && out.size() < 3) out.push_back({per_cu, 1, waves, 1});
    }
    return out;
}

// Autotune cache: (dtype, r and t wanted, pol, mean-layer bucket, unit-count bucket) -> shape.
std::mutex g_tune_mutex;
std::map<std::tuple<int, int, int, int, int>, Shape> g_tune_cache;

}  // namespace ragged
}  // namespace tmm

struct tmm_ragged_plan {
    int B;
    uint32_t pol_mask;
    int P;
    std::vector<int64_t> layer_off, wl_off, th_off, out_off;
    int64_t n_units[3];     // per lanes-per-point choice (1, 2, 4)
    int64_t out_size;
    int32_t* d_unit_stack[3];
    tmm::ragged::StackInfo* d_info[3];
    unsigned long long* d_counter;
    int n_cu;
    bool tuned[4];
    tmm::ragged::Shape shape[4];  // per dtype (0 F64, 1 F32), + 2 with r and t
    hipGraph_t graph;
    hipGraphExec_t graph_exec;
    int mean_layers;
};

namespace {

using tmm::fail;
using tmm::ok;

template <typename R>
tmm::ragged::Params<R> make_params(const tmm_ragged_plan* pl, const tmm_ragged_data* a) {
    tmm::ragged::Params<R> p;
    p.B = pl->B;
    p.info = pl->d_info[0];
    p.d = static_cast<const R*>(a->d);
    p.mat = a->mat;
    p.ends = a->ends;
    p.wl = static_cast<const R*>(a->wl);
    p.sin_t = static_cast<const R*>(a->sin_theta);
    p.cos_t = static_cast<const R*>(a->cos_theta);
    p.nk = static_cast<const R*>(a->nk);
    p.n_mat = a->n_mat;
    p.nk_stride = pl->wl_off[pl->B];
    p.R_out = static_cast<R*>(a->R);
    p.T_out = static_cast<R*>(a->T);
    p.unit_stack = pl->d_unit_stack[0];
    p.n_units = pl->n_units[0];
    p.counter = pl->d_counter;
    p.grain = 1;
    p.r_out = static_cast<R*>(a->r);
    p.t_out = static_cast<R*>(a->t);
    return p;
}

// Shape slot of a run: the dtype, plus 2 when r or t is wanted (those runs
// have their own kernels and tuned shape).
int shape_slot(const tmm_ragged_data* a, tmm_dtype dt) { return (dt == TMM_F64 ? 0 : 1) + (a->r || a->t ? 2 : 0); }

template <typename R, int POL, int LPP, bool AMP = false>
void launch_one(const tmm::ragged::Params<R>& p, int blocks, dim3 threads, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((tmm::ragged::ragged_kernel<R, POL, LPP, AMP>), dim3(blocks), threads, lds, s, p);
}

template <typename R, int POL>
void launch_pol(const tmm::ragged::Params<R>& p, int lpp, int blocks, dim3 threads, size_t lds, hipStream_t s) {
    if (p.r_out || p.t_out) launch_one<R, POL, 1, true>(p, blocks, threads, lds, s);  // one lane per point
    else if (lpp == 1) launch_one<R, POL, 1>(p, blocks, threads, lds, s);
    else if (lpp == 2) launch_one<R, POL, 2>(p, blocks, threads, lds, s);
    else launch_one<R, POL, 4>(p, blocks, threads, lds, s);
}

template <typename R>
hipError_t launch(const tmm_ragged_plan* pl, tmm::ragged::Params<R> p, tmm::ragged::Shape sh, hipStream_t s) {
    if (p.r_out || p.t_out) sh.lpp = 1;  // the amplitude kernels run one lane per point
    const int li = tmm::ragged::lpp_index(sh.lpp);
    p.grain = sh.grain;
    p.unit_stack = pl->d_unit_stack[li];
    p.info = pl->d_info[li];
    p.n_units = pl->n_units[li];
    const size_t lds = tmm::ragged::shape_lds<R>(p.n_mat, sh.waves);
    const int blocks = pl->n_cu * sh.blocks_per_cu;
    const dim3 threads(sh.waves * tmm::kWave);
    hipLaunchKernelGGL(tmm::ragged::reset_counter, dim3(1), dim3(64), 0, s, pl->d_counter);
    if (pl->pol_mask == 1u)
        launch_pol<R, 1>(p, sh.lpp, blocks, threads, lds, s);
    else if (pl->pol_mask == 2u)
        launch_pol<R, 2>(p, sh.lpp, blocks, threads, lds, s);
    else
        launch_pol<R, 3>(p, sh.lpp, blocks, threads, lds, s);
    return hipGetLastError();
}

// Times every candidate shape on the real data (each run produces the full,
// valid output) and keeps the fastest; the result is cached per
// (dtype, pol, layer bucket, unit bucket) for later plans.
// Dynamic LDS above 64 KiB: raise the kernels' limit (outside any capture).
template <typename R, int POL, int LPP, bool AMP = false>
void raise_one() {
    (void)hipFuncSetAttribute((const void*)&tmm::ragged::ragged_kernel<R, POL, LPP, AMP>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)tmm::ragged::kLdsPerCU);
}

template <typename R>
void raise_lds_limit() {
    raise_one<R, 1, 1>(); raise_one<R, 2, 1>(); raise_one<R, 3, 1>();
    raise_one<R, 1, 2>(); raise_one<R, 2, 2>(); raise_one<R, 3, 2>();
    raise_one<R, 1, 4>(); raise_one<R, 2, 4>(); raise_one<R, 3, 4>();
    raise_one<R, 1, 1, true>(); raise_one<R, 2, 1, true>(); raise_one<R, 3, 1, true>();
    (void)hipGetLastError();
}

// si: the shape slot (shape_slot).
template <typename R>
tmm_status tune(tmm_ragged_plan* pl, const tmm::ragged::Params<R>& p, int si, hipStream_t s) {
    raise_lds_limit<R>();
    const int lb = pl->mean_layers / 16;
    int ub = 0;
    for (int64_t u = pl->n_units[0]; u > 1; u >>= 2) ++ub;
    const bool amp = si >= 2;
    const auto key = std::make_tuple(si & 1, (int)amp, (int)pl->pol_mask, lb, ub);
    {
        std::lock_guard<std::mutex> g(tmm::ragged::g_tune_mutex);
        auto it = tmm::ragged::g_tune_cache.find(key);
        if (it != tmm::ragged::g_tune_cache.end()) {
            // shape known from an earlier plan of the same kind: this run's output
            // still has to be computed
            pl->shape[si] = it->second;
            pl->tuned[si] = true;
            if (launch<R>(pl, p, pl->shape[si], s) != hipSuccess)
                return fail(TMM_ERR_HIP, "tmm_ragged_run: launch failed");
            return ok();
        }
    }
    const std::vector<tmm::ragged::Shape> shapes = amp ? tmm::ragged::candidate_shapes<R, true>(p.n_mat)
                                                       : tmm::ragged::candidate_shapes<R, false>(p.n_mat);
    const int grains[] = {1, 4};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        release();
        return fail(TMM_ERR_HIP, "tmm_ragged_run: event creation failed");
    }
    float best = 1e30f;
    tmm::ragged::Shape best_sh = shapes.front();
    std::vector<tmm::ragged::Shape> trials;
    for (const tmm::ragged::Shape& base : shapes)
        for (int g : grains) trials.push_back({base.blocks_per_cu, g, base.waves, 1});
    // lanes per point 2 and 4 (16- and 32-point tiles) at the largest workgroup shape (R and T only)
    if (!amp)
        for (int lpp : {2, 4})
            for (int g : grains) trials.push_back({shapes.front().blocks_per_cu, g, shapes.front().waves, lpp});
    {
        for (const tmm::ragged::Shape& sh : trials) {
            if (hipEventRecord(e0, s) != hipSuccess || launch<R>(pl, p, sh, s) != hipSuccess ||
                hipEventRecord(e1, s) != hipSuccess) {
                release();
                return fail(TMM_ERR_HIP, "tmm_ragged_run: launch failed while tuning");
            }
            float ms = 0.0f;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                release();
                return fail(TMM_ERR_HIP, "tmm_ragged_run: kernel failed while tuning");
            }
            if (ms < best) {
                best = ms;
                best_sh = sh;
            }
        }
    }
    release();
    pl->shape[si] = best_sh;
    pl->tuned[si] = true;
    // the shapes differ in arithmetic order (lanes per point), so the run's
    // output comes from the chosen one: launch it once more unless it ran last
    const tmm::ragged::Shape& last = trials.back();
    if (last.blocks_per_cu != best_sh.blocks_per_cu || last.grain != best_sh.grain || last.waves != best_sh.waves ||
        last.lpp != best_sh.lpp) {
        if (launch<R>(pl, p, best_sh, s) != hipSuccess) return fail(TMM_ERR_HIP, "tmm_ragged_run: launch failed");
    }
    std::lock_guard<std::mutex> g(tmm::ragged::g_tune_mutex);
    tmm::ragged::g_tune_cache[key] = best_sh;
    return ok();
}

tmm_status check_data(const tmm_ragged_plan* pl, const tmm_ragged_data* a, tmm_dtype dt, const char* who) {
    if (!pl || !a) return fail(TMM_ERR_INVALID_ARG, "%s: NULL argument", who);
    if (dt != TMM_F64 && dt != TMM_F32) return fail(TMM_ERR_INVALID_ARG, "%s: unknown dtype", who);
    if (a->n_mat < 1) return fail(TMM_ERR_INVALID_ARG, "%s: n_mat must be >= 1", who);
    if (a->n_mat > tmm::ragged::kMaxMat)
        return fail(TMM_ERR_UNSUPPORTED, "%s: at most %d index-table rows are supported", who, tmm::ragged::kMaxMat);
    if (!a->R && !a->T && !a->r && !a->t) return fail(TMM_ERR_INVALID_ARG, "%s: no output requested", who);
    if (pl->B > 0 && (!a->ends || !a->wl || !a->sin_theta || !a->cos_theta || !a->nk))
        return fail(TMM_ERR_INVALID_ARG, "%s: ends, wl, sin_theta, cos_theta and nk must be non-NULL", who);
    if (pl->layer_off[pl->B] > 0 && (!a->d || !a->mat))
        return fail(TMM_ERR_INVALID_ARG, "%s: d and mat must be non-NULL", who);
    return ok();
}

}  // namespace

extern "C" {

tmm_status tmm_ragged_plan_create(int32_t B, const int64_t* layer_off, const int64_t* wl_off, const int64_t* th_off,
                                  uint32_t pol_mask, tmm_ragged_plan** out) {
    if (!out) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_create: out is NULL");
    *out = nullptr;
    if (B < 0 || !layer_off || !wl_off || !th_off)
        return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_create: B >= 0 and host offset arrays required");
    if (pol_mask < 1u || pol_mask > 3u) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_create: bad pol_mask");
    if (layer_off[0] != 0 || wl_off[0] != 0 || th_off[0] != 0)
        return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_create: offsets must start at 0");
    const int P = pol_mask == 3u ? 2 : 1;
    std::vector<int64_t> oo(B + 1, 0);
    std::vector<int> order(B);
    for (int b = 0; b < B; ++b) {
        const int64_t L = layer_off[b + 1] - layer_off[b];
        const int64_t nw = wl_off[b + 1] - wl_off[b];
        const int64_t nt = th_off[b + 1] - th_off[b];
        if (L < 0 || L > (1 << 20) || nw < 1 || nt < 1 || nw > 64 * 65535 || nt > 32767)
            return fail(TMM_ERR_INVALID_ARG,
                        "tmm_ragged_plan_create: stack %d has L=%lld, n_wl=%lld, n_theta=%lld (need 0 <= L <= 2^20, "
                        "1 <= n_wl <= 4194240, 1 <= n_theta <= 32767)", b, (long long)L, (long long)nw, (long long)nt);
        oo[b + 1] = oo[b] + P * nt * nw;
        order[b] = b;
    }
    if (wl_off[B] > ((int64_t)1 << 40)) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_create: too many wavelengths");
    // longest chains first; ties keep the input order
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return layer_off[x + 1] - layer_off[x] > layer_off[y + 1] - layer_off[y];
    });
    // work lists per lanes-per-point choice: the tiles of consecutive points of
    // each stack, stacks in the sorted order; unit -> stack, stack -> first unit
    std::vector<int32_t> unit_stack[3];
    std::vector<tmm::ragged::StackInfo> info[3];
    int64_t n_units[3];
    for (int li = 0; li < 3; ++li) {
        const int64_t ppw = tmm::kWave / tmm::ragged::kLppChoices[li];
        info[li].assign((size_t)B, tmm::ragged::StackInfo{});
        int64_t n = 0;
        for (int b : order) n += ((wl_off[b + 1] - wl_off[b]) * (th_off[b + 1] - th_off[b]) + ppw - 1) / ppw;
        if (n > ((int64_t)1 << 31) - 1)
            return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_create: more than 2^31 work units");
        unit_stack[li].reserve((size_t)n);
        for (int b : order) {
            const int64_t tiles = ((wl_off[b + 1] - wl_off[b]) * (th_off[b + 1] - th_off[b]) + ppw - 1) / ppw;
            tmm::ragged::StackInfo& r = info[li][b];
            r.l0 = layer_off[b];
            r.w0 = wl_off[b];
            r.t0 = th_off[b];
            r.out0 = oo[b];
            r.first_unit = (int64_t)unit_stack[li].size();
            r.end_unit = r.first_unit + tiles;
            r.L = (int32_t)(layer_off[b + 1] - layer_off[b]);
            r.n_wl = (int32_t)(wl_off[b + 1] - wl_off[b]);
            r.n_th = (int32_t)(th_off[b + 1] - th_off[b]);
            r.pad = 0;
            unit_stack[li].insert(unit_stack[li].end(), (size_t)tiles, b);
        }
        n_units[li] = n;
    }
    tmm_ragged_plan* pl = new tmm_ragged_plan();
    pl->B = B;
    pl->pol_mask = pol_mask;
    pl->P = P;
    pl->layer_off.assign(layer_off, layer_off + B + 1);
    pl->wl_off.assign(wl_off, wl_off + B + 1);
    pl->th_off.assign(th_off, th_off + B + 1);
    pl->out_off = oo;
    for (int li = 0; li < 3; ++li) {
        pl->n_units[li] = n_units[li];
        pl->d_unit_stack[li] = nullptr;
        pl->d_info[li] = nullptr;
    }
    pl->out_size = oo[B];
    for (int i = 0; i < 4; ++i) pl->tuned[i] = false;
    pl->graph = nullptr;
    pl->graph_exec = nullptr;
    pl->d_counter = nullptr;
    pl->mean_layers = B > 0 ? (int)(layer_off[B] / B) : 0;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete pl;
        return fail(TMM_ERR_HIP, "tmm_ragged_plan_create: no device");
    }
    pl->n_cu = prop.multiProcessorCount;
    bool okk = hipMalloc((void**)&pl->d_counter, sizeof(unsigned long long)) == hipSuccess;
    for (int li = 0; okk && li < 3; ++li) {
        const size_t nu = std::max<size_t>(1, unit_stack[li].size()) * sizeof(int32_t);
        const size_t ns = std::max<size_t>(1, (size_t)B) * sizeof(tmm::ragged::StackInfo);
        okk = hipMalloc((void**)&pl->d_unit_stack[li], nu) == hipSuccess &&
              hipMalloc((void**)&pl->d_info[li], ns) == hipSuccess &&
              (unit_stack[li].empty() || hipMemcpy(pl->d_unit_stack[li], unit_stack[li].data(),
                                                   unit_stack[li].size() * sizeof(int32_t),
                                                   hipMemcpyHostToDevice) == hipSuccess) &&
              (B == 0 || hipMemcpy(pl->d_info[li], info[li].data(), (size_t)B * sizeof(tmm::ragged::StackInfo),
                                   hipMemcpyHostToDevice) == hipSuccess);
    }
    if (!okk) {
        tmm_ragged_plan_destroy(pl);
        return fail(TMM_ERR_HIP, "tmm_ragged_plan_create: device allocation or copy failed");
    }
    *out = pl;
    return ok();
}

tmm_status tmm_ragged_plan_destroy(tmm_ragged_plan* pl) {
    if (!pl) return ok();
    (void)hipDeviceSynchronize();
    if (pl->graph_exec) (void)hipGraphExecDestroy(pl->graph_exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    void* ptrs[] = {pl->d_counter,   pl->d_unit_stack[0], pl->d_unit_stack[1], pl->d_unit_stack[2],
                    pl->d_info[0],  pl->d_info[1],       pl->d_info[2]};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete pl;
    return ok();
}

int64_t tmm_ragged_plan_output_size(const tmm_ragged_plan* pl) { return pl ? pl->out_size : -1; }

tmm_status tmm_ragged_plan_output_offsets(const tmm_ragged_plan* pl, int64_t* host_out_off) {
    if (!pl || !host_out_off) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_output_offsets: NULL argument");
    memcpy(host_out_off, pl->out_off.data(), (size_t)(pl->B + 1) * sizeof(int64_t));
    return ok();
}

tmm_status tmm_ragged_run(tmm_ragged_plan* pl, const tmm_ragged_data* a, tmm_dtype dtype, void* stream) {
    tmm_status st = check_data(pl, a, dtype, "tmm_ragged_run");
    if (st != TMM_OK) return st;
    if (pl->n_units[0] == 0) return ok();
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int di = shape_slot(a, dtype);
    (void)hipGetLastError();
    if (dtype == TMM_F64) {
        const auto p = make_params<double>(pl, a);
        if (!pl->tuned[di]) return tune<double>(pl, p, di, s);
        if (launch<double>(pl, p, pl->shape[di], s) != hipSuccess) return tmm::check_launch("tmm_ragged_run");
    } else {
        const auto p = make_params<float>(pl, a);
        if (!pl->tuned[di]) return tune<float>(pl, p, di, s);
        if (launch<float>(pl, p, pl->shape[di], s) != hipSuccess) return tmm::check_launch("tmm_ragged_run");
    }
    return tmm::check_launch("tmm_ragged_run");
}

tmm_status tmm_rt_ragged(tmm_ragged_plan* pl, const tmm_ragged_data* a, tmm_dtype dtype, void* stream) {
    return tmm_ragged_run(pl, a, dtype, stream);
}

tmm_status tmm_ragged_plan_shape(const tmm_ragged_plan* pl, tmm_dtype dtype, int32_t* host_shape) {
    if (!pl || !host_shape) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_shape: NULL argument");
    if (dtype != TMM_F64 && dtype != TMM_F32) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_shape: unknown dtype");
    const int di = dtype == TMM_F64 ? 0 : 1;
    if (!pl->tuned[di]) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_shape: not tuned for this dtype yet");
    const tmm::ragged::Shape& sh = pl->shape[di];
    host_shape[0] = sh.blocks_per_cu;
    host_shape[1] = sh.grain;
    host_shape[2] = sh.waves;
    host_shape[3] = sh.lpp;
    return ok();
}

tmm_status tmm_ragged_plan_set_shape(tmm_ragged_plan* pl, tmm_dtype dtype, const int32_t* host_shape) {
    if (!pl || !host_shape) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_set_shape: NULL argument");
    if (dtype != TMM_F64 && dtype != TMM_F32)
        return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_plan_set_shape: unknown dtype");
    const int bpc = host_shape[0], grain = host_shape[1], waves = host_shape[2], lpp = host_shape[3];
    const int max_waves = dtype == TMM_F64 ? tmm::ragged::Occupancy<double>::kWavesPerCU
                                           : tmm::ragged::Occupancy<float>::kWavesPerCU;
    if (bpc < 1 || grain < 1 || grain > 64 || waves < 1 || waves > max_waves || (lpp != 1 && lpp != 2 && lpp != 4) ||
        bpc * waves > 32)
        return fail(TMM_ERR_INVALID_ARG,
                    "tmm_ragged_plan_set_shape: need workgroups per CU >= 1, 1 <= grain <= 64, 1 <= waves <= %d "
                    "for this dtype, lanes per point 1, 2 or 4, and at most 32 waves per CU", max_waves);
    const int di = dtype == TMM_F64 ? 0 : 1;
    pl->shape[di] = {bpc, grain, waves, lpp};
    pl->tuned[di] = true;
    return ok();
}

tmm_status tmm_ragged_capture(tmm_ragged_plan* pl, const tmm_ragged_data* a, tmm_dtype dtype, void* stream) {
    tmm_status st = check_data(pl, a, dtype, "tmm_ragged_capture");
    if (st != TMM_OK) return st;
    if (!stream) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_capture: needs a non-default stream");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int di = shape_slot(a, dtype);
    if (!pl->tuned[di]) {
        st = tmm_ragged_run(pl, a, dtype, stream);  // tunes (and computes the outputs once)
        if (st != TMM_OK) return st;
        if (hipStreamSynchronize(s) != hipSuccess) return fail(TMM_ERR_HIP, "tmm_ragged_capture: sync failed");
    }
    if (pl->graph_exec) {
        (void)hipGraphExecDestroy(pl->graph_exec);
        pl->graph_exec = nullptr;
    }
    if (pl->graph) {
        (void)hipGraphDestroy(pl->graph);
        pl->graph = nullptr;
    }
    if (pl->n_units[0] == 0) return ok();
    (void)hipGetLastError();
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(TMM_ERR_HIP, "tmm_ragged_capture: begin capture failed");
    hipError_t e;
    if (dtype == TMM_F64)
        e = launch<double>(pl, make_params<double>(pl, a), pl->shape[di], s);
    else
        e = launch<float>(pl, make_params<float>(pl, a), pl->shape[di], s);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return fail(TMM_ERR_HIP, "tmm_ragged_capture: capture failed");
    }
    if (hipGraphInstantiate(&pl->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(TMM_ERR_HIP, "tmm_ragged_capture: instantiate failed");
    }
    pl->graph = g;
    return ok();
}

tmm_status tmm_ragged_replay(tmm_ragged_plan* pl, void* stream) {
    if (!pl) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_replay: plan is NULL");
    if (pl->n_units[0] == 0) return ok();
    if (!pl->graph_exec) return fail(TMM_ERR_INVALID_ARG, "tmm_ragged_replay: nothing captured");
    if (hipGraphLaunch(pl->graph_exec, static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(TMM_ERR_HIP, "tmm_ragged_replay: graph launch failed");
    return ok();
}

}  // extern "C"
