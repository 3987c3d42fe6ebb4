// The per-lane layer recursion shared by the forward kernels (dense and
// ragged): state, step, renormalisation and extraction of r, t, R, T.
// The algebra is described in tmm_device.hpp.
#pragma once

#include "tmm_device.hpp"

namespace tmm {

// Renormalisation period of the layer loop (steps).  Per-step growth of the
// state is bounded by 2(|alpha| + |beta|); 16 double steps or 4 float steps
// stay far from overflow for any physical index.
template <typename R> struct RenormPeriod;
template <> struct RenormPeriod<double> { static constexpr int value = 16; };
template <> struct RenormPeriod<float> { static constexpr int value = 4; };

// ---------------------------------------------------------------------------
// The layer recursion (see tmm_device.hpp).
template <typename R, int POL, bool AMP>
struct Chain {
    static constexpr bool kRatio = false;
    static constexpr double kSLog2 = kNegPiLog2e;  // S times this is log2 of the attenuation
    __device__ __forceinline__ static double exp2_ext(double y) { return exp2_d<true>(y); }
    cx<R> ss, ts, sp, tp;  // sigma, tau of s and p
    int es, ep;            // power-of-two exponents taken out of (ss, ts), (sp, tp)
    R pis, pip;            // prod |q_j|^2, prod |eta_j|^2 (R, T only)
    int epis, epip;
    cx<R> Pq, Pe;          // prod q_j, prod eta_j (amplitudes wanted)
    int ePq, ePe;
    double S;              // sum Im(phi_j)
    double F;              // sum Re(phi_j), reduced modulo 4 (amplitudes wanted)

    __device__ __forceinline__ void init() {
        ss = ts = sp = tp = {(R)1, (R)0};
        es = ep = 0;
        pis = pip = (R)1;
        epis = epip = 0;
        Pq = Pe = {(R)1, (R)0};
        ePq = ePe = 0;
        S = 0.0;
        F = 0.0;
    }

    __device__ __forceinline__ void step(const Layer<R>& cur, const Layer<R>& nxt, double cd, bool lossy,
                                         const TabPhase<R>& phase) {
        const double phr = cd * cur.pr;
        const double phi = cd * cur.pi;
        const cx<R> E = phase(phr, phi, lossy);
        if (POL & 1) {
            const cx<R> A = cmul(cur.q, ss), Bv = cmul(nxt.q, ts);
            const cx<R> a = cadd(A, Bv), b = csub(A, Bv);
            const cx<R> Eb = cmul(E, b);
            ss = cadd(a, Eb);
            ts = csub(a, Eb);
        }
        if (POL & 2) {
            const cx<R> A = cmul(nxt.e, sp), Bv = cmul(cur.e, tp);
            const cx<R> a = cadd(A, Bv), b = csub(A, Bv);
            const cx<R> Eb = cmul(E, b);
            sp = cadd(a, Eb);
            tp = csub(a, Eb);
        }
        if (AMP) {
            if (POL & 1) Pq = cmul(Pq, cur.q);
            if (POL & 2) Pe = cmul(Pe, cur.e);
            S += phi;
            F = reduce4(F + phr);
        } else {
            if (POL & 1) pis *= cur.q2;
            if (POL & 2) pip *= cur.e2;
            S += phi;  // exactly 0 for a lossless row (Im q = 0 in every lane)
        }
    }

    // The same step when the caller knows (wave-uniformly) that the current
    // medium (CR) and / or the next one (NR) is lossless and propagating in
    // every lane: Im q = Im eta = 0, so their products with the state are real
    // scalings, |q|^2 = (Re q)^2 and the step adds nothing to S.  The results
    // are those of step() (the dropped terms are exact zeros).
    template <bool CR, bool NR>
    __device__ __forceinline__ void step_known(const Layer<R>& cur, const Layer<R>& nxt, double cd,
                                               const TabPhase<R>& phase) {
        const double phr = cd * cur.pr;
        const double phi = CR ? 0.0 : cd * cur.pi;
        const cx<R> E = phase(phr, phi, !CR);
        if (POL & 1) {
            const cx<R> A = CR ? cscale(cur.q.re, ss) : cmul(cur.q, ss);
            const cx<R> Bv = NR ? cscale(nxt.q.re, ts) : cmul(nxt.q, ts);
            const cx<R> a = cadd(A, Bv), b = csub(A, Bv);
            const cx<R> Eb = cmul(E, b);
            ss = cadd(a, Eb);
            ts = csub(a, Eb);
        }
        if (POL & 2) {
            const cx<R> A = NR ? cscale(nxt.e.re, sp) : cmul(nxt.e, sp);
            const cx<R> Bv = CR ? cscale(cur.e.re, tp) : cmul(cur.e, tp);
            const cx<R> a = cadd(A, Bv), b = csub(A, Bv);
            const cx<R> Eb = cmul(E, b);
            sp = cadd(a, Eb);
            tp = csub(a, Eb);
        }
        static_assert(!AMP, "amplitude chains use step()");
        if (POL & 1) pis *= CR ? cur.q.re * cur.q.re : cur.q2;
        if (POL & 2) pip *= CR ? cur.e.re * cur.e.re : cur.e2;
        if (!CR) S += phi;
    }

    __device__ __forceinline__ void renorm() {
        if (POL & 1) renorm_pair(ss, ts, es);
        if (POL & 2) renorm_pair(sp, tp, ep);
        if (AMP) {
            if (POL & 1) renorm_cx(Pq, ePq);
            if (POL & 2) renorm_cx(Pe, ePe);
        } else {
            if (POL & 1) renorm_one(pis, epis);
            if (POL & 2) renorm_one(pip, epip);
        }
    }
};

// ---------------------------------------------------------------------------
// Ratio form of the recursion.  Step j divided by q_j (s) or eta_j (p):
//   s: a = sigma + rho_s tau,   b = sigma - rho_s tau,   rho_s = q_{j+1} / q_j
//   p: a = rho_p sigma + tau,   b = rho_p sigma - tau,   rho_p = eta_{j+1} / eta_j
//   sigma <- a + E_j b,  tau <- a - E_j b.
// The state is the division-free one divided by prod q_j (s) or prod eta_j (p)
// over the finite layers, which are exactly the products that T and t carry,
// so they drop out of the extraction (prod = 1).  The ratios depend only on the
// pair (material j, material j + 1) and the lane, so a workgroup tabulates
// them once; per step that saves two complex products and the two running
// products of the division-free form.  Per-step growth is bounded by
// 2 (1 + |rho|); with |rho| <= kPairRatioMax (checked when the table is built)
// 32 double steps or 8 float steps stay far from overflow (kPairRatioMax is in
// tmm_device.hpp).
template <typename R> struct PairRenormPeriod;
template <> struct PairRenormPeriod<double> { static constexpr int value = 32; };
template <> struct PairRenormPeriod<float> { static constexpr int value = 8; };

template <typename R, int POL, bool AMP>
struct PairChain {
    static constexpr bool kRatio = true;
    static constexpr double kSLog2 = 1.0;
    __device__ __forceinline__ static double exp2_ext(double y) { return exp2_d<true>(y); }
    cx<R> ss, ts, sp, tp;
    int es, ep;
    double S;  // sum of y_j = -pi Im(phi_j) / ln 2: log2 of the attenuation
    double F;  // sum 256 Re(phi_j), reduced modulo 1024 (amplitudes wanted)

    __device__ __forceinline__ void init() {
        ss = ts = sp = tp = {(R)1, (R)0};
        es = ep = 0;
        S = 0.0;
        F = 0.0;
    }

    // rs, rp: the pair's ratios; (cre, cim): phi_j = d (cre / 256 + i cim / kNegPiLog2e),
    // i.e. cre is in units of 1/256 half-turn per unit d and cim is already the
    // base-2 exponent of the attenuation per unit d.  d cre < kScFastRange.
    __device__ __forceinline__ void step(cx<R> rs, cx<R> rp, double cre, double cim, double d, bool lossy,
                                         const TabPhase<R>& phase) {
        const double g = d * cre;
        cx<R> E = phase.cis_g(g);
        if (lossy) {
            const double y = d * cim;
            S += y;
            const R att = phase.atten(y);
            E.re *= att;
            E.im *= att;
        }
        if (AMP) F = reduce1024(F + g);
        update(rs, rp, E);
    }

    // The ratio-form update of the state for the step's ratios and phase factor.
    __device__ __forceinline__ void update(cx<R> rs, cx<R> rp, const cx<R>& E) {
        if (POL & 1) {
            const cx<R> X = cmul(rs, ts);
            const cx<R> a = cadd(ss, X), b = csub(ss, X);
            const cx<R> Eb = cmul(E, b);
            ss = cadd(a, Eb);
            ts = csub(a, Eb);
        }
        if (POL & 2) {
            const cx<R> X = cmul(rp, sp);
            const cx<R> a = cadd(X, tp), b = csub(X, tp);
            const cx<R> Eb = cmul(E, b);
            sp = cadd(a, Eb);
            tp = csub(a, Eb);
        }
    }

    // The same step in float with the phase coefficient as a float pair
    // (c_hi + c_lo, per unit d) and a float thickness: the phase d c is formed
    // as an exact float pair (d c_hi and its FMA error, plus d c_lo) and reduced
    // in float (|d c_hi| < 2^21); R and T only (the phase sum F is not kept).
    __device__ __forceinline__ void step_ff(cx<R> rs, cx<R> rp, float c_hi, float c_lo, float cim, float d,
                                            bool lossy, const TabPhase<R>& phase) {
#pragma clang fp contract(off)  // hi must stay the rounded product its FMA error term refers to
        static_assert(sizeof(R) == 4 && !AMP, "float pair phase: float R and T only");
        const float hi = d * c_hi;
        const float lo = __builtin_fmaf(d, c_lo, __builtin_fmaf(d, c_hi, -hi));
        cx<R> E = phase.cis_ff(hi, lo);
        if (lossy) {
            const float y = d * cim;
            S += (double)y;
            const R att = phase.atten_f(y);
            E.re *= att;
            E.im *= att;
        }
        update(rs, rp, E);
    }

    __device__ __forceinline__ void renorm() {
        if (POL & 1) renorm_pair(ss, ts, es);
        if (POL & 2) renorm_pair(sp, tp, ep);
    }
};

struct PointOut {
    double R, T;
    cx<double> r, t;
};

// Ambient step (j = 0, no phase) and extraction of r, t, R, T (Eq. (3), (7)).
// C is Chain (division-free) or PairChain (ratio form: the products are 1);
// C::kSLog2 turns its S into the base-2 exponent of the attenuation, and
// C::exp2_ext is the 2^y the extraction uses.
template <typename R, int POL, bool AMP, class C>
__device__ __forceinline__ void finish(const C& c, const Ambient& amb,
                                       const Layer<R>& first, const Layer<R>& sub,
                                       double nsub_r, double nsub_i, int L, PointOut* out,
                                       const TabPhase<R>& phase) {
    const double ly = c.S * C::kSLog2;
    const double Fh = C::kRatio ? c.F * (1.0 / kScSteps) : c.F;  // half-turns
    // the layer loop's own 2^y and table sin/cos (their constants are already
    // resident; library versions would add their own per stack)
    const double eS = C::exp2_ext(ly);
    const int two_L1 = 2 * (L + 1);
    if (POL & 1) {
        const cx<double> q0 = {amb.q0r, amb.q0i};
        const cx<double> q1 = {first.pr, first.pi};
        const cx<double> A = cmul(q0, widen(c.ss)), Bv = cmul(q1, widen(c.ts));
        const cx<double> a = cadd(A, Bv), b = csub(A, Bv);
        const double na = cnorm(a);
        PointOut& o = out[0];
        const double ina = 1.0 / na;  // one division serves R and T
        o.R = cnorm(b) * ina;
        double prod = 1.0;
        int eprod = 0;
        cx<double> Pq = {1.0, 0.0};
        int ePq = 0;
        if constexpr (!C::kRatio) {
            if (AMP) {
                Pq = widen(c.Pq);
                ePq = c.ePq;
                prod = cnorm(Pq);
                eprod = 2 * ePq;
            } else {
                prod = (double)c.pis;
                eprod = c.epis;
            }
        }
        o.T = ldexp(amb.Ks * prod * sub.pr * eS * ina, two_L1 + eprod - 2 * c.es);
        if (AMP) {
            o.r = cdiv(b, a);
            const cx<R> rot = phase.cis_g(sc_exact_g(0.5 * Fh));
            const double cs = (double)rot.re, sn = (double)rot.im;
            const double m = C::exp2_ext(0.5 * ly);
            const cx<double> ph = {m * cs, m * sn};
            cx<double> num = cmul(cmul(q0, Pq), ph);
            cx<double> tt = cdiv(num, a);
            const int e = (L + 1) + ePq - c.es;
            o.t = {ldexp(tt.re, e), ldexp(tt.im, e)};
        }
    }
    if (POL & 2) {
        const cx<double> e0 = {amb.e0r, amb.e0i};
        const cx<double> e1 = widen(first.e);
        const cx<double> A = cmul(e1, widen(c.sp)), Bv = cmul(e0, widen(c.tp));
        const cx<double> a = cadd(A, Bv), b = csub(A, Bv);
        const double na = cnorm(a);
        PointOut& o = out[(POL & 1) ? 1 : 0];
        const double ina = 1.0 / na;  // one division serves R and T
        o.R = cnorm(b) * ina;
        double prod = 1.0;
        int eprod = 0;
        cx<double> Pe = {1.0, 0.0};
        int ePe = 0;
        if constexpr (!C::kRatio) {
            if (AMP) {
                Pe = widen(c.Pe);
                ePe = c.ePe;
                prod = cnorm(Pe);
                eprod = 2 * ePe;
            } else {
                prod = (double)c.pip;
                eprod = c.epip;
            }
        }
        o.T = ldexp(amb.Kp * prod * (double)sub.e.re * eS * ina, two_L1 + eprod - 2 * c.ep);
        if (AMP) {
            o.r = cdiv(b, a);
            const cx<R> rot = phase.cis_g(sc_exact_g(0.5 * Fh));
            const double cs = (double)rot.re, sn = (double)rot.im;
            const double m = C::exp2_ext(0.5 * ly);
            const cx<double> ph = {m * cs, m * sn};
            // P_p = 2^{L+1} n_0 n_sub / q_sub prod eta_j
            const cx<double> n0 = {amb.n0r, amb.n0i};
            const cx<double> nsub = {nsub_r, nsub_i};
            const cx<double> qsub = {sub.pr, sub.pi};
            const cx<double> num = cmul(cmul(cdiv(cmul(n0, nsub), qsub), Pe), ph);
            const cx<double> tt = cdiv(num, a);
            const int e = (L + 1) + ePe - c.ep;
            o.t = {ldexp(tt.re, e), ldexp(tt.im, e)};
        }
    }
}

// ---------------------------------------------------------------------------
// Media table in LDS, structure-of-arrays, one entry per (material, lane).
template <typename R> struct Table;

// Layout: one block per material, arrays of that material one after another,
// so that a single address (block + lane) reaches every array through the
// immediate offset of the LDS read.
template <>
struct Table<double> {
    static constexpr int kEntryBytes = 48;               // per (material, lane)
    static constexpr int kBlockBytes = kWave * kEntryBytes;
    unsigned char* base;
    __device__ Table(unsigned char* b, int) : base(b) {}
    __device__ __forceinline__ void put(int m, int lane, const Medium& md) {
        double2* blk = reinterpret_cast<double2*>(base + m * kBlockBytes);
        blk[lane] = make_double2(md.qr, md.qi);
        blk[kWave + lane] = make_double2(md.er, md.ei);
        blk[2 * kWave + lane] = make_double2(md.q2, md.e2);
    }
    __device__ __forceinline__ Layer<double> get(int m, int lane) const {
        const double2* blk = reinterpret_cast<const double2*>(base + m * kBlockBytes) + lane;
        const double2 a = blk[0], b = blk[kWave], c = blk[2 * kWave];
        Layer<double> v;
        v.q = {a.x, a.y};
        v.e = {b.x, b.y};
        v.q2 = c.x;
        v.e2 = c.y;
        v.pr = a.x;
        v.pi = a.y;
        return v;
    }
};

template <>
struct Table<float> {
    static constexpr int kEntryBytes = 40;
    static constexpr int kBlockBytes = kWave * kEntryBytes;
    unsigned char* base;
    __device__ Table(unsigned char* b, int) : base(b) {}
    __device__ __forceinline__ void put(int m, int lane, const Medium& md) {
        unsigned char* blk = base + m * kBlockBytes;
        reinterpret_cast<double2*>(blk)[lane] = make_double2(md.qr, md.qi);
        float2* f = reinterpret_cast<float2*>(blk + kWave * 16);
        f[lane] = make_float2((float)md.qr, (float)md.qi);
        f[kWave + lane] = make_float2((float)md.er, (float)md.ei);
        f[2 * kWave + lane] = make_float2((float)md.q2, (float)md.e2);
    }
    __device__ __forceinline__ Layer<float> get(int m, int lane) const {
        const unsigned char* blk = base + m * kBlockBytes;
        const double2 p = reinterpret_cast<const double2*>(blk)[lane];
        const float2* f = reinterpret_cast<const float2*>(blk + kWave * 16) + lane;
        const float2 a = f[0], b = f[kWave], c = f[2 * kWave];
        Layer<float> v;
        v.q = {a.x, a.y};
        v.e = {b.x, b.y};
        v.q2 = c.x;
        v.e2 = c.y;
        v.pr = p.x;
        v.pi = p.y;
        return v;
    }
};

}  // namespace tmm
