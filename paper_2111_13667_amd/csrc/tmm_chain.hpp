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

struct PointOut {
    double R, T;
    cx<double> r, t;
};

// Ambient step (j = 0, no phase) and extraction of r, t, R, T (Eq. (3), (7)).
template <typename R, int POL, bool AMP>
__device__ __forceinline__ void finish(const Chain<R, POL, AMP>& c, const Ambient& amb,
                                       const Layer<R>& first, const Layer<R>& sub,
                                       double nsub_r, double nsub_i, int L, PointOut* out) {
    const double eS = exp2(c.S * kNegPiLog2e);
    const int two_L1 = 2 * (L + 1);
    if (POL & 1) {
        const cx<double> q0 = {amb.q0r, amb.q0i};
        const cx<double> q1 = {first.pr, first.pi};
        const cx<double> A = cmul(q0, widen(c.ss)), Bv = cmul(q1, widen(c.ts));
        const cx<double> a = cadd(A, Bv), b = csub(A, Bv);
        const double na = cnorm(a);
        PointOut& o = out[0];
        o.R = cnorm(b) / na;
        double prod;
        int eprod;
        if (AMP) {
            prod = cnorm(widen(c.Pq));
            eprod = 2 * c.ePq;
        } else {
            prod = (double)c.pis;
            eprod = c.epis;
        }
        o.T = ldexp(amb.Ks * prod * sub.pr * eS / na, two_L1 + eprod - 2 * c.es);
        if (AMP) {
            o.r = cdiv(b, a);
            double sn, cs;
            sincospi(0.5 * c.F, &sn, &cs);
            const double m = exp2(0.5 * c.S * kNegPiLog2e);
            const cx<double> ph = {m * cs, m * sn};
            cx<double> num = cmul(cmul(q0, widen(c.Pq)), ph);
            cx<double> tt = cdiv(num, a);
            const int e = (L + 1) + c.ePq - c.es;
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
        o.R = cnorm(b) / na;
        double prod;
        int eprod;
        if (AMP) {
            prod = cnorm(widen(c.Pe));
            eprod = 2 * c.ePe;
        } else {
            prod = (double)c.pip;
            eprod = c.epip;
        }
        o.T = ldexp(amb.Kp * prod * (double)sub.e.re * eS / na, two_L1 + eprod - 2 * c.ep);
        if (AMP) {
            o.r = cdiv(b, a);
            double sn, cs;
            sincospi(0.5 * c.F, &sn, &cs);
            const double m = exp2(0.5 * c.S * kNegPiLog2e);
            const cx<double> ph = {m * cs, m * sn};
            // P_p = 2^{L+1} n_0 n_sub / q_sub prod eta_j
            const cx<double> n0 = {amb.n0r, amb.n0i};
            const cx<double> nsub = {nsub_r, nsub_i};
            const cx<double> qsub = {sub.pr, sub.pi};
            const cx<double> num = cmul(cmul(cdiv(cmul(n0, nsub), qsub), widen(c.Pe)), ph);
            const cx<double> tt = cdiv(num, a);
            const int e = (L + 1) + c.ePe - c.ep;
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
