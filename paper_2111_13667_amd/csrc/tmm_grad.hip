// Adjoint (reverse-mode) gradients of R and T w.r.t. layer thicknesses and
// layer refractive indices (gfx950, float64) and the tmm_rt_grad entry point.
//
// The paper differentiates its transfer-matrix graph with PyTorch autograd
// (section "TMM-Torch"); here the reverse sweep is written by hand for the
// division-free recursion of tmm_device.hpp.  Per lane = one (stack, lambda,
// theta) with both polarisations:
//
//   pass A  forward from the substrate to the ambient, storing the (s, p)
//           state every kSeg layers (after a power-of-two renormalisation) in
//           a per-wave workspace slot; at the ambient form R, T and the output
//           adjoints from the upstream gradients dl/dR, dl/dT.
//   pass B  segments from the ambient back to the substrate: reload the
//           segment's checkpoint, recompute its kSeg steps keeping the inputs
//           in registers, then run the adjoint of each step (layer j
//           ascending) and form the lane's share of dl/dd_j and dl/dn_j.  The
//           3 kSeg shares of a segment go through a per-wave LDS transpose and
//           are summed over the wave's 64 wavelengths; one partial sum per
//           (column, stack, layer) goes to the workspace, where column =
//           (wavelength tile, angle).
//   reduce  a second kernel sums the partials over the columns in a fixed
//           order, so the gradients are the same bits on every run.
//
// Launch: persistent blocks of four waves walk a static range of tasks
// (column, group of four stacks); the block keeps an LDS table of the index
// table's rows at its column (q, eta and the per-material adjoint factors)
// and rebuilds it when the column or the ambient row changes.
//
// Adjoint conventions: for a complex intermediate z the adjoint is
// zb = dl/dRe z + i dl/dIm z, so w = c z gives zb = conj(c) wb.  Per step
// (a = alpha s + beta t, b = alpha s - beta t, s' = a + E b, t' = a - E b):
//   ab = sb' + tb',  X = sb' - tb',  bb = conj(E) X,  Eb += conj(b) X,
//   Ab = ab + bb,  Bb = ab - bb,  sb = conj(alpha) Ab,  tb = conj(beta) Bb,
//   alphab = conj(s) Ab,  betab = conj(t) Bb.
// With E = e^{2 i delta}: deltab = -2i conj(E) Eb; T also carries
// e^{-2 Im sum delta} (deltab += -2i gT T) and prod w_j (w = |q|^2 or |eta|^2:
// wb = gT T / w, qb += 2 q wb).  delta_j = 2 pi d_j q_j / lambda gives
// db_j = 2 pi / lambda Re(conj(deltab) q_j) and qb_j += 2 pi d_j / lambda deltab;
// finally nb_j = conj(n/q) qb_j + conj((n/q)(2 - eta/q)) etab_j since
// dq/dn = n/q and d(eta)/dn = (n/q)(2 - eta/q).
#include <limits.h>
#include <math.h>

#include <map>
#include <mutex>
#include <type_traits>

#include "tmm_check.hpp"
#include "tmm_device.hpp"
#include "tmm_host.hpp"

namespace tmm {

constexpr int kGradBlock = 256;
constexpr int kGradWaves = kGradBlock / kWave;
constexpr int kSeg = 3;                  // layers per checkpoint segment (the ratio-form kernel
                                         // takes its own SEG: 5 for tables of at most four rows)
constexpr int kRed = 3 * kSeg;           // shares per segment: dl/dd, dl/dRe n, dl/dIm n per layer
constexpr int kGradMaxTableMat = 16;
constexpr int kTabFields = 6;            // q, eta, n/q, (n/q)(2 - eta/q), 2q/|q|^2, 2 eta/|eta|^2
constexpr int kCkptDoubles = 8;          // (sigma, tau) of s and p, complex
constexpr int kGradMaxBlocks = 1024;     // persistent grid bound (and checkpoint slots)
constexpr size_t kPartialCap = (size_t)1 << 29;  // partial-sum bytes of the preferred workspace

struct GradParams {
    int B, L, n_wl, n_theta;
    const double* d;
    const double* nk;
    int n_mat, dispersive;
    const int32_t* mat;
    const double* wl;
    const double* sin_t;
    const double* cos_t;
    const double* gR;
    const double* gT;
    double* R_out;
    double* T_out;
    double* ws;        // checkpoints: [block][wave][n_seg + 1][kCkptDoubles][kWave]
    double* partial;   // [column][stack - b_begin][L][3]
    int b_begin, b_end;
    int n_tiles, n_seg;  // n_seg: segments of kSeg layers (division-free adjoint, and the
                         // checkpoint stride of every kernel)
    int n_seg_pair;      // segments of the ratio-form kernel's own length SEG
    int64_t n_tasks;   // columns * ceil((b_end - b_begin) / waves per block)
    int64_t n_tasks_pair;  // the same for the ratio-form kernel's blocks
    int64_t per_block;
    int64_t slots;     // checkpoint slots in the workspace (waves of the persistent grid)
    unsigned char* redo;  // [column][stack - b_begin]: 1 = left to the checkpointing kernels by
                          // the inverse-walk kernel (NULL: every stack is processed)
};

// Per-stack layer data is read-only during the launch and read at
// wave-uniform indices: through these pointers it is fetched with scalar loads
// and the row arithmetic stays on the scalar unit.
typedef const __attribute__((address_space(4))) double* cdptr;
typedef const __attribute__((address_space(4))) int32_t* ciptr;

// Forward values of a medium: q and eta.
struct FL {
    cx<double> q, e;
};
// Adjoint factors of a medium (see the header comment).
struct AL {
    cx<double> nq, de, wq, we;
};

__device__ __forceinline__ FL fl_from(const Medium& m) { return FL{{m.qr, m.qi}, {m.er, m.ei}}; }

__device__ __forceinline__ AL al_from(double nr, double ni, const FL& f) {
    const double iq2 = 1.0 / cnorm(f.q);
    const cx<double> nq = {(nr * f.q.re + ni * f.q.im) * iq2, (ni * f.q.re - nr * f.q.im) * iq2};
    const cx<double> eq = {(f.e.re * f.q.re + f.e.im * f.q.im) * iq2, (f.e.im * f.q.re - f.e.re * f.q.im) * iq2};
    AL a;
    a.nq = nq;
    a.de = cmul(nq, cx<double>{2.0 - eq.re, -eq.im});
    a.wq = cscale(2.0 * iq2, f.q);
    a.we = cscale(2.0 / cnorm(f.e), f.e);
    return a;
}

// Media from the block's LDS table (material ids, at most kGradMaxTableMat rows);
// thicknesses and rows by scalar loads.
struct TabSrc {
    const double2* tab;   // this lane's entries: tab[(m * kTabFields + f) * kWave]
    ciptr mrow;  // the stack's rows [L + 2]
    cdptr drow;  // the stack's thicknesses [L]
    int n_mat;
    __device__ __forceinline__ double d(int j) const { return drow[j - 1]; }
    __device__ __forceinline__ int row(int j) const {
        const int m = mrow[j];
        return m < 0 ? 0 : (m >= n_mat ? n_mat - 1 : m);
    }
    __device__ __forceinline__ FL fwd(int j) const {
        const double2* e = tab + row(j) * kTabFields * kWave;
        const double2 a = e[0], b = e[kWave];
        return FL{{a.x, a.y}, {b.x, b.y}};
    }
    __device__ __forceinline__ AL adj(int j, const FL&) const {
        const double2* e = tab + row(j) * kTabFields * kWave;
        const double2 a = e[2 * kWave], b = e[3 * kWave], c = e[4 * kWave], d = e[5 * kWave];
        return AL{{a.x, a.y}, {b.x, b.y}, {c.x, c.y}, {d.x, d.y}};
    }
};

// Same table, with the stack's thicknesses and rows held one per lane
// (L + 2 <= 64) and broadcast by readlane: no memory access per layer.
struct TabRegSrc {
    const double2* tab;
    double my_d;  // lane l: thickness of layer l + 1
    int my_row;   // lane l: table row of medium l, clamped to the table
    __device__ __forceinline__ double d(int j) const {
        return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(my_d), j - 1),
                                __builtin_amdgcn_readlane(__double2loint(my_d), j - 1));
    }
    __device__ __forceinline__ int row(int j) const { return __builtin_amdgcn_readlane(my_row, j); }
    __device__ __forceinline__ FL fwd(int j) const {
        const double2* e = tab + row(j) * kTabFields * kWave;
        const double2 a = e[0], b = e[kWave];
        return FL{{a.x, a.y}, {b.x, b.y}};
    }
    __device__ __forceinline__ AL adj(int j, const FL&) const {
        const double2* e = tab + row(j) * kTabFields * kWave;
        const double2 a = e[2 * kWave], b = e[3 * kWave], c = e[4 * kWave], d = e[5 * kWave];
        return AL{{a.x, a.y}, {b.x, b.y}, {c.x, c.y}, {d.x, d.y}};
    }
};

// Media computed in place (per-layer rows, or tables too large for LDS).
struct InlSrc {
    const double* nk;
    cdptr drow;  // the stack's thicknesses [L]
    ciptr mrow;  // NULL: implicit rows base + j
    int64_t base;
    int n_mat, dispersive, n_wl, i;
    double kx;
    __device__ __forceinline__ double d(int j) const { return drow[j - 1]; }
    __device__ __forceinline__ int64_t row(int j) const {
        if (!mrow) return base + j;
        const int m = mrow[j];
        return m < 0 ? 0 : (m >= n_mat ? n_mat - 1 : m);
    }
    __device__ __forceinline__ FL fwd(int j) const {
        double nr, ni;
        load_n(nk, dispersive, n_wl, row(j), i, nr, ni);
        return fl_from(make_medium(nr, ni, kx));
    }
    __device__ __forceinline__ AL adj(int j, const FL& f) const {
        double nr, ni;
        load_n(nk, dispersive, n_wl, row(j), i, nr, ni);
        return al_from(nr, ni, f);
    }
};

struct State {
    cx<double> ss, ts, sp, tp;
};

template <int POL>
__device__ __forceinline__ void fwd_step(State& z, const FL& cur, const FL& nxt, const cx<double>& E) {
    if (POL & 1) {
        const cx<double> A = cmul(cur.q, z.ss), Bv = cmul(nxt.q, z.ts);
        const cx<double> a = cadd(A, Bv), b = csub(A, Bv);
        const cx<double> Eb = cmul(E, b);
        z.ss = cadd(a, Eb);
        z.ts = csub(a, Eb);
    }
    if (POL & 2) {
        const cx<double> A = cmul(nxt.e, z.sp), Bv = cmul(cur.e, z.tp);
        const cx<double> a = cadd(A, Bv), b = csub(A, Bv);
        const cx<double> Eb = cmul(E, b);
        z.sp = cadd(a, Eb);
        z.tp = csub(a, Eb);
    }
}

// conj(a) * b
__device__ __forceinline__ cx<double> cmulc(cx<double> a, cx<double> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

// Adjoint of one polarisation's step.  (s, t) is the step's input, (sb, tb)
// holds the adjoint of its output on entry and of its input on return.
__device__ __forceinline__ void adj_step(cx<double> s, cx<double> t, cx<double> alpha, cx<double> beta,
                                         cx<double> E, cx<double>& sb, cx<double>& tb, cx<double>& alphab,
                                         cx<double>& betab, cx<double>& Eb) {
    const cx<double> A = cmul(alpha, s), Bv = cmul(beta, t);
    const cx<double> b = csub(A, Bv);
    const cx<double> ab = cadd(sb, tb), X = csub(sb, tb);
    const cx<double> bb = cmulc(E, X);
    Eb = cadd(Eb, cmulc(b, X));
    const cx<double> Ab = cadd(ab, bb), Bb = csub(ab, bb);
    sb = cmulc(alpha, Ab);
    tb = cmulc(beta, Bb);
    alphab = cmulc(s, Ab);
    betab = cmulc(t, Bb);
}

// Exponent taken out by renorm_pair for this pair (same computation).
__device__ __forceinline__ int pair_exp(const cx<double>& a, const cx<double>& b) {
    const double m = fmax(fmax(fabs(a.re), fabs(a.im)), fmax(fabs(b.re), fabs(b.im)));
    return frexp_exp(m);
}

// v + v of the lane whose index differs in bit 0 (CTRL 0xB1) or bit 1 (0x4E),
// by DPP quad permutes; every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ double quad_add(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return v + __hiloint2double(hi, lo);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The stack's layer data is valid: finite non-negative thicknesses and row ids
// inside the index table (wave-uniform result).
__device__ __forceinline__ bool stack_bad(const GradParams& p, const double* drow, ciptr mrow, int lane) {
    bool bad = false;
    for (int j = lane; j < p.L; j += kWave) {
        bad = bad || bad_thickness(drow[j]);
        if (mrow) bad = bad || (uint32_t)mrow[j + 1] >= (uint32_t)p.n_mat;
    }
    if (mrow && lane == 0)
        bad = bad || (uint32_t)mrow[0] >= (uint32_t)p.n_mat || (uint32_t)mrow[p.L + 1] >= (uint32_t)p.n_mat;
    return __any(bad);
}

template <int POL, typename Src>
__device__ void grad_stack(const GradParams& p, const Src& src, const Ambient& amb, int b, int k, int i, int lane,
                           bool active, bool valid, double* ws, double* red, double* part,
                           const TabPhase<double>& phase) {
    const int L = p.L;
    constexpr int P = (POL == 3) ? 2 : 1;
    const double lam = p.wl[i];
    const double c4lam = 4.0 / lam;           // phi = c4lam d q (half-turns of 2 delta)
    const double two_pi_lam = 2.0 * M_PI / lam;
    auto ck = [&](int c, int comp) -> double& { return ws[((size_t)c * kCkptDoubles + comp) * kWave + lane]; };
    auto save = [&](int c, const State& z) {
        ck(c, 0) = z.ss.re; ck(c, 1) = z.ss.im; ck(c, 2) = z.ts.re; ck(c, 3) = z.ts.im;
        ck(c, 4) = z.sp.re; ck(c, 5) = z.sp.im; ck(c, 6) = z.tp.re; ck(c, 7) = z.tp.im;
    };
    auto load = [&](int c) -> State {
        State z;
        z.ss = {ck(c, 0), ck(c, 1)}; z.ts = {ck(c, 2), ck(c, 3)};
        z.sp = {ck(c, 4), ck(c, 5)}; z.tp = {ck(c, 6), ck(c, 7)};
        return z;
    };

    // ---- pass A: forward with checkpoints --------------------------------
    State z;
    z.ss = z.ts = z.sp = z.tp = {1.0, 0.0};
    int es = 0, ep = 0, epis = 0, epip = 0;
    double pis = 1.0, pip = 1.0, S = 0.0;
    save(0, z);
    const FL sub = src.fwd(L + 1);
    FL nxt = sub;
    for (int s = 0; s < p.n_seg; ++s) {
        const int top = L - s * kSeg;
        const int lo = top - kSeg + 1 > 1 ? top - kSeg + 1 : 1;
        for (int j = top; j >= lo; --j) {
            const FL cur = src.fwd(j);
            const double cd = src.d(j) * c4lam;
            const double phi = cd * cur.q.im;
            const bool lossy = __any(phi != 0.0);
            const cx<double> E = phase(cd * cur.q.re, phi, lossy);
            fwd_step<POL>(z, cur, nxt, E);
            if (POL & 1) pis *= cnorm(cur.q);
            if (POL & 2) pip *= cnorm(cur.e);
            S += phi;
            nxt = cur;
        }
        if (POL & 1) renorm_pair(z.ss, z.ts, es);
        if (POL & 2) renorm_pair(z.sp, z.tp, ep);
        if (POL & 1) renorm_one(pis, epis);
        if (POL & 2) renorm_one(pip, epip);
        save(s + 1, z);
    }
    const FL first = nxt;
    const double eS = exp2(S * kNegPiLog2e);
    const int two_L1 = 2 * (L + 1);
    const double nan = __builtin_nan("");
    const double w_act = active ? 1.0 : 0.0;  // ragged-tail lanes contribute nothing

    // ambient step and output adjoints
    cx<double> sb_s = {0, 0}, tb_s = {0, 0}, sb_p = {0, 0}, tb_p = {0, 0};
    cx<double> pend_q = {0, 0}, pend_e = {0, 0};  // qb / etab already owed to the next layer
    double cT_s = 0.0, cT_p = 0.0;
    const cx<double> q0 = {amb.q0r, amb.q0i}, e0 = {amb.e0r, amb.e0i};
    if (POL & 1) {
        const cx<double> A = cmul(q0, z.ss), Bv = cmul(first.q, z.ts);
        const cx<double> a = cadd(A, Bv), bb = csub(A, Bv);
        const double na = cnorm(a);
        const double R = cnorm(bb) / na;
        const double T = ldexp(amb.Ks * pis * sub.q.re * eS / na, two_L1 + epis - 2 * es);
        const int64_t o = (((int64_t)b * P + 0) * p.n_theta + k) * p.n_wl + i;
        if (active && p.R_out) p.R_out[o] = valid ? R : nan;
        if (active && p.T_out) p.T_out[o] = valid ? T : nan;
        const double gR = p.gR ? p.gR[o] * w_act : 0.0;
        const double gT = p.gT ? p.gT[o] * w_act : 0.0;
        cT_s = gT * T;
        const cx<double> abar = cscale(-2.0 * (gR * R + gT * T) / na, a);
        const cx<double> bbar = cscale(2.0 * gR / na, bb);
        const cx<double> Ab = cadd(abar, bbar), Bb = csub(abar, bbar);
        sb_s = cmulc(q0, Ab);
        tb_s = cmulc(first.q, Bb);
        pend_q = cmulc(z.ts, Bb);  // beta_0 = q_1
    }
    if (POL & 2) {
        const cx<double> A = cmul(first.e, z.sp), Bv = cmul(e0, z.tp);
        const cx<double> a = cadd(A, Bv), bb = csub(A, Bv);
        const double na = cnorm(a);
        const double R = cnorm(bb) / na;
        const double T = ldexp(amb.Kp * pip * sub.e.re * eS / na, two_L1 + epip - 2 * ep);
        const int64_t o = (((int64_t)b * P + (P - 1)) * p.n_theta + k) * p.n_wl + i;
        if (active && p.R_out) p.R_out[o] = valid ? R : nan;
        if (active && p.T_out) p.T_out[o] = valid ? T : nan;
        const double gR = p.gR ? p.gR[o] * w_act : 0.0;
        const double gT = p.gT ? p.gT[o] * w_act : 0.0;
        cT_p = gT * T;
        const cx<double> abar = cscale(-2.0 * (gR * R + gT * T) / na, a);
        const cx<double> bbar = cscale(2.0 * gR / na, bb);
        const cx<double> Ab = cadd(abar, bbar), Bb = csub(abar, bbar);
        sb_p = cmulc(first.e, Ab);
        tb_p = cmulc(e0, Bb);
        pend_e = cmulc(z.sp, Ab);  // alpha_0 = eta_1
    }
    const double cT = (POL & 1 ? cT_s : 0.0) + (POL & 2 ? cT_p : 0.0);
    if (!valid) {  // poison the gradients of this lane's stack
        sb_s = tb_s = sb_p = tb_p = pend_q = pend_e = {nan, nan};
    }

    // ---- pass B: segments from the ambient side ----------------------------
    const int v_red = lane >> 2 < kRed ? lane >> 2 : kRed - 1;  // share this lane sums
    const double2* red_in = reinterpret_cast<const double2*>(red + v_red * kWave + (lane & 3) * 16);
    // One segment of NST steps whose top layer is `top`: recompute from the
    // checkpoint, then the adjoint of each step (no guards: NST is exact).
    auto segment = [&](auto nst_c, int s, int top) {
        constexpr int NST = decltype(nst_c)::value;
        State zin[NST];
        cx<double> Es[NST];
        State zz = load(s);
        FL nx = sub;
        if (top != L) nx = src.fwd(top + 1);
#pragma unroll
        for (int t = 0; t < NST; ++t) {
            const int j = top - t;
            const FL cur = src.fwd(j);
            const double cd = src.d(j) * c4lam;
            const double phi = cd * cur.q.im;
            const bool lossy = __any(phi != 0.0);
            Es[t] = phase(cd * cur.q.re, phi, lossy);
            zin[t] = zz;
            fwd_step<POL>(zz, cur, nx, Es[t]);
            nx = cur;
        }
        // the forward pass renormalised the segment's end state; undo on the adjoint
        if (POL & 1) {
            const double f = ldexp(1.0, -pair_exp(zz.ss, zz.ts));
            sb_s = cscale(f, sb_s);
            tb_s = cscale(f, tb_s);
        }
        if (POL & 2) {
            const double f = ldexp(1.0, -pair_exp(zz.sp, zz.tp));
            sb_p = cscale(f, sb_p);
            tb_p = cscale(f, tb_p);
        }
        FL cur = nx;  // layer top - NST + 1
#pragma unroll
        for (int t = NST - 1; t >= 0; --t) {
            const int j = top - t;
            FL up = sub;
            if (j != L) up = src.fwd(j + 1);
            const AL ca = src.adj(j, cur);
            const double dj = src.d(j);
            cx<double> Eb = {0.0, 0.0};
            cx<double> qb = pend_q, eb = pend_e;
            if (POL & 1) {
                cx<double> alphab, betab;
                adj_step(zin[t].ss, zin[t].ts, cur.q, up.q, Es[t], sb_s, tb_s, alphab, betab, Eb);
                qb = cadd(qb, alphab);  // alpha_j = q_j
                pend_q = betab;         // beta_j = q_{j+1}
                qb = cadd(qb, cscale(cT_s, ca.wq));  // T through |q_j|^2
            }
            if (POL & 2) {
                cx<double> alphab, betab;
                adj_step(zin[t].sp, zin[t].tp, up.e, cur.e, Es[t], sb_p, tb_p, alphab, betab, Eb);
                eb = cadd(eb, betab);   // beta_j = eta_j
                pend_e = alphab;        // alpha_j = eta_{j+1}
                eb = cadd(eb, cscale(cT_p, ca.we));  // T through |eta_j|^2
            }
            // deltab = -2i conj(E) Eb - 2i cT  (chain and e^{-2 Im sum delta})
            const cx<double> cE = cmulc(Es[t], Eb);
            const cx<double> db = {2.0 * cE.im, -2.0 * cE.re - 2.0 * cT};
            const double gd = two_pi_lam * (db.re * cur.q.re + db.im * cur.q.im);
            qb = cadd(qb, cscale(two_pi_lam * dj, db));
            const cx<double> nb = cadd(cmulc(ca.nq, qb), cmulc(ca.de, eb));
            red[(3 * t + 0) * kWave + lane] = gd;
            red[(3 * t + 1) * kWave + lane] = nb.re;
            red[(3 * t + 2) * kWave + lane] = nb.im;
            cur = up;
        }
    };
    for (int s = p.n_seg - 1; s >= 0; --s) {
        const int top = L - s * kSeg;
        const int lo = top - kSeg + 1 > 1 ? top - kSeg + 1 : 1;
        const int nst = top - lo + 1;
        if (nst == kSeg) {
            segment(std::integral_constant<int, kSeg>(), s, top);
        } else {
            static_assert(kSeg <= 4, "segment lengths below are spelled out");
            if (nst == 1) segment(std::integral_constant<int, 1>(), s, top);
            if (kSeg > 2 && nst == 2) segment(std::integral_constant<int, (kSeg > 2 ? 2 : 1)>(), s, top);
            if (kSeg > 3 && nst == 3) segment(std::integral_constant<int, (kSeg > 3 ? 3 : 1)>(), s, top);
        }
        wave_sync();
        // lane 4v + c sums quarter c of share v; quad permutes finish the sums
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double2 x = red_in[u];
            acc += x.x;
            acc += x.y;
        }
        acc = quad_add<0xB1>(acc);
        acc = quad_add<0x4E>(acc);
        if ((lane & 3) == 0 && (lane >> 2) < 3 * nst) {
            const int v = lane >> 2;
            const int t = v / 3;
            part[(top - t - 1) * 3 + (v - 3 * t)] = acc;
        }
        wave_sync();
    }
}

// Fills the block's LDS table for one column and ambient row: every wave
// computes rows wave, wave + 4, ... at its lanes' wavelength.
__device__ void build_table(const GradParams& p, double2* tab, int amb_row, int i, double st, double ct, int wave,
                            int lane) {
    double n0r, n0i;
    load_n(p.nk, p.dispersive, p.n_wl, amb_row, i, n0r, n0i);
    const Ambient a = make_ambient(n0r, n0i, st, ct);
    for (int m = wave; m < p.n_mat; m += kGradWaves) {
        double nr, ni;
        load_n(p.nk, p.dispersive, p.n_wl, m, i, nr, ni);
        const FL f = fl_from(make_medium(nr, ni, a.kx));
        const AL g = al_from(nr, ni, f);
        double2* e = tab + m * kTabFields * kWave + lane;
        e[0] = make_double2(f.q.re, f.q.im);
        e[kWave] = make_double2(f.e.re, f.e.im);
        e[2 * kWave] = make_double2(g.nq.re, g.nq.im);
        e[3 * kWave] = make_double2(g.de.re, g.de.im);
        e[4 * kWave] = make_double2(g.wq.re, g.wq.im);
        e[5 * kWave] = make_double2(g.we.re, g.we.im);
    }
}

// Task t = (column, group of kGradWaves stacks), column = (angle k, tile).
struct Task {
    int k, tile, b;
};
__device__ __forceinline__ Task task_of(const GradParams& p, int64_t t, int wave) {
    const int64_t groups = (p.b_end - p.b_begin + kGradWaves - 1) / kGradWaves;
    const int64_t col = t / groups;
    Task r;
    r.k = (int)(col / p.n_tiles);
    r.tile = (int)(col - (int64_t)r.k * p.n_tiles);
    r.b = p.b_begin + (int)(t - col * groups) * kGradWaves + wave;
    return r;
}

template <int POL, bool TABLE>
__global__ void __launch_bounds__(kGradBlock) __attribute__((amdgpu_waves_per_eu(2))) grad_kernel(GradParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_rows[kGradWaves];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    fill_phase_tab<double>(smem, threadIdx.x, kGradBlock);
    __syncthreads();
    const TabPhase<double> phase = phase_of<double>(smem);
    unsigned char* const lds = smem + phase_tab_bytes<double>();
    double* red = reinterpret_cast<double*>(lds) + wave * kRed * kWave;
    double2* tab = reinterpret_cast<double2*>(lds + (size_t)kGradWaves * kRed * kWave * sizeof(double));
    double* ws = p.ws + ((size_t)blockIdx.x * kGradWaves + wave) * (size_t)(p.n_seg + 1) * kCkptDoubles * kWave;
    const int L2 = p.L + 2;
    const int64_t nbs = p.b_end - p.b_begin;
    const int64_t t0 = (int64_t)blockIdx.x * p.per_block;
    const int64_t t1 = t0 + p.per_block < p.n_tasks ? t0 + p.per_block : p.n_tasks;
    int64_t tab_col = -1;
    int tab_row = -1;
    for (int64_t t = t0; t < t1; ++t) {
        const Task tk = task_of(p, t, wave);
        const int i_raw = tk.tile * kWave + lane;
        const bool active = i_raw < p.n_wl;
        const int i = active ? i_raw : p.n_wl - 1;
        const double lam = p.wl[i];
        const bool lam_ok = lam > 0.0 && lam < __builtin_inf();
        const double st = p.sin_t[tk.k], ct = p.cos_t[tk.k];
        const int64_t col = (int64_t)tk.k * p.n_tiles + tk.tile;
        // after the inverse-walk kernel: only the stacks it left
        const bool has = tk.b < p.b_end &&
                         (!p.redo || p.redo[(size_t)col * nbs + (tk.b - p.b_begin)] != 0);
        if (p.redo && __syncthreads_or(has ? 1 : 0) == 0) continue;
        const int b = tk.b < p.b_end ? tk.b : p.b_end - 1;
        const ciptr mrow = p.mat ? (ciptr)(p.mat + (int64_t)b * L2) : nullptr;
        double* part = p.partial + ((size_t)col * nbs + (b - p.b_begin)) * (size_t)p.L * 3;
        const bool bad = stack_bad(p, p.d + (int64_t)b * p.L, mrow, lane);
        if (TABLE) {
            int a_row = mrow[0];
            a_row = a_row < 0 ? 0 : (a_row >= p.n_mat ? p.n_mat - 1 : a_row);
            bool done = !has;
            // one sub-round per distinct ambient row among the block's stacks
            for (;;) {
                __syncthreads();
                if (lane == 0) s_rows[wave] = done ? INT_MAX : a_row;
                __syncthreads();
                int r = s_rows[0];
                for (int w = 1; w < kGradWaves; ++w) r = min(r, s_rows[w]);
                if (r == INT_MAX) break;
                if (r != tab_row || col != tab_col) {
                    build_table(p, tab, r, i, st, ct, wave, lane);
                    tab_row = r;
                    tab_col = col;
                }
                __syncthreads();
                if (!done && a_row == r) {
                    double n0r, n0i;
                    load_n(p.nk, p.dispersive, p.n_wl, a_row, i, n0r, n0i);
                    const Ambient amb = make_ambient(n0r, n0i, st, ct);
                    const bool ok = lam_ok && amb.ok && !bad;
                    if (L2 <= kWave) {
                        TabRegSrc src;
                        src.tab = tab + lane;
                        src.my_d = lane < p.L ? p.d[(int64_t)b * p.L + lane] : 0.0;
                        const int m = lane < L2 ? p.mat[(int64_t)b * L2 + lane] : 0;
                        src.my_row = m < 0 ? 0 : (m >= p.n_mat ? p.n_mat - 1 : m);
                        grad_stack<POL>(p, src, amb, b, tk.k, i, lane, active, ok, ws, red, part, phase);
                    } else {
                        TabSrc src;
                        src.tab = tab + lane;
                        src.mrow = mrow;
                        src.drow = (cdptr)(p.d + (int64_t)b * p.L);
                        src.n_mat = p.n_mat;
                        grad_stack<POL>(p, src, amb, b, tk.k, i, lane, active, ok, ws, red, part, phase);
                    }
                    done = true;
                }
            }
        } else if (has) {
            InlSrc src;
            src.nk = p.nk;
            src.drow = (cdptr)(p.d + (int64_t)b * p.L);
            src.mrow = mrow;
            src.base = (int64_t)b * L2;
            src.n_mat = p.n_mat;
            src.dispersive = p.dispersive;
            src.n_wl = p.n_wl;
            src.i = i;
            double n0r, n0i;
            load_n(p.nk, p.dispersive, p.n_wl, src.row(0), i, n0r, n0i);
            const Ambient amb = make_ambient(n0r, n0i, st, ct);
            src.kx = amb.kx;
            grad_stack<POL>(p, src, amb, b, tk.k, i, lane, active, lam_ok && amb.ok && !bad, ws, red, part, phase);
        }
    }
}

// ---------------------------------------------------------------------------
// Ratio form (material ids, small tables, L + 2 <= 128).  The forward steps are
// those of the forward kernel's pair path: step j divided by q_j (s) or eta_j
// (p), with rho_s = q_{j+1}/q_j and rho_p = eta_{j+1}/eta_j tabulated per
// ordered material pair, and the normalisation products gone from T.
// Adjoint of one step, X = rho tau (s) or rho sigma (p):
//   s: a = s + X, b = s - X        p: a = X + t, b = X - t
//   ab = sb' + tb', Y = sb' - tb', bb = conj(E) Y, Eb += conj(b) Y,
//   s: sb = ab + bb, Xb = ab - bb, tb = conj(rho) Xb
//   p: Xb = ab + bb, tb = ab - bb, sb = conj(rho) Xb
//   rhob = conj(tau) Xb (s) or conj(sigma) Xb (p), and w = conj(rho) rhob = conj(X) Xb.
// rho_j depends on q_j as -rho/q_j and on q_{j+1} as rho/q_{j+1}, so layer j
// collects conj(1/q_j) (w_{j-1} - w_j) (w_0 = 0: the ambient step keeps the
// division-free form), and dl/dn_j takes it through (dq/dn)/q (same for eta).
constexpr int kGradPairWaves = 8;        // two per SIMD at the kernel's register count
constexpr int kGradPairBlock = kGradPairWaves * kWave;
constexpr int kGradPairMaxBlocks = kGradMaxBlocks * kGradWaves / kGradPairWaves;  // same checkpoint slots
constexpr int kGradPairMaxMat = 5;
constexpr int kGradPairLongSegMaxMat = 4;  // five-layer segments: 60 KiB of shares, 140 KiB in all at 4 rows
constexpr int kPairFields = 6;           // q, eta, dq/dn, deta/dn, (dq/dn)/q, (deta/dn)/eta
constexpr int kGradPairBlockBytes = 3 * kWave * 16;  // rho_s[64], rho_p[64], (cre, cim)[64]

__host__ __device__ constexpr size_t grad_pair_lds_bytes(int n_mat, int seg) {
    return phase_tab_bytes<double>() + (size_t)kGradPairWaves * 3 * seg * kWave * sizeof(double) +
           (size_t)n_mat * kPairFields * kWave * sizeof(double2) + (size_t)n_mat * n_mat * kGradPairBlockBytes;
}

// Per-layer values of a stack held N to a lane (lane l of register r: element
// 64 r + l), broadcast at a wave-uniform index x: one register for stacks with
// L + 2 <= 64, two for L + 2 <= 128.
template <int N>
__device__ __forceinline__ int lane_bcast(const int (&v)[N], int x) {
    if (N == 1 || x < kWave) return __builtin_amdgcn_readlane(v[0], x);
    return __builtin_amdgcn_readlane(v[N - 1], x - kWave);
}
template <int N>
__device__ __forceinline__ double lane_bcast(const double (&v)[N], int x) {
    const int r = (N == 1 || x < kWave) ? 0 : N - 1;
    const int y = r == 0 ? x : x - kWave;
    if (N == 1 || r == 0)
        return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v[0]), y),
                                __builtin_amdgcn_readlane(__double2loint(v[0]), y));
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v[N - 1]), y),
                            __builtin_amdgcn_readlane(__double2loint(v[N - 1]), y));
}

// A stack's layer data for the ratio-form kernels: lane l of register r holds
// layer 64 r + l + 1 (its thickness, and the table rows of media 64 r + l + 1
// and + 2, from which the kernel forms the layer's code) and the row of medium
// 64 r + l; rows clamped into the table.
template <int N>
__device__ __forceinline__ void load_layers(const GradParams& p, const double* drow, ciptr mrow, int lane,
                                            double (&d)[N], int (&row)[N], int (&cur)[N], int (&nxt)[N]) {
    const int L2 = p.L + 2;
    auto clamp_row = [&](int m) { return m < 0 ? 0 : (m >= p.n_mat ? p.n_mat - 1 : m); };
    if (N == 1) {
        // rows of media l and l + 1 per lane; the layer's two from the lane above
        d[0] = lane < p.L ? drow[lane] : 0.0;
        row[0] = clamp_row(lane < L2 ? mrow[lane] : 0);
        const int m_nx = clamp_row(lane + 1 < L2 ? mrow[lane + 1] : 0);
        cur[0] = __shfl_down(row[0], 1, kWave);
        nxt[0] = __shfl_down(m_nx, 1, kWave);
        return;
    }
    for (int r = 0; r < N; ++r) {
        const int l = lane + r * kWave;
        d[r] = l < p.L ? drow[l] : 0.0;
        row[r] = clamp_row(l < L2 ? mrow[l] : 0);
        cur[r] = clamp_row(l + 1 < L2 ? mrow[l + 1] : 0);
        nxt[r] = clamp_row(l + 2 < L2 ? mrow[l + 2] : 0);
    }
}

// Whether a layer of the stack is thicker than the fast phase reduction allows
// at the largest phase coefficient cm (wave-uniform).
template <int N>
__device__ __forceinline__ bool any_far(const double (&d)[N], int L, int lane, double cm) {
    bool far = false;
    for (int r = 0; r < N; ++r) far = far || (lane + r * kWave < L && !(d[r] <= (0.5 * kScFastRange) / cm));
    return __any(far);
}

// Layer data of the stack, N per lane (L + 2 <= 64 N), broadcast by readlane.
template <int N>
struct PairLayers {
    const double2* mtab;            // material table + lane: mtab[(row * kPairFields + f) * kWave]
    const unsigned char* pair_lane; // pair blocks + lane * 16
    double my_d[N];   // lane l, register r: thickness of layer 64 r + l + 1
    int my_code[N];   // pair block offset of that layer | lossy << 31
    int my_row[N];    // material row of medium 64 r + l
    __device__ __forceinline__ double d(int j) const { return lane_bcast(my_d, j - 1); }
    __device__ __forceinline__ int code(int j) const { return lane_bcast(my_code, j - 1); }
    __device__ __forceinline__ int row(int j) const { return lane_bcast(my_row, j); }
    __device__ __forceinline__ cx<double> field(int m, int f) const {
        const double2 v = mtab[(m * kPairFields + f) * kWave];
        return {v.x, v.y};
    }
    // rho_s, rho_p and the phase coefficients of step j
    __device__ __forceinline__ void pair(int code, cx<double>& rs, cx<double>& rp, double& cre, double& cim) const {
        const double2* e = reinterpret_cast<const double2*>(pair_lane + (code & 0x7fffffff));
        const double2 x = e[0], y = e[kWave], z = e[2 * kWave];
        rs = {x.x, x.y};
        rp = {y.x, y.y};
        cre = z.x;
        cim = z.y;
    }
};

template <int POL>
__device__ __forceinline__ void ratio_step(State& z, const cx<double>& rs, const cx<double>& rp,
                                           const cx<double>& E) {
    if (POL & 1) {
        const cx<double> X = cmul(rs, z.ts);
        const cx<double> a = cadd(z.ss, X), b = csub(z.ss, X);
        const cx<double> Eb = cmul(E, b);
        z.ss = cadd(a, Eb);
        z.ts = csub(a, Eb);
    }
    if (POL & 2) {
        const cx<double> X = cmul(rp, z.sp);
        const cx<double> a = cadd(X, z.tp), b = csub(X, z.tp);
        const cx<double> Eb = cmul(E, b);
        z.sp = cadd(a, Eb);
        z.tp = csub(a, Eb);
    }
}

// E_j and the base-2 attenuation exponent of step j (|d cre| < kScFastRange).
__device__ __forceinline__ cx<double> pair_phase(double dj, double cre, double cim, bool lossy,
                                                 const TabPhase<double>& phase, double& y) {
    cx<double> E = phase.cis_g(dj * cre);
    y = 0.0;
    if (lossy) {
        y = dj * cim;
        const double att = phase.atten(y);
        E.re *= att;
        E.im *= att;
    }
    return E;
}

template <int POL, int SEG, class LY>
__device__ void grad_stack_pair(const GradParams& p, const LY& src, const Ambient& amb, int b, int k, int i,
                                int lane, bool active, bool valid, double* ws, double* red, double* part,
                                const TabPhase<double>& phase) {
    const int L = p.L;
    constexpr int P = (POL == 3) ? 2 : 1;
    const double two_pi_lam = 2.0 * M_PI / p.wl[i];
    auto ck = [&](int c, int comp) -> double& { return ws[((size_t)c * kCkptDoubles + comp) * kWave + lane]; };
    auto save = [&](int c, const State& z) {
        ck(c, 0) = z.ss.re; ck(c, 1) = z.ss.im; ck(c, 2) = z.ts.re; ck(c, 3) = z.ts.im;
        ck(c, 4) = z.sp.re; ck(c, 5) = z.sp.im; ck(c, 6) = z.tp.re; ck(c, 7) = z.tp.im;
    };
    auto load = [&](int c) -> State {
        State z;
        z.ss = {ck(c, 0), ck(c, 1)}; z.ts = {ck(c, 2), ck(c, 3)};
        z.sp = {ck(c, 4), ck(c, 5)}; z.tp = {ck(c, 6), ck(c, 7)};
        return z;
    };

    // ---- pass A: forward with checkpoints --------------------------------
    State z;
    z.ss = z.ts = z.sp = z.tp = {1.0, 0.0};
    int es = 0, ep = 0;
    double S = 0.0;  // sum of the base-2 attenuation exponents
    save(0, z);
    for (int s = 0; s < p.n_seg_pair; ++s) {
        const int top = L - s * SEG;
        const int lo = top - SEG + 1 > 1 ? top - SEG + 1 : 1;
        for (int j = top; j >= lo; --j) {
            const int code = src.code(j);
            cx<double> rs, rp;
            double cre, cim, y;
            src.pair(code, rs, rp, cre, cim);
            const cx<double> E = pair_phase(src.d(j), cre, cim, code < 0, phase, y);
            S += y;
            ratio_step<POL>(z, rs, rp, E);
        }
        if (POL & 1) renorm_pair(z.ss, z.ts, es);
        if (POL & 2) renorm_pair(z.sp, z.tp, ep);
        save(s + 1, z);
    }
    const int m1 = src.row(1), msub = src.row(L + 1);
    const cx<double> q1 = src.field(m1, 0), e1 = src.field(m1, 1);
    const double eS = exp2_d<true>(S);
    const int two_L1 = 2 * (L + 1);
    const double nan = __builtin_nan("");
    const double w_act = active ? 1.0 : 0.0;  // ragged-tail lanes contribute nothing

    // ambient step (division-free: a = q0 sigma + q1 tau, a = eta1 sigma + eta0 tau) and output adjoints
    cx<double> sb_s = {0, 0}, tb_s = {0, 0}, sb_p = {0, 0}, tb_p = {0, 0};
    cx<double> pend_q = {0, 0}, pend_e = {0, 0};  // adjoints of q_1, eta_1 from the ambient step
    double cT_s = 0.0, cT_p = 0.0;
    const cx<double> q0 = {amb.q0r, amb.q0i}, e0 = {amb.e0r, amb.e0i};
    if (POL & 1) {
        const cx<double> A = cmul(q0, z.ss), Bv = cmul(q1, z.ts);
        const cx<double> a = cadd(A, Bv), bb = csub(A, Bv);
        const double na = cnorm(a);
        const double R = cnorm(bb) / na;
        const double T = ldexp(amb.Ks * src.field(msub, 0).re * eS / na, two_L1 - 2 * es);
        const int64_t o = (((int64_t)b * P + 0) * p.n_theta + k) * p.n_wl + i;
        if (active && p.R_out) p.R_out[o] = valid ? R : nan;
        if (active && p.T_out) p.T_out[o] = valid ? T : nan;
        const double gR = p.gR ? p.gR[o] * w_act : 0.0;
        const double gT = p.gT ? p.gT[o] * w_act : 0.0;
        cT_s = gT * T;
        const cx<double> abar = cscale(-2.0 * (gR * R + gT * T) / na, a);
        const cx<double> bbar = cscale(2.0 * gR / na, bb);
        const cx<double> Ab = cadd(abar, bbar), Bb = csub(abar, bbar);
        sb_s = cmulc(q0, Ab);
        tb_s = cmulc(q1, Bb);
        pend_q = cmulc(z.ts, Bb);
    }
    if (POL & 2) {
        const cx<double> A = cmul(e1, z.sp), Bv = cmul(e0, z.tp);
        const cx<double> a = cadd(A, Bv), bb = csub(A, Bv);
        const double na = cnorm(a);
        const double R = cnorm(bb) / na;
        const double T = ldexp(amb.Kp * src.field(msub, 1).re * eS / na, two_L1 - 2 * ep);
        const int64_t o = (((int64_t)b * P + (P - 1)) * p.n_theta + k) * p.n_wl + i;
        if (active && p.R_out) p.R_out[o] = valid ? R : nan;
        if (active && p.T_out) p.T_out[o] = valid ? T : nan;
        const double gR = p.gR ? p.gR[o] * w_act : 0.0;
        const double gT = p.gT ? p.gT[o] * w_act : 0.0;
        cT_p = gT * T;
        const cx<double> abar = cscale(-2.0 * (gR * R + gT * T) / na, a);
        const cx<double> bbar = cscale(2.0 * gR / na, bb);
        const cx<double> Ab = cadd(abar, bbar), Bb = csub(abar, bbar);
        sb_p = cmulc(e1, Ab);
        tb_p = cmulc(e0, Bb);
        pend_e = cmulc(z.sp, Ab);
    }
    const double cT = (POL & 1 ? cT_s : 0.0) + (POL & 2 ? cT_p : 0.0);
    if (!valid) {  // poison the gradients of this lane's stack
        sb_s = tb_s = sb_p = tb_p = pend_q = pend_e = {nan, nan};
    }
    cx<double> wprev_s = {0, 0}, wprev_p = {0, 0};  // w of the step below the current layer

    // ---- pass B: segments from the ambient side ----------------------------
    const int v_red = lane >> 2 < (3 * SEG) ? lane >> 2 : (3 * SEG) - 1;  // share this lane sums
    const double2* red_in = reinterpret_cast<const double2*>(red + v_red * kWave + (lane & 3) * 16);
    auto segment = [&](auto nst_c, int s, int top) {
        constexpr int NST = decltype(nst_c)::value;
        State zin[NST];
        cx<double> Es[NST];
        State zz = load(s);
#pragma unroll
        for (int t = 0; t < NST; ++t) {
            const int j = top - t;
            const int code = src.code(j);
            cx<double> rs, rp;
            double cre, cim, y;
            src.pair(code, rs, rp, cre, cim);
            Es[t] = pair_phase(src.d(j), cre, cim, code < 0, phase, y);
            zin[t] = zz;
            ratio_step<POL>(zz, rs, rp, Es[t]);
        }
        // the forward pass renormalised the segment's end state; undo on the adjoint
        if (POL & 1) {
            const double f = ldexp(1.0, -pair_exp(zz.ss, zz.ts));
            sb_s = cscale(f, sb_s);
            tb_s = cscale(f, tb_s);
        }
        if (POL & 2) {
            const double f = ldexp(1.0, -pair_exp(zz.sp, zz.tp));
            sb_p = cscale(f, sb_p);
            tb_p = cscale(f, tb_p);
        }
#pragma unroll
        for (int t = NST - 1; t >= 0; --t) {
            const int j = top - t;
            cx<double> rs, rp;
            double cre, cim;
            src.pair(src.code(j), rs, rp, cre, cim);
            const cx<double> E = Es[t];
            cx<double> Eb = {0.0, 0.0};
            cx<double> w_s = {0, 0}, w_p = {0, 0};
            if (POL & 1) {
                const cx<double> X = cmul(rs, zin[t].ts);
                const cx<double> bv = csub(zin[t].ss, X);
                const cx<double> ab = cadd(sb_s, tb_s), Y = csub(sb_s, tb_s);
                const cx<double> bb = cmulc(E, Y);
                Eb = cadd(Eb, cmulc(bv, Y));
                const cx<double> Xb = csub(ab, bb);
                sb_s = cadd(ab, bb);
                tb_s = cmulc(rs, Xb);
                w_s = cmulc(X, Xb);
            }
            if (POL & 2) {
                const cx<double> X = cmul(rp, zin[t].sp);
                const cx<double> bv = csub(X, zin[t].tp);
                const cx<double> ab = cadd(sb_p, tb_p), Y = csub(sb_p, tb_p);
                const cx<double> bb = cmulc(E, Y);
                Eb = cadd(Eb, cmulc(bv, Y));
                const cx<double> Xb = cadd(ab, bb);
                tb_p = csub(ab, bb);
                sb_p = cmulc(rp, Xb);
                w_p = cmulc(X, Xb);
            }
            const int m = src.row(j);
            const cx<double> qj = src.field(m, 0);
            const double dj = src.d(j);
            // deltab = -2i conj(E) Eb - 2i cT  (chain and e^{-2 Im sum delta})
            const cx<double> cE = cmulc(E, Eb);
            const cx<double> db = {2.0 * cE.im, -2.0 * cE.re - 2.0 * cT};
            const double gd = two_pi_lam * (db.re * qj.re + db.im * qj.im);
            const cx<double> qb = cadd(pend_q, cscale(two_pi_lam * dj, db));
            cx<double> nb = cmulc(src.field(m, 2), qb);
            if (POL & 2) nb = cadd(nb, cmulc(src.field(m, 3), pend_e));
            if (POL & 1) nb = cadd(nb, cmulc(src.field(m, 4), csub(wprev_s, w_s)));
            if (POL & 2) nb = cadd(nb, cmulc(src.field(m, 5), csub(wprev_p, w_p)));
            wprev_s = w_s;
            wprev_p = w_p;
            pend_q = pend_e = {0.0, 0.0};
            red[(3 * t + 0) * kWave + lane] = gd;
            red[(3 * t + 1) * kWave + lane] = nb.re;
            red[(3 * t + 2) * kWave + lane] = nb.im;
        }
    };
    for (int s = p.n_seg_pair - 1; s >= 0; --s) {
        const int top = L - s * SEG;
        const int lo = top - SEG + 1 > 1 ? top - SEG + 1 : 1;
        const int nst = top - lo + 1;
        if (nst == SEG) {
            segment(std::integral_constant<int, SEG>(), s, top);
        } else {
            static_assert(SEG <= 5, "segment lengths below are spelled out");
            if (nst == 1) segment(std::integral_constant<int, 1>(), s, top);
            if (SEG > 2 && nst == 2) segment(std::integral_constant<int, (SEG > 2 ? 2 : 1)>(), s, top);
            if (SEG > 3 && nst == 3) segment(std::integral_constant<int, (SEG > 3 ? 3 : 1)>(), s, top);
            if (SEG > 4 && nst == 4) segment(std::integral_constant<int, (SEG > 4 ? 4 : 1)>(), s, top);
        }
        wave_sync();
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double2 x = red_in[u];
            acc += x.x;
            acc += x.y;
        }
        acc = quad_add<0xB1>(acc);
        acc = quad_add<0x4E>(acc);
        if ((lane & 3) == 0 && (lane >> 2) < 3 * nst) {
            const int v = lane >> 2;
            const int t = v / 3;
            part[(top - t - 1) * 3 + (v - 3 * t)] = acc;
        }
        wave_sync();
    }
}

// Fills the block's material table and pair blocks for one column and ambient
// row (all waves share the work), and per wave: a ratio out of bound in a used
// lane, the largest phase coefficient, and the lossy flag of each material.
__device__ void build_pair_table(const GradParams& p, double2* mtab, unsigned char* pairs, int amb_row, int i,
                                 bool lane_used, double st, double ct, int wave, int lane, int* s_bad,
                                 double* s_cmax, int* s_lossy, int nwaves = kGradPairWaves) {
    double n0r, n0i;
    load_n(p.nk, p.dispersive, p.n_wl, amb_row, i, n0r, n0i);
    const Ambient a = make_ambient(n0r, n0i, st, ct);
    const double lam = p.wl[i];
    for (int m = wave; m < p.n_mat; m += nwaves) {
        double nr, ni;
        load_n(p.nk, p.dispersive, p.n_wl, m, i, nr, ni);
        const Medium md = make_medium(nr, ni, a.kx);
        const FL f = fl_from(md);
        const AL g = al_from(nr, ni, f);
        const cx<double> lq = cdiv(g.nq, f.q), le = cdiv(g.de, f.e);
        double2* e = mtab + m * kPairFields * kWave + lane;
        e[0] = make_double2(f.q.re, f.q.im);
        e[kWave] = make_double2(f.e.re, f.e.im);
        e[2 * kWave] = make_double2(g.nq.re, g.nq.im);
        e[3 * kWave] = make_double2(g.de.re, g.de.im);
        e[4 * kWave] = make_double2(lq.re, lq.im);
        e[5 * kWave] = make_double2(le.re, le.im);
        const bool lossy = __any(md.qi != 0.0);
        if (lane == 0) s_lossy[m] = lossy ? 1 : 0;
    }
    bool bad = false;
    double cmax = 0.0;
    const double c4lam = 4.0 / lam;
    for (int pi = wave; pi < p.n_mat * p.n_mat; pi += nwaves) {
        const int mc = pi / p.n_mat, mn = pi - mc * p.n_mat;
        double ar, ai, br, bi;
        load_n(p.nk, p.dispersive, p.n_wl, mc, i, ar, ai);
        load_n(p.nk, p.dispersive, p.n_wl, mn, i, br, bi);
        const Medium ma = make_medium(ar, ai, a.kx), mb = make_medium(br, bi, a.kx);
        const cx<double> rs = cdiv({mb.qr, mb.qi}, {ma.qr, ma.qi});
        const cx<double> rp = cdiv({mb.er, mb.ei}, {ma.er, ma.ei});
        const double cre = (c4lam * kScSteps) * ma.qr, cim = c4lam * ma.qi * kNegPiLog2e;
        double2* e = reinterpret_cast<double2*>(pairs + (size_t)pi * kGradPairBlockBytes) + lane;
        e[0] = make_double2(rs.re, rs.im);
        e[kWave] = make_double2(rp.re, rp.im);
        e[2 * kWave] = make_double2(cre, cim);
        if (lane_used) {
            const double mag = fmax(fmax(fabs(rs.re), fabs(rs.im)), fmax(fabs(rp.re), fabs(rp.im)));
            bad = bad || !(mag <= kPairRatioMax);
            cmax = fmax(cmax, fabs(cre));
        }
    }
    const bool wbad = __any(bad);
    for (int off = kWave / 2; off >= 1; off >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, off));
    if (lane == 0) {
        s_bad[wave] = wbad ? 1 : 0;
        s_cmax[wave] = cmax;
    }
}

template <int POL, int SEG, int N>
__global__ void __launch_bounds__(kGradPairBlock) __attribute__((amdgpu_waves_per_eu(2)))
grad_pair_kernel(GradParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_rows[kGradPairWaves];
    __shared__ int s_bad[kGradPairWaves];
    __shared__ double s_cmax[kGradPairWaves];
    __shared__ int s_lossy[kGradPairMaxMat];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    fill_phase_tab<double>(smem, threadIdx.x, kGradPairBlock);
    __syncthreads();
    const TabPhase<double> phase = phase_of<double>(smem);
    unsigned char* const lds = smem + phase_tab_bytes<double>();
    double* red = reinterpret_cast<double*>(lds) + wave * (3 * SEG) * kWave;
    double2* mtab = reinterpret_cast<double2*>(lds + (size_t)kGradPairWaves * (3 * SEG) * kWave * sizeof(double));
    unsigned char* pairs = reinterpret_cast<unsigned char*>(mtab + (size_t)p.n_mat * kPairFields * kWave);
    double* ws = p.ws + ((size_t)blockIdx.x * kGradPairWaves + wave) * (size_t)(p.n_seg + 1) * kCkptDoubles * kWave;
    const int L2 = p.L + 2;
    const int64_t nbs = p.b_end - p.b_begin;
    const int64_t groups = (nbs + kGradPairWaves - 1) / kGradPairWaves;
    const int64_t t0 = (int64_t)blockIdx.x * p.per_block;
    const int64_t t1 = t0 + p.per_block < p.n_tasks ? t0 + p.per_block : p.n_tasks;
    int64_t tab_col = -1;
    int tab_row = -1;
    for (int64_t t = t0; t < t1; ++t) {
        // task = (column, group of kGradPairWaves stacks)
        const int64_t col = t / groups;
        const int tk_k = (int)(col / p.n_tiles);
        const int tk_tile = (int)(col - (int64_t)tk_k * p.n_tiles);
        const int tk_b = p.b_begin + (int)(t - col * groups) * kGradPairWaves + wave;
        const int i_raw = tk_tile * kWave + lane;
        const bool active = i_raw < p.n_wl;
        const int i = active ? i_raw : p.n_wl - 1;
        const double lam = p.wl[i];
        const bool lam_ok = lam > 0.0 && lam < __builtin_inf();
        const double st = p.sin_t[tk_k], ct = p.cos_t[tk_k];
        const bool has = tk_b < p.b_end;
        const int b = has ? tk_b : p.b_end - 1;
        const ciptr mrow = (ciptr)(p.mat + (int64_t)b * L2);
        double* part = p.partial + ((size_t)col * nbs + (b - p.b_begin)) * (size_t)p.L * 3;
        const double* drow = p.d + (int64_t)b * p.L;
        // after the inverse-walk kernel: only the stacks it left
        const bool mine = has && (!p.redo || p.redo[(size_t)col * nbs + (b - p.b_begin)] != 0);
        if (p.redo && __syncthreads_or(mine ? 1 : 0) == 0) continue;
        const bool bad = mine && stack_bad(p, drow, mrow, lane);
        int a_row = mrow[0];
        a_row = a_row < 0 ? 0 : (a_row >= p.n_mat ? p.n_mat - 1 : a_row);
        bool done = !mine;
        // one sub-round per distinct ambient row among the block's stacks
        for (;;) {
            __syncthreads();
            if (lane == 0) s_rows[wave] = done ? INT_MAX : a_row;
            __syncthreads();
            int r = s_rows[0];
            for (int w = 1; w < kGradPairWaves; ++w) r = min(r, s_rows[w]);
            if (r == INT_MAX) break;
            if (r != tab_row || col != tab_col) {
                double n0r, n0i;
                load_n(p.nk, p.dispersive, p.n_wl, r, i, n0r, n0i);
                const bool used = active && lam_ok && make_ambient(n0r, n0i, st, ct).ok;
                build_pair_table(p, mtab, pairs, r, i, used, st, ct, wave, lane, s_bad, s_cmax, s_lossy);
                tab_row = r;
                tab_col = col;
            }
            __syncthreads();
            if (!done && a_row == r) {
                int any_bad = 0;
                double cm = 0.0;
                for (int w = 0; w < kGradPairWaves; ++w) {
                    any_bad |= s_bad[w];
                    cm = fmax(cm, s_cmax[w]);
                }
                uint32_t mask = 0;
                for (int m = 0; m < p.n_mat; ++m) mask |= (uint32_t)s_lossy[m] << m;
                double n0r, n0i;
                load_n(p.nk, p.dispersive, p.n_wl, a_row, i, n0r, n0i);
                const Ambient amb = make_ambient(n0r, n0i, st, ct);
                const bool ok = lam_ok && amb.ok && !bad;
                // layer data N per lane; a layer thicker than 2^49 / (256 max cre) would
                // leave the fast phase reduction's range
                PairLayers<N> src;
                src.mtab = mtab + lane;
                src.pair_lane = pairs + lane * 16;
                int m_cur[N], m_nxt[N];
                load_layers(p, drow, mrow, lane, src.my_d, src.my_row, m_cur, m_nxt);
                for (int r = 0; r < N; ++r)
                    src.my_code[r] =
                        (m_cur[r] * p.n_mat + m_nxt[r]) * kGradPairBlockBytes | (int)(((mask >> m_cur[r]) & 1u) << 31);
                const bool far = any_far(src.my_d, p.L, lane, cm);
                if (any_bad == 0 && !far) {
                    grad_stack_pair<POL, SEG>(p, src, amb, b, tk_k, i, lane, active, ok, ws, red, part, phase);
                } else {
                    InlSrc isrc;
                    isrc.nk = p.nk;
                    isrc.drow = (cdptr)drow;
                    isrc.mrow = mrow;
                    isrc.base = (int64_t)b * L2;
                    isrc.n_mat = p.n_mat;
                    isrc.dispersive = p.dispersive;
                    isrc.n_wl = p.n_wl;
                    isrc.i = i;
                    isrc.kx = amb.kx;
                    grad_stack<POL>(p, isrc, amb, b, tk_k, i, lane, active, ok, ws, red, part, phase);
                }
                done = true;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Inverse walk (ratio form, lossless media).  When every table row is lossless
// and propagating at the block's column (Im q = 0 in every lane), every q and
// eta is real, so are the ratios rho_s = q_{j+1}/q_j and rho_p = eta_{j+1}/eta_j
// and the derivative factors of the adjoint, and every layer factor
// E_j = e^{2 i delta_j} has modulus 1.  The ratio step is then inverted exactly
// and stably: with u = s' + t', D = s' - t' of the step's output and
// v = conj(E) D / 4,
//   s: s = u/4 + v, X = rho t = u/4 - v, t = X / rho_s
//   p: X = rho s = u/4 + v, t = u/4 - v, s = X / rho_p
// where 1 / rho is the ratio of the reversed material pair (tabulated too).
// Pass B walks from the ambient to the substrate recovering each step's input
// from its output, with no checkpoints and no per-segment register arrays.
// The adjoint of each step is that of grad_stack_pair with real rho; its
// difference term b (s - X or X - t) equals 2 v, so conj(E) Eb reduces to
// sum_pol conj(D) Y / 2.  The state and its adjoint are rescaled together by
// powers of two (their products, which make the gradients, are unchanged).
// Shares are reduced per SEG layers as in grad_stack_pair.
//
// Real tables (per lane): material row m holds kInvRows double2 entries
//   0 {cre, dq/dn}  1 {(dq/dn)/q, (deta/dn)/eta}  2 {q, eta}  3 {deta/dn, 0}
// with cre = 4 kScSteps q / lambda (the phase of layer thickness d is d cre in
// units of 1/kScSteps half-turn); the ordered pair (m, m') holds {rho_s, rho_p}.
constexpr int kInvRows = 4;
// Table rows the inverse walk takes: seven at twelve waves per block (146 KiB
// of LDS), six at sixteen; pair codes of 6 bits.
constexpr int kGradInvMaxMat = 7;
constexpr int kInvRenormSegs = 2;  // segments between rescalings: growth <= 2^9 per step either way
// Share vectors of the inverse walk are kInvRedStride doubles apart (64 values +
// 8 of padding): with each lane quad reading its vector in interleaved 16-byte
// pieces, any eight consecutive lanes then read 128 distinct bytes (no bank
// conflicts in the segment reduction).
constexpr int kInvRedStride = kWave + 8;

template <int N>
struct InvLayers {
    const double2* mt;  // material rows + lane: mt[(m * kInvRows + f) * kWave]
    const double2* pr;  // pair ratios + lane: pr[pair * kWave]
    double my_d[N];     // lane l, register r: thickness of layer 64 r + l + 1
    int my_code[N];     // that layer: pair | reversed pair << 6 | material << 12
    int my_row[N];      // material row of medium 64 r + l
    __device__ __forceinline__ double d(int j) const { return lane_bcast(my_d, j - 1); }
    __device__ __forceinline__ int code(int j) const { return lane_bcast(my_code, j - 1); }
    __device__ __forceinline__ int row(int j) const { return lane_bcast(my_row, j); }
    __device__ __forceinline__ double2 ratio(int pair) const { return pr[pair * kWave]; }
    __device__ __forceinline__ double2 mat(int m, int f) const { return mt[(m * kInvRows + f) * kWave]; }
};

__host__ __device__ constexpr size_t grad_inv_lds_bytes(int n_mat, int seg, int waves) {
    return phase_tab_bytes<double>() + (size_t)waves * 3 * seg * kInvRedStride * sizeof(double) +
           (size_t)n_mat * kInvRows * kWave * sizeof(double2) + (size_t)n_mat * n_mat * kWave * sizeof(double2);
}

// Fill the real tables for the column of wavelength i (this lane) and the
// ambient row amb_row; flag rows that are lossy or evanescent in some lane
// (s_lossy), ratios beyond kPairRatioMax (s_bad) and the largest |cre| (s_cmax).
__device__ void build_inv_table(const GradParams& p, double2* mt, double2* pr, int amb_row, int i, bool lane_used,
                                double st, double ct, int wave, int lane, int* s_bad, double* s_cmax, int* s_lossy,
                                int nwaves) {
    double n0r, n0i;
    load_n(p.nk, p.dispersive, p.n_wl, amb_row, i, n0r, n0i);
    const Ambient a = make_ambient(n0r, n0i, st, ct);
    const double c4s = (4.0 / p.wl[i]) * kScSteps;
    double cmax = 0.0;
    for (int m = wave; m < p.n_mat; m += nwaves) {
        double nr, ni;
        load_n(p.nk, p.dispersive, p.n_wl, m, i, nr, ni);
        const Medium md = make_medium(nr, ni, a.kx);
        const FL f = fl_from(md);
        const AL g = al_from(nr, ni, f);
        double2* e = mt + m * kInvRows * kWave + lane;
        const double cre = c4s * md.qr;
        e[0] = make_double2(cre, g.nq.re);
        e[kWave] = make_double2(g.nq.re / md.qr, g.de.re / md.er);
        e[2 * kWave] = make_double2(md.qr, md.er);
        e[3 * kWave] = make_double2(g.de.re, 0.0);
        const bool lossy = __any(md.qi != 0.0);
        if (lane == 0) s_lossy[m] = lossy ? 1 : 0;
        if (lane_used) cmax = fmax(cmax, fabs(cre));
    }
    bool bad = false;
    for (int pi = wave; pi < p.n_mat * p.n_mat; pi += nwaves) {
        const int mc = pi / p.n_mat, mn = pi - mc * p.n_mat;
        double ar, ai, br, bi;
        load_n(p.nk, p.dispersive, p.n_wl, mc, i, ar, ai);
        load_n(p.nk, p.dispersive, p.n_wl, mn, i, br, bi);
        const Medium ma = make_medium(ar, ai, a.kx), mb = make_medium(br, bi, a.kx);
        const double rs = mb.qr / ma.qr, rp = mb.er / ma.er;
        pr[pi * kWave + lane] = make_double2(rs, rp);
        if (lane_used) bad = bad || !(fmax(fabs(rs), fabs(rp)) <= kPairRatioMax);
    }
    const bool wbad = __any(bad);
    for (int off = kWave / 2; off >= 1; off >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, off));
    if (lane == 0) {
        s_bad[wave] = wbad ? 1 : 0;
        s_cmax[wave] = cmax;
    }
}

template <int POL, int SEG, class LY>
__device__ void grad_stack_inv(const GradParams& p, const LY& src, const Ambient& amb, int b, int k, int i,
                               int lane, bool active, bool valid, double* red, double* part,
                               const TabPhase<double>& phase) {
    const int L = p.L;
    constexpr int P = (POL == 3) ? 2 : 1;
    const double two_pi_lam = 2.0 * M_PI / p.wl[i];
    constexpr double kG = M_PI / (2.0 * kScSteps);  // 2 pi q / lambda = kG cre

    // ---- pass A: forward (ratio form), renormalised every block ------------
    State z;
    z.ss = z.ts = z.sp = z.tp = {1.0, 0.0};
    int es = 0, ep = 0;
    constexpr int RPA = 32;  // steps between renormalisations: growth <= 2 (1 + 256) per step
    for (int top = L; top >= 1; top -= RPA) {
        const int lo = top - RPA + 1 > 1 ? top - RPA + 1 : 1;
        for (int j = top; j >= lo; --j) {
            const int c = src.code(j);
            const double2 r = src.ratio(c & 63);
            const cx<double> E = phase.cis_g(src.d(j) * src.mat(c >> 12, 0).x);
            if (POL & 1) {
                const cx<double> X = cscale(r.x, z.ts);
                const cx<double> a = cadd(z.ss, X), bd = csub(z.ss, X);
                const cx<double> Eb = cmul(E, bd);
                z.ss = cadd(a, Eb);
                z.ts = csub(a, Eb);
            }
            if (POL & 2) {
                const cx<double> X = cscale(r.y, z.sp);
                const cx<double> a = cadd(X, z.tp), bd = csub(X, z.tp);
                const cx<double> Eb = cmul(E, bd);
                z.sp = cadd(a, Eb);
                z.tp = csub(a, Eb);
            }
        }
        if (POL & 1) renorm_pair(z.ss, z.ts, es);
        if (POL & 2) renorm_pair(z.sp, z.tp, ep);
    }
    const int m1 = src.row(1), msub = src.row(L + 1);
    const double2 qe1 = src.mat(m1, 2);
    const cx<double> q1 = {qe1.x, 0.0}, e1 = {qe1.y, 0.0};
    const double2 qesub = src.mat(msub, 2);
    const int two_L1 = 2 * (L + 1);
    const double nan = __builtin_nan("");
    const double w_act = active ? 1.0 : 0.0;  // ragged-tail lanes contribute nothing

    // ambient step (division-free) and output adjoints, as in grad_stack_pair (no attenuation)
    cx<double> sb_s = {0, 0}, tb_s = {0, 0}, sb_p = {0, 0}, tb_p = {0, 0};
    cx<double> pend_q = {0, 0}, pend_e = {0, 0};
    double cT = 0.0;  // sum of gT T: T's dependence on Im delta (through Im n) survives at Im n = 0
    const cx<double> q0 = {amb.q0r, amb.q0i}, e0 = {amb.e0r, amb.e0i};
    if (POL & 1) {
        const cx<double> A = cmul(q0, z.ss), Bv = cmul(q1, z.ts);
        const cx<double> a = cadd(A, Bv), bb = csub(A, Bv);
        const double na = cnorm(a);
        const double R = cnorm(bb) / na;
        const double T = ldexp(amb.Ks * qesub.x / na, two_L1 - 2 * es);
        const int64_t o = (((int64_t)b * P + 0) * p.n_theta + k) * p.n_wl + i;
        if (active && p.R_out) p.R_out[o] = valid ? R : nan;
        if (active && p.T_out) p.T_out[o] = valid ? T : nan;
        const double gR = p.gR ? p.gR[o] * w_act : 0.0;
        const double gT = p.gT ? p.gT[o] * w_act : 0.0;
        cT += gT * T;
        const cx<double> abar = cscale(-2.0 * (gR * R + gT * T) / na, a);
        const cx<double> bbar = cscale(2.0 * gR / na, bb);
        const cx<double> Ab = cadd(abar, bbar), Bb = csub(abar, bbar);
        sb_s = cmulc(q0, Ab);
        tb_s = cmulc(q1, Bb);
        pend_q = cmulc(z.ts, Bb);
    }
    if (POL & 2) {
        const cx<double> A = cmul(e1, z.sp), Bv = cmul(e0, z.tp);
        const cx<double> a = cadd(A, Bv), bb = csub(A, Bv);
        const double na = cnorm(a);
        const double R = cnorm(bb) / na;
        const double T = ldexp(amb.Kp * qesub.y / na, two_L1 - 2 * ep);
        const int64_t o = (((int64_t)b * P + (P - 1)) * p.n_theta + k) * p.n_wl + i;
        if (active && p.R_out) p.R_out[o] = valid ? R : nan;
        if (active && p.T_out) p.T_out[o] = valid ? T : nan;
        const double gR = p.gR ? p.gR[o] * w_act : 0.0;
        const double gT = p.gT ? p.gT[o] * w_act : 0.0;
        cT += gT * T;
        const cx<double> abar = cscale(-2.0 * (gR * R + gT * T) / na, a);
        const cx<double> bbar = cscale(2.0 * gR / na, bb);
        const cx<double> Ab = cadd(abar, bbar), Bb = csub(abar, bbar);
        sb_p = cmulc(e1, Ab);
        tb_p = cmulc(e0, Bb);
        pend_e = cmulc(z.sp, Ab);
    }
    if (!valid) sb_s = tb_s = sb_p = tb_p = pend_q = pend_e = {nan, nan};
    cx<double> wprev_s = {0, 0}, wprev_p = {0, 0};
    // the ambient step's share of layer 1's index adjoint (through q_1 and eta_1)
    cx<double> pend_nb = {0.0, 0.0};
    if (POL & 1) pend_nb = cscale(src.mat(m1, 0).y, pend_q);
    if (POL & 2) pend_nb = cadd(pend_nb, cscale(src.mat(m1, 3).x, pend_e));

    // ---- pass B: from the ambient to the substrate -------------------------
    const int n_seg = (L + SEG - 1) / SEG;
    const int v_red = lane >> 2 < (3 * SEG) ? lane >> 2 : (3 * SEG) - 1;  // share this lane sums
    // quarter (lane & 3) of that share: values 8u + 2 (lane & 3) and the next, u = 0..7
    const double2* red_in = reinterpret_cast<const double2*>(red + v_red * kInvRedStride) + (lane & 3);
    for (int s = n_seg - 1; s >= 0; --s) {
        const int top = L - s * SEG;
        const int lo = top - SEG + 1 > 1 ? top - SEG + 1 : 1;
        const int nst = top - lo + 1;
        for (int j = lo; j <= top; ++j) {
            const int t = top - j;  // share slot, as in grad_stack_pair
            const int c = src.code(j);
            const double2 r = src.ratio(c & 63), rr = src.ratio((c >> 6) & 63);
            const double2 f0 = src.mat(c >> 12, 0), f1 = src.mat(c >> 12, 1);  // {cre, dq/dn}, {dlog q, dlog eta}
            const double dj = src.d(j);
            const cx<double> E = phase.cis_g(dj * f0.x);
            const cx<double> Eq = {0.25 * E.re, -0.25 * E.im};  // conj(E) / 4
            cx<double> cD;  // sum over the polarisations of conj(D) Y
            cx<double> w_s = {0, 0}, w_p = {0, 0};
            if (POL & 1) {
                const cx<double> D = csub(z.ss, z.ts), u4 = cscale(0.25, cadd(z.ss, z.ts));
                const cx<double> v = cmul(Eq, D);
                const cx<double> X = csub(u4, v);
                z.ss = cadd(u4, v);
                z.ts = cscale(rr.x, X);
                const cx<double> ab = cadd(sb_s, tb_s), Y = csub(sb_s, tb_s);
                const cx<double> bb = cmulc(E, Y);
                cD = cmulc(D, Y);
                const cx<double> Xb = csub(ab, bb);
                sb_s = cadd(ab, bb);
                tb_s = cscale(r.x, Xb);
                w_s = cmulc(X, Xb);
            }
            if (POL & 2) {
                const cx<double> D = csub(z.sp, z.tp), u4 = cscale(0.25, cadd(z.sp, z.tp));
                const cx<double> v = cmul(Eq, D);
                const cx<double> X = cadd(u4, v);
                z.tp = csub(u4, v);
                z.sp = cscale(rr.y, X);
                const cx<double> ab = cadd(sb_p, tb_p), Y = csub(sb_p, tb_p);
                const cx<double> bb = cmulc(E, Y);
                cD = (POL & 1) ? cadd(cD, cmulc(D, Y)) : cmulc(D, Y);
                const cx<double> Xb = cadd(ab, bb);
                tb_p = csub(ab, bb);
                sb_p = cscale(r.y, Xb);
                w_p = cmulc(X, Xb);
            }
            // deltab = -2i conj(E) Eb - 2i cT = -i cD - 2i cT (chain and e^{-2 Im sum delta})
            const cx<double> db = {two_pi_lam * cD.im, -two_pi_lam * (cD.re + 2.0 * cT)};
            const double gd = kG * cD.im * f0.x;
            cx<double> nb = cadd(pend_nb, cscale(f0.y * dj, db));
            if (POL & 1) nb = cadd(nb, cscale(f1.x, csub(wprev_s, w_s)));
            if (POL & 2) nb = cadd(nb, cscale(f1.y, csub(wprev_p, w_p)));
            wprev_s = w_s;
            wprev_p = w_p;
            pend_nb = {0.0, 0.0};
            red[(3 * t + 0) * kInvRedStride + lane] = gd;
            red[(3 * t + 1) * kInvRedStride + lane] = nb.re;
            red[(3 * t + 2) * kInvRedStride + lane] = nb.im;
        }
        // keep the walked state near 1: scale it and its adjoint inversely
        if (s % kInvRenormSegs == 0) {
            if (POL & 1) {
                const int e = pair_exp(z.ss, z.ts);
                const double f = ldexp(1.0, -e), g = ldexp(1.0, e);
                z.ss = cscale(f, z.ss);
                z.ts = cscale(f, z.ts);
                sb_s = cscale(g, sb_s);
                tb_s = cscale(g, tb_s);
            }
            if (POL & 2) {
                const int e = pair_exp(z.sp, z.tp);
                const double f = ldexp(1.0, -e), g = ldexp(1.0, e);
                z.sp = cscale(f, z.sp);
                z.tp = cscale(f, z.tp);
                sb_p = cscale(g, sb_p);
                tb_p = cscale(g, tb_p);
            }
        }
        wave_sync();
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double2 x = red_in[4 * u];
            acc += x.x;
            acc += x.y;
        }
        acc = quad_add<0xB1>(acc);
        acc = quad_add<0x4E>(acc);
        if ((lane & 3) == 0 && (lane >> 2) < 3 * nst) {
            const int v = lane >> 2;
            const int t = v / 3;
            part[(top - t - 1) * 3 + (v - 3 * t)] = acc;
        }
        wave_sync();
    }
}

// Persistent blocks of WAVES waves over tasks (column, group of WAVES stacks),
// the block's real tables built per (column, ambient row) as in grad_pair_kernel.
// Stacks whose column is not lossless, whose ratios leave their bound or whose
// phases leave the fast range are marked in p.redo and left to grad_pair_kernel
// (at most five rows) or to grad_kernel.
template <int POL, int SEG, int WAVES, int N>
__global__ void __launch_bounds__(WAVES * kWave) grad_inv_kernel(GradParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_rows[WAVES];
    __shared__ int s_bad[WAVES];
    __shared__ double s_cmax[WAVES];
    __shared__ int s_lossy[kGradInvMaxMat];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    fill_phase_tab<double>(smem, threadIdx.x, WAVES * kWave);
    __syncthreads();
    const TabPhase<double> phase = phase_of<double>(smem);
    unsigned char* const lds = smem + phase_tab_bytes<double>();
    double* red = reinterpret_cast<double*>(lds) + wave * (3 * SEG) * kInvRedStride;
    double2* mt = reinterpret_cast<double2*>(lds + (size_t)WAVES * (3 * SEG) * kInvRedStride * sizeof(double));
    double2* pr = mt + (size_t)p.n_mat * kInvRows * kWave;
    const int L2 = p.L + 2;
    const int64_t nbs = p.b_end - p.b_begin;
    const int64_t groups = (nbs + WAVES - 1) / WAVES;
    const int64_t t0 = (int64_t)blockIdx.x * p.per_block;
    const int64_t t1 = t0 + p.per_block < p.n_tasks ? t0 + p.per_block : p.n_tasks;
    int64_t tab_col = -1;
    int tab_row = -1;
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t col = t / groups;
        const int tk_k = (int)(col / p.n_tiles);
        const int tk_tile = (int)(col - (int64_t)tk_k * p.n_tiles);
        const int tk_b = p.b_begin + (int)(t - col * groups) * WAVES + wave;
        const int i_raw = tk_tile * kWave + lane;
        const bool active = i_raw < p.n_wl;
        const int i = active ? i_raw : p.n_wl - 1;
        const double lam = p.wl[i];
        const bool lam_ok = lam > 0.0 && lam < __builtin_inf();
        const double st = p.sin_t[tk_k], ct = p.cos_t[tk_k];
        const bool has = tk_b < p.b_end;
        const int b = has ? tk_b : p.b_end - 1;
        const ciptr mrow = (ciptr)(p.mat + (int64_t)b * L2);
        double* part = p.partial + ((size_t)col * nbs + (b - p.b_begin)) * (size_t)p.L * 3;
        const double* drow = p.d + (int64_t)b * p.L;
        const bool bad = stack_bad(p, drow, mrow, lane);
        int a_row = mrow[0];
        a_row = a_row < 0 ? 0 : (a_row >= p.n_mat ? p.n_mat - 1 : a_row);
        bool done = !has;
        for (;;) {
            __syncthreads();
            if (lane == 0) s_rows[wave] = done ? INT_MAX : a_row;
            __syncthreads();
            int r = s_rows[0];
            for (int w = 1; w < WAVES; ++w) r = min(r, s_rows[w]);
            if (r == INT_MAX) break;
            if (r != tab_row || col != tab_col) {
                double n0r, n0i;
                load_n(p.nk, p.dispersive, p.n_wl, r, i, n0r, n0i);
                const bool used = active && lam_ok && make_ambient(n0r, n0i, st, ct).ok;
                build_inv_table(p, mt, pr, r, i, used, st, ct, wave, lane, s_bad, s_cmax, s_lossy, WAVES);
                tab_row = r;
                tab_col = col;
            }
            __syncthreads();
            if (!done && a_row == r) {
                int any_bad = 0, any_lossy = 0;
                double cm = 0.0;
                for (int w = 0; w < WAVES; ++w) {
                    any_bad |= s_bad[w];
                    cm = fmax(cm, s_cmax[w]);
                }
                for (int m2 = 0; m2 < p.n_mat; ++m2) any_lossy |= s_lossy[m2];
                double n0r, n0i;
                load_n(p.nk, p.dispersive, p.n_wl, a_row, i, n0r, n0i);
                const Ambient amb = make_ambient(n0r, n0i, st, ct);
                const bool ok = lam_ok && amb.ok && !bad;
                InvLayers<N> src;
                src.mt = mt + lane;
                src.pr = pr + lane;
                int m_cur[N], m_nxt[N];
                load_layers(p, drow, mrow, lane, src.my_d, src.my_row, m_cur, m_nxt);
                for (int r = 0; r < N; ++r)
                    src.my_code[r] =
                        (m_cur[r] * p.n_mat + m_nxt[r]) | (m_nxt[r] * p.n_mat + m_cur[r]) << 6 | m_cur[r] << 12;
                const bool far = any_far(src.my_d, p.L, lane, cm);
                const bool mine = any_bad == 0 && any_lossy == 0 && !far;
                if (mine) grad_stack_inv<POL, SEG>(p, src, amb, b, tk_k, i, lane, active, ok, red, part, phase);
                if (lane == 0) p.redo[(size_t)col * nbs + (b - p.b_begin)] = mine ? 0 : 1;
                done = true;
            }
        }
    }
}

// grad[g] = sum over the columns of partial[col][g] in column order (g runs
// over the launch's stacks x layers x {d, Re n, Im n}).
__global__ void grad_reduce(const double* partial, int64_t cols, int64_t n, int64_t g0, double* grad_d,
                            double* grad_n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        double s = 0.0;
        for (int64_t c = 0; c < cols; ++c) s += partial[c * n + t];
        const int64_t g = g0 + t / 3;
        const int comp = (int)(t % 3);
        if (comp == 0) {
            if (grad_d) grad_d[g] = s;
        } else if (grad_n) {
            grad_n[2 * g + comp - 1] = s;
        }
    }
}

__global__ void zero_fill(double* x, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) x[t] = 0.0;
}

// Workspace layout: checkpoint slots of the persistent grid, then the
// partial sums of the stacks one launch covers (per_stack bytes per stack).
struct GradShape {
    int n_tiles, n_seg;
    int64_t cols;
    int64_t slots;  // checkpoint slots (one per wave of the persistent grid)
    size_t per_stack;          // partial sums and inverse-walk flags of one stack
    size_t per_stack_partial;  // the partial sums alone
    size_t slot_bytes, ckpt_bytes;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// max_slots caps the checkpoint slots, and with them the persistent grid (the
// launches then use fewer blocks); it must allow one block of either kernel.
static GradShape grad_shape(const tmm_rt_args* a, int64_t max_slots = INT64_MAX) {
    GradShape g;
    g.n_tiles = (int)ceil_div(a->n_wl, kWave);
    g.n_seg = (int)ceil_div(a->L, kSeg);
    g.cols = (int64_t)g.n_tiles * a->n_theta;
    g.per_stack_partial = (size_t)g.cols * a->L * 3 * sizeof(double);
    g.per_stack = g.per_stack_partial + (size_t)g.cols;
    // checkpoint slots of the persistent grid: blocks of kGradWaves (division-free
    // kernel) or kGradPairWaves (ratio-form kernel) waves, whichever needs more
    const int64_t tasks = g.cols * ceil_div(a->B, kGradWaves);
    const int64_t blocks = tasks < kGradMaxBlocks ? tasks : kGradMaxBlocks;
    const int64_t tasks8 = g.cols * ceil_div(a->B, kGradPairWaves);
    const int64_t blocks8 = tasks8 < kGradPairMaxBlocks ? tasks8 : kGradPairMaxBlocks;
    const int64_t slots = blocks * kGradWaves > blocks8 * kGradPairWaves ? blocks * kGradWaves : blocks8 * kGradPairWaves;
    g.slots = slots < max_slots ? slots : max_slots;
    g.slot_bytes = (size_t)(g.n_seg + 1) * kCkptDoubles * kWave * sizeof(double);
    g.ckpt_bytes = align256((size_t)g.slots * g.slot_bytes);
    return g;
}

static size_t ws_bytes(const GradShape& g, int64_t stacks) { return g.ckpt_bytes + align256((size_t)stacks * g.per_stack); }

// Stacks per launch for a workspace of `bytes` (0 if it is too small): all B,
// else a multiple of kGradWaves, at least min(B, kGradWaves).
static int64_t stacks_per_launch(const GradShape& g, int64_t B, size_t bytes) {
    if (bytes < g.ckpt_bytes) return 0;
    int64_t n = (int64_t)((bytes - g.ckpt_bytes) / g.per_stack);
    if (n >= B) return B;
    n = n / kGradWaves * kGradWaves;
    return n >= kGradWaves ? n : 0;
}

static int64_t preferred_stacks(const GradShape& g, int64_t B) {
    int64_t n = (int64_t)(kPartialCap / g.per_stack);
    if (n >= B) return B;
    n = n / kGradWaves * kGradWaves;
    const int64_t lo = B < kGradWaves ? B : kGradWaves;
    return n > lo ? n : lo;
}

// Resident blocks per CU of one kernel variant at this LDS size (cached).
template <int POL, bool TABLE>
static int occupancy_blocks(size_t lds) {
    static std::mutex mu;
    static std::map<size_t, int> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(lds);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, grad_kernel<POL, TABLE>, kGradBlock, lds) != hipSuccess || n < 1)
        n = 1;
    cache[lds] = n;
    return n;
}

template <int POL, int SEG, int N>
static int occupancy_pair_blocks(size_t lds) {
    static std::mutex mu;
    static std::map<size_t, int> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(lds);
    if (it != cache.end()) return it->second;
    // dynamic LDS above 64 KiB: raise the kernel's limit first
    (void)hipFuncSetAttribute((const void*)&grad_pair_kernel<POL, SEG, N>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    (void)hipGetLastError();
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, grad_pair_kernel<POL, SEG, N>, kGradPairBlock, lds) != hipSuccess ||
        n < 1)
        n = 1;
    cache[lds] = n;
    return n;
}

template <int POL, int SEG, int N>
static hipError_t launch_grad_pair(GradParams p, int n_cu, size_t lds, hipStream_t s) {
    p.n_tasks = p.n_tasks_pair;
    // The ratio-form stacks walk segments of SEG layers; stacks that fall back to
    // the division-free adjoint inside the same kernel keep p.n_seg segments of
    // kSeg, and p.n_seg + 1 stays the per-wave checkpoint stride (SEG >= kSeg).
    static_assert(SEG >= kSeg, "checkpoint slots are sized for segments of kSeg layers");
    p.n_seg_pair = (int)ceil_div(p.L, SEG);
    int64_t grid = (int64_t)n_cu * occupancy_pair_blocks<POL, SEG, N>(lds);
    if (grid > kGradPairMaxBlocks) grid = kGradPairMaxBlocks;
    if (grid > p.slots / kGradPairWaves) grid = p.slots / kGradPairWaves;
    if (grid > p.n_tasks) grid = p.n_tasks;
    p.per_block = ceil_div(p.n_tasks, grid);
    grid = ceil_div(p.n_tasks, p.per_block);
    hipLaunchKernelGGL((grad_pair_kernel<POL, SEG, N>), dim3((unsigned)grid), dim3(kGradPairBlock), lds, s, p);
    return hipGetLastError();
}

template <int POL, bool TABLE>
static hipError_t launch_grad(GradParams p, int n_cu, size_t lds, hipStream_t s) {
    int64_t grid = (int64_t)n_cu * occupancy_blocks<POL, TABLE>(lds);
    if (grid > kGradMaxBlocks) grid = kGradMaxBlocks;
    if (grid > p.slots / kGradWaves) grid = p.slots / kGradWaves;
    if (grid > p.n_tasks) grid = p.n_tasks;
    p.per_block = ceil_div(p.n_tasks, grid);
    grid = ceil_div(p.n_tasks, p.per_block);
    hipLaunchKernelGGL((grad_kernel<POL, TABLE>), dim3((unsigned)grid), dim3(kGradBlock), lds, s, p);
    return hipGetLastError();
}

template <int POL, int SEG, int WAVES, int N>
static hipError_t launch_grad_inv_t(GradParams p, int n_cu, hipStream_t s) {
    const size_t lds = grad_inv_lds_bytes(p.n_mat, SEG, WAVES);
    static std::mutex mu;
    static std::map<size_t, int> cache;
    int occ = 1;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(lds);
        if (it != cache.end()) {
            occ = it->second;
        } else {
            (void)hipFuncSetAttribute((const void*)&grad_inv_kernel<POL, SEG, WAVES, N>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            (void)hipGetLastError();
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, grad_inv_kernel<POL, SEG, WAVES, N>, WAVES * kWave,
                                                             lds) != hipSuccess ||
                occ < 1)
                occ = 1;
            cache[lds] = occ;
        }
    }
    p.n_tasks = p.n_tasks_pair = 0;
    const int64_t n_tasks = ((int64_t)p.n_tiles * p.n_theta) * ceil_div(p.b_end - p.b_begin, WAVES);
    p.n_tasks = n_tasks;
    int64_t grid = (int64_t)n_cu * occ;
    if (grid > n_tasks) grid = n_tasks;
    p.per_block = ceil_div(n_tasks, grid);
    grid = ceil_div(n_tasks, p.per_block);
    hipLaunchKernelGGL((grad_inv_kernel<POL, SEG, WAVES, N>), dim3((unsigned)grid), dim3(WAVES * kWave), lds, s, p);
    return hipGetLastError();
}

// Sixteen-wave blocks (four waves per SIMD at 128 VGPRs); stacks of 63-126
// layers (two registers of layer data) and seven-row tables in twelve-wave
// blocks.
static hipError_t launch_grad_inv(const GradParams& p, uint32_t pol, int n_cu, hipStream_t s) {
    static_assert(grad_inv_lds_bytes(kGradInvMaxMat - 1, 3, 16) <= 160 * 1024, "inverse-walk tables exceed LDS");
    static_assert(grad_inv_lds_bytes(kGradInvMaxMat, 3, 12) <= 160 * 1024, "inverse-walk tables exceed LDS");
    static_assert(kGradInvMaxMat * kGradInvMaxMat <= 64, "pair codes are 6 bits");
    if (p.L + 2 > kWave || grad_inv_lds_bytes(p.n_mat, 3, 16) > 160 * 1024) {
        if (pol == 1u) return launch_grad_inv_t<1, 3, 12, 2>(p, n_cu, s);
        if (pol == 2u) return launch_grad_inv_t<2, 3, 12, 2>(p, n_cu, s);
        return launch_grad_inv_t<3, 3, 12, 2>(p, n_cu, s);
    }
    if (pol == 1u) return launch_grad_inv_t<1, 3, 16, 1>(p, n_cu, s);
    if (pol == 2u) return launch_grad_inv_t<2, 3, 16, 1>(p, n_cu, s);
    return launch_grad_inv_t<3, 3, 16, 1>(p, n_cu, s);
}

template <int SEG, int N>
static hipError_t launch_grad_pair_pol(const GradParams& p, uint32_t pol, int n_cu, size_t lds, hipStream_t s) {
    if (pol == 1u) return launch_grad_pair<1, SEG, N>(p, n_cu, lds, s);
    if (pol == 2u) return launch_grad_pair<2, SEG, N>(p, n_cu, lds, s);
    return launch_grad_pair<3, SEG, N>(p, n_cu, lds, s);
}

// Checks and the cases without gradient kernels, shared by the entry points.
// *done = true: nothing (more) to launch, the returned status is final.
static tmm_status grad_prologue(const tmm_rt_args* a, const void* dl_dR, const void* dl_dT, void* grad_d,
                                void* grad_n, tmm_dtype dtype, hipStream_t s, const char* who, bool* done) {
    *done = true;
    tmm_status st = check_rt_args(a, who, false);
    if (st != TMM_OK) return st;
    if (dtype != TMM_F64) return fail(TMM_ERR_UNSUPPORTED, "%s: only TMM_F64 is implemented", who);
    if (a->r || a->t) return fail(TMM_ERR_INVALID_ARG, "%s: r and t outputs are not produced here", who);
    if (!dl_dR && !dl_dT) return fail(TMM_ERR_INVALID_ARG, "%s: dl_dR and dl_dT are both NULL", who);
    if (!grad_d && !grad_n) return fail(TMM_ERR_INVALID_ARG, "%s: grad_d and grad_n are both NULL", who);
    if (a->B == 0 || a->L == 0) return ok();
    if (a->flags & TMM_CHECK_FINITE) {
        const int P = a->pol_mask == 3u ? 2 : 1;
        const int64_t n_pts = (int64_t)a->B * P * a->n_theta * a->n_wl;
        st = check_rt_inputs<double>(a, static_cast<const double*>(dl_dR), n_pts, static_cast<const double*>(dl_dT),
                                     n_pts, who, s);
        if (st != TMM_OK) return st;
    }
    if (a->n_wl == 0 || a->n_theta == 0) {
        // no points: the gradients are zero
        const int64_t n_grad = (int64_t)a->B * a->L;
        (void)hipGetLastError();
        if (grad_d) hipLaunchKernelGGL(zero_fill, dim3(256), dim3(256), 0, s, (double*)grad_d, n_grad);
        if (grad_n) hipLaunchKernelGGL(zero_fill, dim3(256), dim3(256), 0, s, (double*)grad_n, 2 * n_grad);
        return check_launch(who);
    }
    *done = false;
    return ok();
}

// The gradient launches over `chunk` stacks at a time with the workspace
// laid out as g describes (checkpoints of g.slots waves, then partial sums).
static tmm_status grad_launch(const tmm_rt_args* a, const void* dl_dR, const void* dl_dT, void* grad_d,
                              void* grad_n, void* workspace, const GradShape& g, int64_t chunk, hipStream_t s,
                              const char* who) {
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1)
        return fail(TMM_ERR_HIP, "%s: no device", who);
    GradParams p;
    p.B = a->B;
    p.L = a->L;
    p.n_wl = a->n_wl;
    p.n_theta = a->n_theta;
    p.d = static_cast<const double*>(a->d);
    p.nk = static_cast<const double*>(a->nk);
    p.n_mat = a->n_mat;
    p.dispersive = a->dispersive;
    p.mat = a->mat;
    p.wl = static_cast<const double*>(a->wl);
    p.sin_t = static_cast<const double*>(a->sin_theta);
    p.cos_t = static_cast<const double*>(a->cos_theta);
    p.gR = static_cast<const double*>(dl_dR);
    p.gT = static_cast<const double*>(dl_dT);
    p.R_out = static_cast<double*>(a->R);
    p.T_out = static_cast<double*>(a->T);
    p.ws = static_cast<double*>(workspace);
    p.partial = reinterpret_cast<double*>(static_cast<unsigned char*>(workspace) + g.ckpt_bytes);
    p.redo = nullptr;
    unsigned char* const redo = reinterpret_cast<unsigned char*>(p.partial) + (size_t)chunk * g.per_stack_partial;
    p.n_tiles = g.n_tiles;
    p.n_seg = g.n_seg;
    p.n_seg_pair = g.n_seg;
    p.slots = g.slots;
    const bool table = a->mat != nullptr && a->n_mat <= kGradMaxTableMat;
    // ratio form: material ids, a small table, and the stack's layer data one
    // (L + 2 <= 64) or two (<= 128) per lane
    const bool pair = a->mat != nullptr && a->n_mat <= kGradPairMaxMat && a->L + 2 <= 2 * kWave;
    const bool two = a->L + 2 > kWave;
    // the inverse walk first (lossless columns) up to seven rows; the columns it
    // leaves go to the ratio-form kernel (at most five rows) or the division-free one
    const bool inv = a->mat != nullptr && a->n_mat <= kGradInvMaxMat && a->L + 2 <= 2 * kWave;
    // segments of five layers where their larger share buffer still fits the LDS
    // beside the table (at most four rows; 15 shares fill 60 reduction lanes), else of three
    const bool seg5 = pair && a->n_mat <= kGradPairLongSegMaxMat;
    const size_t lds = pair ? grad_pair_lds_bytes(a->n_mat, seg5 ? 5 : kSeg)
                            : phase_tab_bytes<double>() + (size_t)kGradWaves * kRed * kWave * sizeof(double) +
                                  (table ? (size_t)a->n_mat * kTabFields * kWave * sizeof(double2) : 0);
    (void)hipGetLastError();
    for (int64_t b0 = 0; b0 < a->B; b0 += chunk) {
        p.b_begin = (int)b0;
        p.b_end = (int)(b0 + chunk < a->B ? b0 + chunk : a->B);
        p.n_tasks = g.cols * ceil_div(p.b_end - p.b_begin, kGradWaves);
        p.n_tasks_pair = g.cols * ceil_div(p.b_end - p.b_begin, kGradPairWaves);
        hipError_t e = hipSuccess;
        p.redo = nullptr;
        if (inv) {
            // lossless columns by the inverse walk; the rest marked for the kernels below
            p.redo = redo;
            e = launch_grad_inv(p, a->pol_mask, n_cu, s);
            if (e != hipSuccess) return check_launch(who);
        }
        if (pair && seg5)
            e = two ? launch_grad_pair_pol<5, 2>(p, a->pol_mask, n_cu, lds, s)
                    : launch_grad_pair_pol<5, 1>(p, a->pol_mask, n_cu, lds, s);
        else if (pair)
            e = two ? launch_grad_pair_pol<kSeg, 2>(p, a->pol_mask, n_cu, lds, s)
                    : launch_grad_pair_pol<kSeg, 1>(p, a->pol_mask, n_cu, lds, s);
        else if (a->pol_mask == 1u)
            e = table ? launch_grad<1, true>(p, n_cu, lds, s) : launch_grad<1, false>(p, n_cu, lds, s);
        else if (a->pol_mask == 2u)
            e = table ? launch_grad<2, true>(p, n_cu, lds, s) : launch_grad<2, false>(p, n_cu, lds, s);
        else
            e = table ? launch_grad<3, true>(p, n_cu, lds, s) : launch_grad<3, false>(p, n_cu, lds, s);
        if (e != hipSuccess) return check_launch(who);
        const int64_t n = (int64_t)(p.b_end - p.b_begin) * a->L * 3;
        const int64_t blocks = ceil_div(n, 256) < 2048 ? ceil_div(n, 256) : 2048;
        hipLaunchKernelGGL(grad_reduce, dim3((unsigned)blocks), dim3(256), 0, s, p.partial, g.cols, n,
                           (int64_t)p.b_begin * a->L, static_cast<double*>(grad_d), static_cast<double*>(grad_n));
    }
    return check_launch(who);
}

// ---------------------------------------------------------------------------
// Workspace without allocation: a static device array per GPU, for callers
// that cannot allocate (graph capture, serving loops).  Host code reaches it
// only through the address hipGetSymbolAddress returns for the current device.
constexpr size_t kGradScratchBytes = (size_t)192 << 20;
static __device__ __align__(256) unsigned char scratch[kGradScratchBytes];
constexpr int kScratchMaxDevices = 64;

static unsigned char* scratch_on(int dev, hipError_t* err) {
    static std::mutex mu;
    static unsigned char* addr[kScratchMaxDevices] = {};
    std::lock_guard<std::mutex> g(mu);
    *err = hipSuccess;
    if (dev < 0 || dev >= kScratchMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    if (!addr[dev]) {
        void* ptr = nullptr;
        *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        addr[dev] = static_cast<unsigned char*>(ptr);
    }
    return addr[dev];
}

// Workspace shape inside the static scratch: the full persistent grid if its
// checkpoints fit in three quarters of it, else a grid capped to that share;
// the rest holds the partial sums of as many stacks as fit (several launches).
static bool scratch_shape(const tmm_rt_args* a, GradShape* g, int64_t* chunk) {
    *g = grad_shape(a);
    const size_t ckpt_cap = kGradScratchBytes / 4 * 3;
    if (g->ckpt_bytes > ckpt_cap) {
        const int64_t max_slots = (int64_t)(ckpt_cap / g->slot_bytes);
        if (max_slots < kGradPairWaves) return false;
        *g = grad_shape(a, max_slots);
    }
    *chunk = stacks_per_launch(*g, a->B, kGradScratchBytes);
    return *chunk > 0;
}

}  // namespace tmm

extern "C" {

size_t tmm_rt_grad_workspace_size(const tmm_rt_args* a) {
    if (!a || a->B <= 0 || a->L <= 0 || a->n_wl <= 0 || a->n_theta <= 0) return 0;
    const tmm::GradShape g = tmm::grad_shape(a);
    return tmm::ws_bytes(g, tmm::preferred_stacks(g, a->B));
}

size_t tmm_rt_grad_workspace_min_size(const tmm_rt_args* a) {
    if (!a || a->B <= 0 || a->L <= 0 || a->n_wl <= 0 || a->n_theta <= 0) return 0;
    const tmm::GradShape g = tmm::grad_shape(a);
    return tmm::ws_bytes(g, a->B < tmm::kGradWaves ? a->B : tmm::kGradWaves);
}

tmm_status tmm_rt_grad(const tmm_rt_args* a, const void* dl_dR, const void* dl_dT, void* grad_d, void* grad_n,
                       void* workspace, size_t workspace_bytes, tmm_dtype dtype, void* stream) {
    using tmm::fail;
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool done = true;
    tmm_status st = tmm::grad_prologue(a, dl_dR, dl_dT, grad_d, grad_n, dtype, s, "tmm_rt_grad", &done);
    if (st != TMM_OK || done) return st;
    const tmm::GradShape g = tmm::grad_shape(a);
    const int64_t chunk = workspace ? tmm::stacks_per_launch(g, a->B, workspace_bytes) : 0;
    if (chunk == 0)
        return fail(TMM_ERR_WORKSPACE, "tmm_rt_grad: workspace of at least %zu bytes needed (%zu preferred), %zu given",
                    tmm::ws_bytes(g, a->B < tmm::kGradWaves ? a->B : tmm::kGradWaves),
                    tmm::ws_bytes(g, tmm::preferred_stacks(g, a->B)), workspace ? workspace_bytes : (size_t)0);
    return tmm::grad_launch(a, dl_dR, dl_dT, grad_d, grad_n, workspace, g, chunk, s, "tmm_rt_grad");
}

size_t tmm_rt_grad_noalloc_scratch_bytes(void) { return tmm::kGradScratchBytes; }

tmm_status tmm_rt_grad_noalloc(const tmm_rt_args* a, const void* dl_dR, const void* dl_dT, void* grad_d,
                               void* grad_n, tmm_dtype dtype, void* stream) {
    using tmm::fail;
    hipStream_t s = static_cast<hipStream_t>(stream);
    bool done = true;
    tmm_status st = tmm::grad_prologue(a, dl_dR, dl_dT, grad_d, grad_n, dtype, s, "tmm_rt_grad_noalloc", &done);
    if (st != TMM_OK || done) return st;
    tmm::GradShape g;
    int64_t chunk = 0;
    if (!tmm::scratch_shape(a, &g, &chunk))
        return fail(TMM_ERR_WORKSPACE,
                    "tmm_rt_grad_noalloc: B=%d L=%d n_wl=%d n_theta=%d needs more than the %zu-byte static scratch "
                    "(use tmm_rt_grad with a workspace)",
                    a->B, a->L, a->n_wl, a->n_theta, tmm::kGradScratchBytes);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TMM_ERR_HIP, "tmm_rt_grad_noalloc: no device");
    hipError_t e = hipSuccess;
    unsigned char* ws = tmm::scratch_on(dev, &e);
    if (!ws)
        return fail(TMM_ERR_HIP, "tmm_rt_grad_noalloc: static scratch not found on device %d: %s", dev,
                    hipGetErrorString(e));
    return tmm::grad_launch(a, dl_dR, dl_dT, grad_d, grad_n, ws, g, chunk, s, "tmm_rt_grad_noalloc");
}

}  // extern "C"
