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
//           ascending), form dl/dd_j and dl/dn_j, reduce them over the wave's
//           64 wavelengths and add them to the outputs with float64 atomics.
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
#include <math.h>

#include "tmm_device.hpp"
#include "tmm_host.hpp"

namespace tmm {

constexpr int kGradBlock = 256;
constexpr int kGradWaves = kGradBlock / kWave;
constexpr int kSeg = 4;                  // layers per checkpoint segment
constexpr int kGradMaxTableMat = 16;
constexpr int kCkptDoubles = 8;          // (sigma, tau) of s and p, complex
constexpr int kGradMaxBlocks = 2048;     // bounds the workspace

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
    double* grad_d;
    double* grad_n;
    double* ws;
    int n_tiles, chunk, n_seg;
    int use_table;
};

struct GLayer {
    cx<double> q, e, n;
};

__device__ __forceinline__ GLayer glayer_from(double nr, double ni, double kx) {
    const Medium m = make_medium(nr, ni, kx);
    GLayer g;
    g.q = {m.qr, m.qi};
    g.e = {m.er, m.ei};
    g.n = {nr, ni};
    return g;
}

// Layer values: from the LDS table (material ids, small table, same ambient)
// or computed in place.
struct GSource {
    const double2* tab;  // [m][3][lane] double2, or NULL
    const double* nk;
    const int32_t* mrow;  // NULL: implicit rows
    int64_t base;
    int n_mat, dispersive, n_wl, i, lane;
    double kx;
    __device__ __forceinline__ int row(int j) const {
        if (!mrow) return (int)(base + j);
        const int m = mrow[j];
        return m < 0 ? 0 : (m >= n_mat ? n_mat - 1 : m);
    }
    __device__ __forceinline__ bool row_bad(int j) const {
        return mrow ? (uint32_t)mrow[j] >= (uint32_t)n_mat : false;
    }
    __device__ __forceinline__ GLayer get(int j) const {
        if (tab) {
            const double2* blk = tab + (size_t)row(j) * 3 * kWave + lane;
            const double2 a = blk[0], b = blk[kWave], c = blk[2 * kWave];
            return GLayer{{a.x, a.y}, {b.x, b.y}, {c.x, c.y}};
        }
        const int64_t r = mrow ? (int64_t)row(j) : base + j;
        double nr, ni;
        load_n(nk, dispersive, n_wl, r, i, nr, ni);
        return glayer_from(nr, ni, kx);
    }
};

struct State {
    cx<double> ss, ts, sp, tp;
};

template <int POL>
__device__ __forceinline__ void fwd_step(State& z, const GLayer& cur, const GLayer& nxt, const cx<double>& E) {
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

__device__ __forceinline__ cx<double> cconj(cx<double> a) { return {a.re, -a.im}; }
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <int POL>
__device__ void grad_stack(const GradParams& p, const GSource& src, const Ambient& amb, int b, int k, int i,
                           bool active, bool lane_ok, double* ws) {
    const int L = p.L;
    constexpr int P = (POL == 3) ? 2 : 1;
    const double lam = p.wl[i];
    const double c4lam = 4.0 / lam;           // phi = c4lam d q (half-turns of 2 delta)
    const double two_pi_lam = 2.0 * M_PI / lam;
    const double* drow = p.d + (int64_t)b * L;
    const int lane = src.lane;
    bool bad = src.row_bad(0) || src.row_bad(L + 1);
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
    const GLayer sub = src.get(L + 1);
    GLayer nxt = sub;
    for (int s = 0; s < p.n_seg; ++s) {
        const int top = L - s * kSeg;
        const int lo = top - kSeg + 1 > 1 ? top - kSeg + 1 : 1;
        for (int j = top; j >= lo; --j) {
            const double dj = drow[j - 1];
            bad = bad || bad_thickness(dj) || src.row_bad(j);
            const GLayer cur = src.get(j);
            const double cd = dj * c4lam;
            const double phi = cd * cur.q.im;
            const bool lossy = __any(phi != 0.0);
            const cx<double> E = phase_factor<double>(cd * cur.q.re, phi, lossy);
            fwd_step<POL>(z, cur, nxt, E);
            pis *= cnorm(cur.q);
            pip *= cnorm(cur.e);
            S += phi;
            nxt = cur;
        }
        if (POL & 1) renorm_pair(z.ss, z.ts, es);
        if (POL & 2) renorm_pair(z.sp, z.tp, ep);
        renorm_one(pis, epis);
        renorm_one(pip, epip);
        save(s + 1, z);
    }
    const GLayer first = nxt;
    const double eS = exp2(S * kNegPiLog2e);
    const int two_L1 = 2 * (L + 1);
    const bool valid = lane_ok && !bad;
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
    for (int s = p.n_seg - 1; s >= 0; --s) {
        const int top = L - s * kSeg;
        const int lo = top - kSeg + 1 > 1 ? top - kSeg + 1 : 1;
        const int nst = top - lo + 1;
        State zin[kSeg];
        cx<double> Es[kSeg];
        State zz = load(s);
        GLayer nx = (top == L) ? sub : src.get(top + 1);
#pragma unroll
        for (int t = 0; t < kSeg; ++t) {
            if (t < nst) {
                const int j = top - t;
                const GLayer cur = src.get(j);
                const double cd = drow[j - 1] * c4lam;
                const double phi = cd * cur.q.im;
                const bool lossy = __any(phi != 0.0);
                Es[t] = phase_factor<double>(cd * cur.q.re, phi, lossy);
                zin[t] = zz;
                fwd_step<POL>(zz, cur, nx, Es[t]);
                nx = cur;
            }
        }
        // the forward pass renormalised the segment's end state; undo on the adjoint
        if (POL & 1) {
            const int e = pair_exp(zz.ss, zz.ts);
            sb_s = cscale(ldexp(1.0, -e), sb_s);
            tb_s = cscale(ldexp(1.0, -e), tb_s);
        }
        if (POL & 2) {
            const int e = pair_exp(zz.sp, zz.tp);
            sb_p = cscale(ldexp(1.0, -e), sb_p);
            tb_p = cscale(ldexp(1.0, -e), tb_p);
        }
#pragma unroll
        for (int t = kSeg - 1; t >= 0; --t) {
            if (t < nst) {
                const int j = top - t;
                const GLayer cur = src.get(j);
                const GLayer nxj = (j == L) ? sub : src.get(j + 1);
                const double dj = drow[j - 1];
                cx<double> Eb = {0.0, 0.0};
                cx<double> qb = pend_q, eb = pend_e;
                if (POL & 1) {
                    cx<double> alphab, betab;
                    adj_step(zin[t].ss, zin[t].ts, cur.q, nxj.q, Es[t], sb_s, tb_s, alphab, betab, Eb);
                    qb = cadd(qb, alphab);  // alpha_j = q_j
                    pend_q = betab;         // beta_j = q_{j+1}
                    qb = cadd(qb, cscale(2.0 * cT_s / cnorm(cur.q), cur.q));  // T through |q_j|^2
                }
                if (POL & 2) {
                    cx<double> alphab, betab;
                    adj_step(zin[t].sp, zin[t].tp, nxj.e, cur.e, Es[t], sb_p, tb_p, alphab, betab, Eb);
                    eb = cadd(eb, betab);   // beta_j = eta_j
                    pend_e = alphab;        // alpha_j = eta_{j+1}
                    eb = cadd(eb, cscale(2.0 * cT_p / cnorm(cur.e), cur.e));  // T through |eta_j|^2
                }
                // deltab = -2i conj(E) Eb - 2i cT  (chain and e^{-2 Im sum delta})
                const cx<double> cE = cmulc(Es[t], Eb);
                const cx<double> db = {2.0 * cE.im, -2.0 * cE.re - 2.0 * cT};
                const double gd = two_pi_lam * (db.re * cur.q.re + db.im * cur.q.im);
                qb = cadd(qb, cscale(two_pi_lam * dj, db));
                // nb = conj(n/q) qb + conj((n/q)(2 - eta/q)) etab
                const cx<double> nq = cdiv(cur.n, cur.q);
                const cx<double> eq = cdiv(cur.e, cur.q);
                const cx<double> de = cmul(nq, cx<double>{2.0 - eq.re, -eq.im});
                const cx<double> nb = cadd(cmulc(nq, qb), cmulc(de, eb));
                const double s0 = wave_sum(gd);
                const double s1 = wave_sum(nb.re);
                const double s2 = wave_sum(nb.im);
                if (lane == 0) {
                    const int64_t g = (int64_t)b * L + (j - 1);
                    if (p.grad_d) atomicAdd(p.grad_d + g, s0);
                    if (p.grad_n) {
                        atomicAdd(p.grad_n + 2 * g, s1);
                        atomicAdd(p.grad_n + 2 * g + 1, s2);
                    }
                }
            }
        }
    }
}

template <int POL>
__global__ void __launch_bounds__(kGradBlock) grad_kernel(GradParams p) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    int bid = blockIdx.x;
    const int tile = bid % p.n_tiles;
    bid /= p.n_tiles;
    const int k = bid % p.n_theta;
    bid /= p.n_theta;
    const int b0 = bid * p.chunk;
    const int b1 = min(b0 + p.chunk, p.B);
    const int i_raw = tile * kWave + lane;
    const bool active = i_raw < p.n_wl;
    const int i = active ? i_raw : p.n_wl - 1;
    const double lam = p.wl[i];
    const bool lam_ok = lam > 0.0 && lam < __builtin_inf();
    const double st = p.sin_t[k], ct = p.cos_t[k];
    const int L2 = p.L + 2;
    double* ws = p.ws + ((size_t)blockIdx.x * kGradWaves + wave) * (size_t)(p.n_seg + 1) * kCkptDoubles * kWave;

    double2* tab = nullptr;
    int amb_row = 0;
    Ambient amb_t;
    if (p.use_table) {
        amb_row = p.mat[(int64_t)b0 * L2];
        amb_row = amb_row < 0 ? 0 : (amb_row >= p.n_mat ? p.n_mat - 1 : amb_row);
        double n0r, n0i;
        load_n(p.nk, p.dispersive, p.n_wl, amb_row, i, n0r, n0i);
        amb_t = make_ambient(n0r, n0i, st, ct);
        tab = reinterpret_cast<double2*>(smem);
        for (int m = wave; m < p.n_mat; m += kGradWaves) {
            double nr, ni;
            load_n(p.nk, p.dispersive, p.n_wl, m, i, nr, ni);
            const GLayer g = glayer_from(nr, ni, amb_t.kx);
            double2* blk = tab + (size_t)m * 3 * kWave + lane;
            blk[0] = make_double2(g.q.re, g.q.im);
            blk[kWave] = make_double2(g.e.re, g.e.im);
            blk[2 * kWave] = make_double2(g.n.re, g.n.im);
        }
        __syncthreads();
    }
    for (int b = b0 + wave; b < b1; b += kGradWaves) {
        const int32_t* mrow = p.mat ? p.mat + (int64_t)b * L2 : nullptr;
        GSource src;
        src.nk = p.nk;
        src.mrow = mrow;
        src.base = (int64_t)b * L2;
        src.n_mat = p.n_mat;
        src.dispersive = p.dispersive;
        src.n_wl = p.n_wl;
        src.i = i;
        src.lane = lane;
        const int a_row = src.row(0);
        Ambient amb;
        if (p.use_table && mrow[0] == amb_row) {
            amb = amb_t;
            src.tab = tab;
        } else {
            double n0r, n0i;
            load_n(p.nk, p.dispersive, p.n_wl, a_row, i, n0r, n0i);
            amb = make_ambient(n0r, n0i, st, ct);
            src.tab = nullptr;
        }
        src.kx = amb.kx;
        grad_stack<POL>(p, src, amb, b, k, i, active, lam_ok && amb.ok, ws);
    }
}

__global__ void zero_fill(double* x, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) x[t] = 0.0;
}

struct GradShape {
    int n_tiles, chunk, n_seg;
    int64_t blocks;
    size_t ws_bytes;
};

static GradShape grad_shape(const tmm_rt_args* a) {
    GradShape g;
    g.n_tiles = (int)ceil_div(a->n_wl, kWave);
    g.n_seg = (int)ceil_div(a->L, kSeg);
    const int64_t cols = (int64_t)g.n_tiles * a->n_theta;
    int64_t chunk = ceil_div((int64_t)a->B * cols, kGradMaxBlocks);
    chunk = ceil_div(chunk, kGradWaves) * kGradWaves;
    if (chunk < kGradWaves) chunk = kGradWaves;
    g.chunk = (int)chunk;
    g.blocks = cols * ceil_div(a->B, chunk);
    g.ws_bytes = (size_t)g.blocks * kGradWaves * (size_t)(g.n_seg + 1) * kCkptDoubles * kWave * sizeof(double);
    return g;
}

}  // namespace tmm

extern "C" {

size_t tmm_rt_grad_workspace_size(const tmm_rt_args* a) {
    if (!a || a->B <= 0 || a->L <= 0 || a->n_wl <= 0 || a->n_theta <= 0) return 0;
    return tmm::grad_shape(a).ws_bytes;
}

tmm_status tmm_rt_grad(const tmm_rt_args* a, const void* dl_dR, const void* dl_dT, void* grad_d, void* grad_n,
                       void* workspace, size_t workspace_bytes, tmm_dtype dtype, void* stream) {
    using tmm::fail;
    tmm_status st = tmm::check_rt_args(a, "tmm_rt_grad", false);
    if (st != TMM_OK) return st;
    if (dtype != TMM_F64) return fail(TMM_ERR_UNSUPPORTED, "tmm_rt_grad: only TMM_F64 is implemented");
    if (a->r || a->t) return fail(TMM_ERR_INVALID_ARG, "tmm_rt_grad: r and t outputs are not produced here");
    if (!dl_dR && !dl_dT) return fail(TMM_ERR_INVALID_ARG, "tmm_rt_grad: dl_dR and dl_dT are both NULL");
    if (!grad_d && !grad_n) return fail(TMM_ERR_INVALID_ARG, "tmm_rt_grad: grad_d and grad_n are both NULL");
    if (a->B == 0 || a->L == 0) return tmm::ok();
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n_grad = (int64_t)a->B * a->L;
    if (a->n_wl == 0 || a->n_theta == 0) {
        // no points: the gradients are zero
        (void)hipGetLastError();
        if (grad_d) hipLaunchKernelGGL(tmm::zero_fill, dim3(256), dim3(256), 0, s, (double*)grad_d, n_grad);
        if (grad_n) hipLaunchKernelGGL(tmm::zero_fill, dim3(256), dim3(256), 0, s, (double*)grad_n, 2 * n_grad);
        return tmm::check_launch("tmm_rt_grad");
    }
    const tmm::GradShape g = tmm::grad_shape(a);
    if (!workspace || workspace_bytes < g.ws_bytes)
        return fail(TMM_ERR_WORKSPACE, "tmm_rt_grad: workspace of %zu bytes needed, %zu given", g.ws_bytes,
                    workspace_bytes);
    tmm::GradParams p;
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
    p.grad_d = static_cast<double*>(grad_d);
    p.grad_n = static_cast<double*>(grad_n);
    p.ws = static_cast<double*>(workspace);
    p.n_tiles = g.n_tiles;
    p.chunk = g.chunk;
    p.n_seg = g.n_seg;
    p.use_table = (a->mat != nullptr && a->n_mat <= tmm::kGradMaxTableMat) ? 1 : 0;
    const size_t lds = p.use_table ? (size_t)a->n_mat * 3 * tmm::kWave * sizeof(double2) : 0;
    (void)hipGetLastError();
    if (grad_d) hipLaunchKernelGGL(tmm::zero_fill, dim3(256), dim3(256), 0, s, p.grad_d, n_grad);
    if (grad_n) hipLaunchKernelGGL(tmm::zero_fill, dim3(256), dim3(256), 0, s, p.grad_n, 2 * n_grad);
    const dim3 grid((unsigned)g.blocks), block(tmm::kGradBlock);
    if (a->pol_mask == 1u)
        hipLaunchKernelGGL(tmm::grad_kernel<1>, grid, block, lds, s, p);
    else if (a->pol_mask == 2u)
        hipLaunchKernelGGL(tmm::grad_kernel<2>, grid, block, lds, s, p);
    else
        hipLaunchKernelGGL(tmm::grad_kernel<3>, grid, block, lds, s, p);
    return tmm::check_launch("tmm_rt_grad");
}

}  // extern "C"
