// Forward transfer-matrix kernels (gfx950) and the tmm_rt entry point.
//
// Work decomposition: one lane = one (stack, wavelength, angle) with both
// polarisations, so the pol-independent work (q_j, the phase factor e^{2 i delta_j})
// is done once for s and p.  A 256-thread workgroup covers one angle and a
// tile of 64 consecutive wavelengths (lanes = wavelengths, so every store of a
// wave is 64 consecutive elements), and its four waves walk a chunk of stacks,
// one stack per wave at a time: the stack index, the layer loop, thicknesses
// and material ids are wave-uniform and stay on the scalar unit.
//
// Three ways to obtain the per-layer values of the layer loop:
//   pair   : when a material-id array is given and the table is small enough
//            (at most 6 materials in double, 8 in float), the workgroup
//            tabulates, for its 64 wavelengths, the ratios q_{j+1}/q_j,
//            eta_{j+1}/eta_j of every ordered pair of materials and the phase
//            coefficient 4 q_j / lambda in LDS, and the layer loop runs the
//            ratio form of the recursion (tmm_chain.hpp) on them: one LDS row
//            per step, no complex products beyond the recursion itself.  The
//            workgroup is as large as the LDS allows (up to 16 waves on one
//            CU).  A stack falls back to the inline source below when the
//            ratios are out of range, its ambient differs, or a phase is beyond
//            the range of the fast argument reduction; that path is kept out of
//            the layer-loop registers' way (it is rare and needs no table).
//   table  : when a material-id array is given and the table has at most
//            kMaxTableMat rows, the workgroup computes q, eta, |q|^2, |eta|^2 of
//            every material for its 64 wavelengths once (complex sqrt and one
//            division per entry) into LDS, and the layer loop only reads them.
//            Stacks whose ambient differs from the one the table was built for
//            fall back to the inline source.
//   inline : otherwise each step loads n_j and computes q_j, eta_j itself.
// The recursion itself is described in tmm_device.hpp.
#include <math.h>
#include <string.h>

#include <atomic>

#include "tmm_chain.hpp"
#include "tmm_check.hpp"
#include "tmm_device.hpp"
#include "tmm_host.hpp"

namespace tmm {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxTableMat = 16;

template <typename R>
struct FwdParams {
    int B, L, n_wl, n_theta;
    const R* d;
    const R* nk;
    int n_mat, dispersive;
    const int32_t* mat;
    const R* wl;
    const R* sin_t;
    const R* cos_t;
    R* R_out;
    R* T_out;
    R* r_out;
    R* t_out;
    int n_tiles, chunk;
};

template <typename R>
__host__ __device__ constexpr size_t table_bytes(int n_mat) {
    // phase table, media table, lossy flags
    return phase_tab_bytes<R>() + (size_t)n_mat * kWave * Table<R>::kEntryBytes + 4 * kMaxTableMat;
}

// Sources of per-layer values for the chain.  Row ids are wave-uniform.
template <typename R>
struct TableSource {
    const Table<R>* tab;
    const int32_t* mrow;
    int lane, n_mat;
    uint32_t lossy_mask;
    __device__ __forceinline__ bool row_bad(int j) const { return (uint32_t)mrow[j] >= (uint32_t)n_mat; }
    __device__ __forceinline__ Layer<R> layer(int j, bool& lossy) const {
        int m = mrow[j];
        m = m < 0 ? 0 : (m >= n_mat ? n_mat - 1 : m);
        lossy = (lossy_mask >> m) & 1u;
        return tab->get(m, lane);
    }
};

template <typename R>
struct InlineSource {
    const R* nk;
    const int32_t* mrow;   // NULL: implicit rows implicit_base + j
    int64_t implicit_base;
    int n_mat, dispersive, n_wl, i;
    double kx;
    __device__ __forceinline__ bool row_bad(int j) const {
        return mrow ? (uint32_t)mrow[j] >= (uint32_t)n_mat : false;
    }
    __device__ __forceinline__ Layer<R> layer(int j, bool& lossy) const {
        int64_t row;
        if (mrow) {
            int m = mrow[j];
            row = m < 0 ? 0 : (m >= n_mat ? n_mat - 1 : m);
        } else {
            row = implicit_base + j;
        }
        double nr, ni;
        load_n(nk, dispersive, n_wl, row, i, nr, ni);
        const Medium md = make_medium(nr, ni, kx);
        lossy = __any(md.qi != 0.0);
        return to_layer<R>(md);
    }
};

}  // namespace tmm

namespace tmm {

template <typename R>
__device__ __forceinline__ void store_point(const FwdParams<R>& p, int b, int k, int i, int pol_slot,
                                            int P, const PointOut& o, bool valid) {
    const int64_t idx = (((int64_t)b * P + pol_slot) * p.n_theta + k) * p.n_wl + i;
    const double nan = __builtin_nan("");
    if (p.R_out) p.R_out[idx] = (R)(valid ? o.R : nan);
    if (p.T_out) p.T_out[idx] = (R)(valid ? o.T : nan);
    if (p.r_out) {
        p.r_out[2 * idx] = (R)(valid ? o.r.re : nan);
        p.r_out[2 * idx + 1] = (R)(valid ? o.r.im : nan);
    }
    if (p.t_out) {
        p.t_out[2 * idx] = (R)(valid ? o.t.re : nan);
        p.t_out[2 * idx + 1] = (R)(valid ? o.t.im : nan);
    }
}

// One stack for this lane's (wavelength, angle): layer loop from the substrate
// to the ambient, then extraction and coalesced stores.
template <typename R, int POL, bool AMP, class Src>
__device__ __forceinline__ void run_stack(const FwdParams<R>& p, const Src& src, const Ambient& amb,
                                          int b, int k, int i, bool active, bool lane_ok,
                                          double c4lam, double nsub_r, double nsub_i, const TabPhase<R>& phase) {
    const int L = p.L;
    const R* drow = p.d + (int64_t)b * L;
    bool bad = src.row_bad(0) || src.row_bad(L + 1);
    bool lossy;
    const Layer<R> sub = src.layer(L + 1, lossy);
    Layer<R> nxt = sub;
    Chain<R, POL, AMP> c;
    c.init();
    int cnt = 0;
    for (int j = L; j >= 1; --j) {
        const R dj = drow[j - 1];
        bad = bad || bad_thickness(dj) || src.row_bad(j);
        const Layer<R> cur = src.layer(j, lossy);
        c.step(cur, nxt, (double)dj * c4lam, lossy, phase);
        nxt = cur;
        if (++cnt == RenormPeriod<R>::value) {
            cnt = 0;
            c.renorm();
        }
    }
    c.renorm();
    PointOut out[2];
    finish<R, POL, AMP>(c, amb, nxt, sub, nsub_r, nsub_i, L, out, phase);
    if (active) {
        const bool valid = lane_ok && !bad;
        constexpr int P = (POL == 3) ? 2 : 1;
        store_point(p, b, k, i, 0, P, out[0], valid);
        if (POL == 3) store_point(p, b, k, i, 1, P, out[1], valid);
    }
}

// Table path: one stack.  The layers are read in chunks of kWave, one per lane
// (coalesced), and the layer loop broadcasts them from the owning lane; whole
// renormalisation blocks are unrolled, so no value is copied between steps.
template <typename R, int POL, bool AMP>
__device__ __forceinline__ void run_stack_table(const FwdParams<R>& p, const Table<R>& tab, uint32_t lossy_mask,
                                                const Ambient& amb, int b, int k, int i, int lane,
                                                bool active, bool lane_ok, double c4lam, double nsub_r,
                                                double nsub_i, const TabPhase<R>& phase) {
    const int L = p.L;
    const int n_mat = p.n_mat;
    const R* drow = p.d + (int64_t)b * L;
    const int32_t* mrow = p.mat + (int64_t)b * (L + 2);
    const int m_sub_raw = mrow[L + 1];
    bool bad = (uint32_t)m_sub_raw >= (uint32_t)n_mat;
    const int m_sub = bad ? 0 : m_sub_raw;
    const Layer<R> sub = tab.get(m_sub, lane);
    // the layer below the current one is carried as its table row (a scalar) and
    // re-read from LDS, so no medium values are copied between registers per step
    int nxt_row = m_sub;
    Chain<R, POL, AMP> c;
    c.init();
    static_assert(kWave % RenormPeriod<R>::value == 0, "chunks must hold whole renormalisation blocks");
    constexpr int RP = RenormPeriod<R>::value;
    for (int top = L; top >= 1; top -= kWave) {
        const int lo = top - kWave + 1 > 1 ? top - kWave + 1 : 1;
        // lane l holds layer lo + l: thickness and table row | lossy flag << 16
        const int j = lo + lane;
        double my_d = 0.0;
        int my_code = 0;
        bool lane_bad = false;
        if (j <= top) {
            const R dj = drow[j - 1];
            const int m = mrow[j];
            const bool mbad = (uint32_t)m >= (uint32_t)n_mat;
            lane_bad = mbad || bad_thickness(dj);
            const int mc = mbad ? 0 : m;
            my_d = (double)dj;
            my_code = mc | (int)(((lossy_mask >> mc) & 1u) << 16);
        }
        bad = bad || __any(lane_bad);
        // one step: layer jj's values broadcast from lane jj - lo
        auto step = [&](int jj) {
            const int sl = jj - lo;
            const int code = __builtin_amdgcn_readlane(my_code, sl);
            const double dj = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(my_d), sl),
                                               __builtin_amdgcn_readlane(__double2loint(my_d), sl));
            const Layer<R> cur = tab.get(code & 0xffff, lane);
            c.step(cur, tab.get(nxt_row, lane), dj * c4lam, (code >> 16) != 0, phase);
            nxt_row = code & 0xffff;
        };
        // blocks of RP steps; chunks start at multiples of kWave steps, so the
        // renormalisation points are those of a running step count
        for (int bt = top; bt >= lo; bt -= RP) {
            if (bt - lo >= RP - 1) {
#pragma unroll 2
                for (int u = 0; u < RP; ++u) step(bt - u);
                c.renorm();
            } else {
                for (int jj = bt; jj >= lo; --jj) step(jj);
            }
        }
    }
    c.renorm();
    PointOut out[2];
    finish<R, POL, AMP>(c, amb, tab.get(nxt_row, lane), sub, nsub_r, nsub_i, L, out, phase);
    if (active) {
        const bool valid = lane_ok && !bad;
        constexpr int P = (POL == 3) ? 2 : 1;
        store_point(p, b, k, i, 0, P, out[0], valid);
        if (POL == 3) store_point(p, b, k, i, 1, P, out[1], valid);
    }
}

template <typename R, int POL, bool AMP, bool TABLE>
__global__ void __launch_bounds__(kBlock) fwd_kernel(FwdParams<R> p) {
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
    const int i = active ? i_raw : p.n_wl - 1;  // ragged tail: compute a valid point, store nothing
    const double lam = (double)p.wl[i];
    const bool lam_ok = lam > 0.0 && lam < __builtin_inf();
    const double c4lam = 4.0 / lam;  // phi_j = 4 d_j q_j / lambda half-turns = 2 delta_j / pi
    const double st = (double)p.sin_t[k], ct = (double)p.cos_t[k];
    const int L2 = p.L + 2;
    fill_phase_tab<R>(smem, threadIdx.x, kBlock);
    const TabPhase<R> phase = phase_of<R>(smem);
    unsigned char* const lds = smem + phase_tab_bytes<R>();
    if (!TABLE) __syncthreads();

    if (TABLE) {
        int amb_row = p.mat[(int64_t)b0 * L2];
        amb_row = amb_row < 0 ? 0 : (amb_row >= p.n_mat ? p.n_mat - 1 : amb_row);
        double n0r, n0i;
        load_n(p.nk, p.dispersive, p.n_wl, amb_row, i, n0r, n0i);
        const Ambient amb = make_ambient(n0r, n0i, st, ct);
        Table<R> tab(lds, p.n_mat);
        int* flags = reinterpret_cast<int*>(lds + (size_t)p.n_mat * kWave * Table<R>::kEntryBytes);
        for (int m = wave; m < p.n_mat; m += kWavesPerBlock) {
            double nr, ni;
            load_n(p.nk, p.dispersive, p.n_wl, m, i, nr, ni);
            const Medium md = make_medium(nr, ni, amb.kx);
            tab.put(m, lane, md);
            const bool lossy = __any(md.qi != 0.0);
            if (lane == 0) flags[m] = lossy ? 1 : 0;
        }
        __syncthreads();
        uint32_t mask = 0;
        for (int m = 0; m < p.n_mat; ++m) mask |= (uint32_t)flags[m] << m;
        mask = __builtin_amdgcn_readfirstlane(mask);
        for (int b = b0 + wave; b < b1; b += kWavesPerBlock) {
            const int32_t* mrow = p.mat + (int64_t)b * L2;
            int sub_row = mrow[p.L + 1];
            sub_row = sub_row < 0 ? 0 : (sub_row >= p.n_mat ? p.n_mat - 1 : sub_row);
            double nsr = 0.0, nsi = 0.0;
            if (AMP) load_n(p.nk, p.dispersive, p.n_wl, sub_row, i, nsr, nsi);
            if (mrow[0] == amb_row) {
                run_stack_table<R, POL, AMP>(p, tab, mask, amb, b, k, i, lane, active,
                                             lam_ok && amb.ok, c4lam, nsr, nsi, phase);
            } else {
                int a_row = mrow[0];
                a_row = a_row < 0 ? 0 : (a_row >= p.n_mat ? p.n_mat - 1 : a_row);
                double ar, ai;
                load_n(p.nk, p.dispersive, p.n_wl, a_row, i, ar, ai);
                const Ambient amb_b = make_ambient(ar, ai, st, ct);
                InlineSource<R> src{p.nk, mrow, 0, p.n_mat, p.dispersive, p.n_wl, i, amb_b.kx};
                run_stack<R, POL, AMP>(p, src, amb_b, b, k, i, active, lam_ok && amb_b.ok, c4lam, nsr, nsi, phase);
            }
        }
    } else {
        for (int b = b0 + wave; b < b1; b += kWavesPerBlock) {
            const int32_t* mrow = p.mat ? p.mat + (int64_t)b * L2 : nullptr;
            const int64_t base = (int64_t)b * L2;
            auto row_of = [&](int j) -> int64_t {
                if (!mrow) return base + j;
                const int m = mrow[j];
                return m < 0 ? 0 : (m >= p.n_mat ? p.n_mat - 1 : m);
            };
            double n0r, n0i;
            load_n(p.nk, p.dispersive, p.n_wl, row_of(0), i, n0r, n0i);
            const Ambient amb = make_ambient(n0r, n0i, st, ct);
            double nsr = 0.0, nsi = 0.0;
            if (AMP) load_n(p.nk, p.dispersive, p.n_wl, row_of(p.L + 1), i, nsr, nsi);
            InlineSource<R> src{p.nk, mrow, base, p.n_mat, p.dispersive, p.n_wl, i, amb.kx};
            run_stack<R, POL, AMP>(p, src, amb, b, k, i, active, lam_ok && amb.ok, c4lam, nsr, nsi, phase);
        }
    }
}

// ---------------------------------------------------------------------------
// Pair path.  LDS: phase table | media Table<R> (finish, fallback) | one block
// per ordered material pair (m, m') | flags.  A block holds, for the 64 lanes,
// rho_s = q_{m'}/q_m, rho_p = eta_{m'}/eta_m and (cre, cim) with
// phi = d (cre / 256 + i cim / kNegPiLog2e): cre = 1024 Re(q_m)/lambda (the
// phase per unit d in units of 1/256 half-turn) and cim = kNegPiLog2e 4 Im(q_m)/lambda
// (the base-2 attenuation exponent per unit d).
template <typename R> struct PairTab;

template <>
struct PairTab<double> {
    static constexpr int kBlockBytes = 3 * kWave * 16;  // rho_s[64], rho_p[64], (cre, cim)[64]
    __device__ static void put(unsigned char* blk, int lane, cx<double> rs, cx<double> rp, double cre, double cim) {
        double2* b = reinterpret_cast<double2*>(blk);
        b[lane] = make_double2(rs.re, rs.im);
        b[kWave + lane] = make_double2(rp.re, rp.im);
        b[2 * kWave + lane] = make_double2(cre, cim);
    }
    // `at` is the block address plus lane * 16
    __device__ __forceinline__ static void get(const unsigned char* at, cx<double>& rs, cx<double>& rp, double& cre,
                                               double& cim) {
        const double2* b = reinterpret_cast<const double2*>(at);
        const double2 x = b[0], y = b[kWave], z = b[2 * kWave];
        rs = {x.x, x.y};
        rp = {y.x, y.y};
        cre = z.x;
        cim = z.y;
    }
};

// The phase coefficient cre as a float pair (hi, lo: hi + lo = cre to about
// 48 bits) beside cim in float, in one 16-byte slot.
__device__ __forceinline__ float4 phase_slot_f(double cre, double cim) {
    const float hi = (float)cre;
    return make_float4(hi, (float)(cre - (double)hi), (float)cim, 0.0f);
}

template <>
struct PairTab<float> {
    static constexpr int kBlockBytes = 2 * kWave * 16;  // (rho_s, rho_p)[64] as float4, (cre hi, lo, cim)[64]
    __device__ static void put(unsigned char* blk, int lane, cx<double> rs, cx<double> rp, double cre, double cim) {
        reinterpret_cast<float4*>(blk)[lane] = make_float4((float)rs.re, (float)rs.im, (float)rp.re, (float)rp.im);
        reinterpret_cast<float4*>(blk + kWave * 16)[lane] = phase_slot_f(cre, cim);
    }
    __device__ __forceinline__ static void get(const unsigned char* at, cx<float>& rs, cx<float>& rp, double& cre,
                                               double& cim) {
        const float4 x = *reinterpret_cast<const float4*>(at);
        const float4 z = *reinterpret_cast<const float4*>(at + kWave * 16);
        rs = {x.x, x.y};
        rp = {x.z, x.w};
        cre = (double)z.x + (double)z.y;
        cim = (double)z.z;
    }
    __device__ __forceinline__ static void get_ff(const unsigned char* at, cx<float>& rs, cx<float>& rp, float& c_hi,
                                                  float& c_lo, float& cim) {
        const float4 x = *reinterpret_cast<const float4*>(at);
        const float4 z = *reinterpret_cast<const float4*>(at + kWave * 16);
        rs = {x.x, x.y};
        rp = {x.z, x.w};
        c_hi = z.x;
        c_lo = z.y;
        cim = z.z;
    }
};

// Row blocks (tables of 7 to 16 rows, where a block per ordered pair no longer
// fits the LDS): one block per table row m with, for the 64 lanes, q_m, eta_m,
// 1 / q_m, 1 / eta_m and (cre, cim) as in PairTab; a step forms the ratios
// rho_s = q_{m'} (1 / q_m) and rho_p = eta_{m'} (1 / eta_m) from the blocks of the
// current row m and the next row m'.
template <typename R> struct RowTab;

template <>
struct RowTab<double> {
    static constexpr int kBlockBytes = 5 * kWave * 16;  // q, eta, 1/q, 1/eta, (cre, cim)
    __device__ static void put(unsigned char* blk, int lane, cx<double> q, cx<double> e, cx<double> iq,
                               cx<double> ie, double cre, double cim) {
        double2* b = reinterpret_cast<double2*>(blk);
        b[lane] = make_double2(q.re, q.im);
        b[kWave + lane] = make_double2(e.re, e.im);
        b[2 * kWave + lane] = make_double2(iq.re, iq.im);
        b[3 * kWave + lane] = make_double2(ie.re, ie.im);
        b[4 * kWave + lane] = make_double2(cre, cim);
    }
    // `at` is the block address plus lane * 16
    __device__ __forceinline__ static void get_cur(const unsigned char* at, cx<double>& iq, cx<double>& ie,
                                                   double& cre, double& cim) {
        const double2* b = reinterpret_cast<const double2*>(at);
        const double2 x = b[2 * kWave], y = b[3 * kWave], z = b[4 * kWave];
        iq = {x.x, x.y};
        ie = {y.x, y.y};
        cre = z.x;
        cim = z.y;
    }
    __device__ __forceinline__ static void get_next(const unsigned char* at, cx<double>& q, cx<double>& e) {
        const double2* b = reinterpret_cast<const double2*>(at);
        const double2 x = b[0], y = b[kWave];
        q = {x.x, x.y};
        e = {y.x, y.y};
    }
    __device__ __forceinline__ static Layer<double> layer(const unsigned char* at) {
        cx<double> q, e;
        get_next(at, q, e);
        Layer<double> v;
        v.q = q;
        v.e = e;
        v.q2 = cnorm(q);
        v.e2 = cnorm(e);
        v.pr = q.re;
        v.pi = q.im;
        return v;
    }
};

template <>
struct RowTab<float> {
    static constexpr int kBlockBytes = 3 * kWave * 16;  // (q, eta) float4, (1/q, 1/eta) float4, (cre hi, lo, cim)
    __device__ static void put(unsigned char* blk, int lane, cx<double> q, cx<double> e, cx<double> iq,
                               cx<double> ie, double cre, double cim) {
        reinterpret_cast<float4*>(blk)[lane] = make_float4((float)q.re, (float)q.im, (float)e.re, (float)e.im);
        reinterpret_cast<float4*>(blk + kWave * 16)[lane] =
            make_float4((float)iq.re, (float)iq.im, (float)ie.re, (float)ie.im);
        reinterpret_cast<float4*>(blk + 2 * kWave * 16)[lane] = phase_slot_f(cre, cim);
    }
    __device__ __forceinline__ static void get_cur(const unsigned char* at, cx<float>& iq, cx<float>& ie,
                                                   double& cre, double& cim) {
        const float4 x = *reinterpret_cast<const float4*>(at + kWave * 16);
        const float4 z = *reinterpret_cast<const float4*>(at + 2 * kWave * 16);
        iq = {x.x, x.y};
        ie = {x.z, x.w};
        cre = (double)z.x + (double)z.y;
        cim = (double)z.z;
    }
    __device__ __forceinline__ static void get_cur_ff(const unsigned char* at, cx<float>& iq, cx<float>& ie,
                                                      float& c_hi, float& c_lo, float& cim) {
        const float4 x = *reinterpret_cast<const float4*>(at + kWave * 16);
        const float4 z = *reinterpret_cast<const float4*>(at + 2 * kWave * 16);
        iq = {x.x, x.y};
        ie = {x.z, x.w};
        c_hi = z.x;
        c_lo = z.y;
        cim = z.z;
    }
    __device__ __forceinline__ static void get_next(const unsigned char* at, cx<float>& q, cx<float>& e) {
        const float4 x = *reinterpret_cast<const float4*>(at);
        q = {x.x, x.y};
        e = {x.z, x.w};
    }
    __device__ __forceinline__ static Layer<float> layer(const unsigned char* at) {
        cx<float> q, e;
        get_next(at, q, e);
        Layer<float> v;
        v.q = q;
        v.e = e;
        v.q2 = cnorm(q);
        v.e2 = cnorm(e);
        v.pr = (double)q.re;
        v.pi = (double)q.im;
        return v;
    }
};

// Waves per workgroup at most: 16 (4 per SIMD, at most 128 VGPRs) for every
// variant but the double-precision two-polarisation amplitude one, which needs
// more registers and runs 12 (3 per SIMD).
template <typename R, int POL, bool AMP>
__host__ __device__ constexpr int pair_max_waves() {
    return (sizeof(R) == 8 && AMP && POL == 3) ? 12 : 16;
}
constexpr int kPairMaxWaves = 16;
constexpr int kPairMaxMat = 8;
constexpr size_t kLdsPerCU = 160 * 1024;
constexpr size_t kPairFlagBytes = 4 * kPairMaxMat + 4 * kPairMaxWaves + 8 * kPairMaxWaves + 16;

template <typename R>
__host__ __device__ constexpr size_t pair_lds_bytes(int n_mat) {
    return phase_tab_bytes<R>() + (size_t)n_mat * Table<R>::kBlockBytes +
           (size_t)n_mat * n_mat * PairTab<R>::kBlockBytes + kPairFlagBytes;
}
// Row-block layout: phase table | one RowTab block per row | flags.
constexpr int kRowMaxMat = 16;
constexpr size_t kRowFlagBytes = 4 * kRowMaxMat + 4 * kPairMaxWaves + 8 * kPairMaxWaves + 16;
template <typename R>
__host__ __device__ constexpr size_t row_lds_bytes(int n_mat) {
    return phase_tab_bytes<R>() + (size_t)n_mat * RowTab<R>::kBlockBytes + kRowFlagBytes;
}
template <typename R, bool ROWS>
__host__ __device__ constexpr size_t pair_kernel_lds_bytes(int n_mat) {
    return ROWS ? row_lds_bytes<R>(n_mat) : pair_lds_bytes<R>(n_mat);
}

template <typename R>
constexpr int pair_max_mat() {
    int n = 0;
    while (n < kPairMaxMat && pair_lds_bytes<R>(n + 1) <= kLdsPerCU) ++n;
    return n;
}

// One stack on the pair table.  Returns false, having stored nothing, when a
// layer's phase could leave the range of the fast reduction (thickness above
// dmax, or not a number); the caller then evaluates the stack on the exact path.
// ROWS: pair_base holds row blocks (RowTab) and the ratios are formed per step
// from the current and the next row; tab is not used.
template <typename R, int POL, bool AMP, bool ROWS>
__device__ __forceinline__ bool run_stack_pair(const FwdParams<R>& p, const unsigned char* pair_base,
                                               const Table<R>& tab, uint32_t lossy_mask, double dmax,
                                               const Ambient& amb, int b, int k, int i, int lane, bool active,
                                               bool lane_ok, double nsub_r, double nsub_i,
                                               const TabPhase<R>& phase) {
    const int L = p.L;
    const int n_mat = p.n_mat;
    const R* drow = p.d + (int64_t)b * L;
    const int32_t* mrow = p.mat + (int64_t)b * (L + 2);
    const int m_sub_raw = mrow[L + 1];
    bool bad = (uint32_t)m_sub_raw >= (uint32_t)n_mat;
    const int m_sub = bad ? 0 : m_sub_raw;
    // float R and T: the phase reduced as a float pair (dmax keeps it below 2^21)
    constexpr bool kFF = sizeof(R) == 4 && !AMP;
    const unsigned char* const lane_base = pair_base + lane * 16;
    int nxt_off = m_sub * RowTab<R>::kBlockBytes;  // ROWS: block of the layer below (the substrate first)
    PairChain<R, POL, AMP> c;
    c.init();
    constexpr int RP = PairRenormPeriod<R>::value;
    static_assert(kWave % RP == 0, "chunks must hold whole renormalisation blocks");
    for (int top = L; top >= 1; top -= kWave) {
        const int lo = top - kWave + 1 > 1 ? top - kWave + 1 : 1;
        // lane l holds layer lo + l: thickness and pair block offset | lossy << 31
        const int j = lo + lane;
        double my_d = 0.0;
        float my_df = 0.0f;  // the same thickness in float (exact for float inputs)
        int my_code = 0;
        bool lane_bad = false, lane_far = false;
        if (j <= top) {
            const R dj = drow[j - 1];
            const int m = mrow[j], mn = mrow[j + 1];
            // ROWS: the next row was checked as the current one of the step below (or as the substrate)
            const bool mbad = (uint32_t)m >= (uint32_t)n_mat || (!ROWS && (uint32_t)mn >= (uint32_t)n_mat);
            lane_bad = mbad || bad_thickness(dj);
            lane_far = !((double)dj <= dmax);
            const int mc = mbad ? 0 : m, mnc = mbad ? 0 : mn;
            my_d = (double)dj;
            my_df = (float)dj;
            const int off = ROWS ? mc * RowTab<R>::kBlockBytes : (mc * n_mat + mnc) * PairTab<R>::kBlockBytes;
            my_code = off | (int)(((lossy_mask >> mc) & 1u) << 31);
        }
        if (__any(lane_far)) return false;
        bad = bad || __any(lane_bad);
        auto step = [&](int jj) {
            const int sl = jj - lo;
            const int code = __builtin_amdgcn_readlane(my_code, sl);
            if constexpr (kFF) {
                // float: the thickness is exact in float, the phase a float pair
                const float df = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(my_df), sl));
                cx<R> rs, rp;
                float c_hi, c_lo, cim;
                if constexpr (ROWS) {
                    const int cur_off = code & 0x7fffffff;
                    cx<R> iq, ie, qn, en;
                    RowTab<R>::get_cur_ff(lane_base + cur_off, iq, ie, c_hi, c_lo, cim);
                    RowTab<R>::get_next(lane_base + nxt_off, qn, en);
                    rs = cmul(qn, iq);
                    rp = cmul(en, ie);
                    nxt_off = cur_off;
                } else {
                    PairTab<R>::get_ff(lane_base + (code & 0x7fffffff), rs, rp, c_hi, c_lo, cim);
                }
                c.step_ff(rs, rp, c_hi, c_lo, cim, df, code < 0, phase);
                return;
            }
            const double dj = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(my_d), sl),
                                               __builtin_amdgcn_readlane(__double2loint(my_d), sl));
            cx<R> rs, rp;
            double cre, cim;
            if constexpr (ROWS) {
                const int cur_off = code & 0x7fffffff;
                cx<R> iq, ie, qn, en;
                RowTab<R>::get_cur(lane_base + cur_off, iq, ie, cre, cim);
                RowTab<R>::get_next(lane_base + nxt_off, qn, en);
                rs = cmul(qn, iq);
                rp = cmul(en, ie);
                nxt_off = cur_off;
            } else {
                PairTab<R>::get(lane_base + (code & 0x7fffffff), rs, rp, cre, cim);
            }
            c.step(rs, rp, cre, cim, dj, code < 0, phase);
        };
        for (int bt = top; bt >= lo; bt -= RP) {
            if (bt - lo >= RP - 1) {
#pragma unroll 2
                for (int u = 0; u < RP; ++u) step(bt - u);
                c.renorm();
            } else {
                for (int jj = bt; jj >= lo; --jj) step(jj);
            }
        }
    }
    c.renorm();
    const int m_first_raw = L >= 1 ? mrow[1] : m_sub;
    const int m_first = (uint32_t)m_first_raw < (uint32_t)n_mat ? m_first_raw : 0;
    PointOut out[2];
    if constexpr (ROWS)
        finish<R, POL, AMP>(c, amb, RowTab<R>::layer(lane_base + m_first * RowTab<R>::kBlockBytes),
                            RowTab<R>::layer(lane_base + m_sub * RowTab<R>::kBlockBytes), nsub_r, nsub_i, L, out,
                            phase);
    else
        finish<R, POL, AMP>(c, amb, tab.get(m_first, lane), tab.get(m_sub, lane), nsub_r, nsub_i, L, out, phase);
    if (active) {
        const bool valid = lane_ok && !bad;
        constexpr int P = (POL == 3) ? 2 : 1;
        store_point(p, b, k, i, 0, P, out[0], valid);
        if (POL == 3) store_point(p, b, k, i, 1, P, out[1], valid);
    }
    return true;
}

template <typename R, int POL, bool AMP, bool ROWS>
__global__ void __launch_bounds__((pair_max_waves<R, POL, AMP>() * kWave)) fwd_pair_kernel(FwdParams<R> p) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nthr = blockDim.x;  // a multiple of kWave, at most pair_max_waves * kWave
    const int nwaves = nthr / kWave;
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
    const int i = active ? i_raw : p.n_wl - 1;  // ragged tail: compute a valid point, store nothing
    const double lam = (double)p.wl[i];
    const bool lam_ok = lam > 0.0 && lam < __builtin_inf();
    const double c4lam = 4.0 / lam;
    const double st = (double)p.sin_t[k], ct = (double)p.cos_t[k];
    const int L2 = p.L + 2;
    const int n_mat = p.n_mat;
    fill_phase_tab<R>(smem, threadIdx.x, nthr);
    unsigned char* const tab_base = smem + phase_tab_bytes<R>();
    // ROWS: no media table; the row blocks start where it would
    unsigned char* const pair_base = ROWS ? tab_base : tab_base + (size_t)n_mat * Table<R>::kBlockBytes;
    unsigned char* const flag_base =
        pair_base + (ROWS ? (size_t)n_mat * RowTab<R>::kBlockBytes : (size_t)n_mat * n_mat * PairTab<R>::kBlockBytes);
    int* const lossy_f = reinterpret_cast<int*>(flag_base);
    int* const bad_w = lossy_f + (ROWS ? kRowMaxMat : kPairMaxMat);  // one lossy flag per row
    double* const cmax_w = reinterpret_cast<double*>(bad_w + kPairMaxWaves);
    int* const next_b = reinterpret_cast<int*>(cmax_w + kPairMaxWaves);

    int amb_row = p.mat[(int64_t)b0 * L2];
    amb_row = amb_row < 0 ? 0 : (amb_row >= n_mat ? n_mat - 1 : amb_row);
    double n0r, n0i;
    load_n(p.nk, p.dispersive, p.n_wl, amb_row, i, n0r, n0i);
    const Ambient amb = make_ambient(n0r, n0i, st, ct);
    Table<R> tab(tab_base, n_mat);
    const bool lane_used = active && lam_ok && amb.ok;
    bool bad_lane = false;
    double cmax = 0.0;
    if constexpr (ROWS) {
        // row blocks: q, eta, their reciprocals and the phase coefficients of every row
        for (int m = wave; m < n_mat; m += nwaves) {
            double nr, ni;
            load_n(p.nk, p.dispersive, p.n_wl, m, i, nr, ni);
            const Medium md = make_medium(nr, ni, amb.kx);
            const cx<double> q = {md.qr, md.qi}, e = {md.er, md.ei};
            const cx<double> iq = cdiv({1.0, 0.0}, q), ie = cdiv({1.0, 0.0}, e);
            const double cre = (c4lam * kScSteps) * md.qr, cim = c4lam * md.qi * kNegPiLog2e;
            RowTab<R>::put(pair_base + (size_t)m * RowTab<R>::kBlockBytes, lane, q, e, iq, ie, cre, cim);
            const bool lossy = __any(md.qi != 0.0);
            if (lane == 0) lossy_f[m] = lossy ? 1 : 0;
        }
    } else {
    for (int m = wave; m < n_mat; m += nwaves) {
        double nr, ni;
        load_n(p.nk, p.dispersive, p.n_wl, m, i, nr, ni);
        const Medium md = make_medium(nr, ni, amb.kx);
        tab.put(m, lane, md);
        const bool lossy = __any(md.qi != 0.0);
        if (lane == 0) lossy_f[m] = lossy ? 1 : 0;
    }
    // pair blocks; lanes whose results are stored check the ratio bound and
    // give the largest phase coefficient
    for (int pi = wave; pi < n_mat * n_mat; pi += nwaves) {
        const int mc = pi / n_mat, mn = pi - mc * n_mat;
        double ar, ai, br, bi;
        load_n(p.nk, p.dispersive, p.n_wl, mc, i, ar, ai);
        load_n(p.nk, p.dispersive, p.n_wl, mn, i, br, bi);
        const Medium ma = make_medium(ar, ai, amb.kx), mb = make_medium(br, bi, amb.kx);
        const cx<double> rs = cdiv({mb.qr, mb.qi}, {ma.qr, ma.qi});
        const cx<double> rp = cdiv({mb.er, mb.ei}, {ma.er, ma.ei});
        const double cre = (c4lam * kScSteps) * ma.qr, cim = c4lam * ma.qi * kNegPiLog2e;
        PairTab<R>::put(pair_base + (size_t)pi * PairTab<R>::kBlockBytes, lane, rs, rp, cre, cim);
        if (lane_used) {
            const double mag = fmax(fmax(fabs(rs.re), fabs(rs.im)), fmax(fabs(rp.re), fabs(rp.im)));
            bad_lane = bad_lane || !(mag <= kPairRatioMax);
            cmax = fmax(cmax, fabs(cre));
        }
    }
    }
    if constexpr (ROWS) {
        // every ratio of two rows is bounded by the largest over the smallest modulus;
        // each wave reads all rows for its lanes after the blocks are written
        __syncthreads();
        if (lane_used) {
            double qmax = 0.0, qmin = __builtin_inf(), emax = 0.0, emin = __builtin_inf();
            for (int m = 0; m < n_mat; ++m) {
                const double2* b = reinterpret_cast<const double2*>(pair_base + (size_t)m * RowTab<R>::kBlockBytes);
                cx<double> q, e;
                if constexpr (sizeof(R) == 8) {
                    const double2 x = b[lane], y = b[kWave + lane];
                    q = {x.x, x.y};
                    e = {y.x, y.y};
                } else {
                    const float4 x = reinterpret_cast<const float4*>(b)[lane];
                    q = {(double)x.x, (double)x.y};
                    e = {(double)x.z, (double)x.w};
                }
                const double aq = sqrt(cnorm(q)), ae = sqrt(cnorm(e));
                qmax = fmax(qmax, aq);
                qmin = fmin(qmin, aq);
                emax = fmax(emax, ae);
                emin = fmin(emin, ae);
                const double cre = reinterpret_cast<const double2*>(
                    pair_base + (size_t)m * RowTab<R>::kBlockBytes + (RowTab<R>::kBlockBytes - kWave * 16))[lane].x;
                cmax = fmax(cmax, fabs(cre));
            }
            bad_lane = !(qmax <= kPairRatioMax * qmin) || !(emax <= kPairRatioMax * emin);
        }
    }
    const bool wave_bad = __any(bad_lane);
    for (int off = kWave / 2; off >= 1; off >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, off));
    if (lane == 0) {
        bad_w[wave] = wave_bad ? 1 : 0;
        cmax_w[wave] = cmax;
    }
    if (threadIdx.x == 0) *next_b = b0 + nwaves;
    __syncthreads();
    uint32_t mask = 0;
    for (int m = 0; m < n_mat; ++m) mask |= (uint32_t)lossy_f[m] << m;
    mask = __builtin_amdgcn_readfirstlane(mask);
    int any_bad = 0;
    double cm = 0.0;
    for (int w = 0; w < nwaves; ++w) {
        any_bad |= bad_w[w];
        cm = fmax(cm, cmax_w[w]);
    }
    const bool pair_ok = __builtin_amdgcn_readfirstlane(any_bad) == 0;
    // every layer of a stack with d <= dmax keeps |phi| below the fast range
    // (the float-pair reduction's in float R and T)
    const double dmax = (sizeof(R) == 4 && !AMP ? kScFastRangeF : 0.5 * kScFastRange) / cm;
    const TabPhase<R> phase = phase_of<R>(smem);
    // stacks are handed out one at a time from an LDS counter (the first one
    // per wave statically): waves that run faster take more stacks, so the
    // workgroup's waves finish together and the CU does not idle at its end
    for (int b = b0 + wave; b < b1;) {
        const int bb = b;
        {
            int nb = 0;
            if (lane == 0) nb = atomicAdd(next_b, 1);
            b = __builtin_amdgcn_readfirstlane(nb);
        }
        const int32_t* mrow = p.mat + (int64_t)bb * L2;
        int sub_row = mrow[p.L + 1];
        sub_row = sub_row < 0 ? 0 : (sub_row >= n_mat ? n_mat - 1 : sub_row);
        double nsr = 0.0, nsi = 0.0;
        if (AMP) load_n(p.nk, p.dispersive, p.n_wl, sub_row, i, nsr, nsi);
        if (pair_ok && mrow[0] == amb_row &&
            run_stack_pair<R, POL, AMP, ROWS>(p, pair_base, tab, mask, dmax, amb, bb, k, i, lane, active,
                                              lam_ok && amb.ok, nsr, nsi, phase))
            continue;
        // per-step media: any ambient, any ratio, any finite phase
        int a_row = mrow[0];
        a_row = a_row < 0 ? 0 : (a_row >= n_mat ? n_mat - 1 : a_row);
        double ar, ai;
        load_n(p.nk, p.dispersive, p.n_wl, a_row, i, ar, ai);
        const Ambient amb_b = make_ambient(ar, ai, st, ct);
        InlineSource<R> src{p.nk, mrow, 0, n_mat, p.dispersive, p.n_wl, i, amb_b.kx};
        run_stack<R, POL, AMP>(p, src, amb_b, bb, k, i, active, lam_ok && amb_b.ok, c4lam, nsr, nsi, phase);
    }
}

// ---------------------------------------------------------------------------
// Host side.

template <typename R, int POL, bool AMP, bool TABLE>
static hipError_t launch_fwd(const FwdParams<R>& p, int blocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((fwd_kernel<R, POL, AMP, TABLE>), dim3(blocks), dim3(kBlock), lds, s, p);
    return hipGetLastError();
}

template <typename R, bool TABLE>
static hipError_t dispatch_pol(const FwdParams<R>& p, unsigned pol, bool amp, int blocks, size_t lds,
                               hipStream_t s) {
    if (amp) {
        if (pol == 1) return launch_fwd<R, 1, true, TABLE>(p, blocks, lds, s);
        if (pol == 2) return launch_fwd<R, 2, true, TABLE>(p, blocks, lds, s);
        return launch_fwd<R, 3, true, TABLE>(p, blocks, lds, s);
    }
    if (pol == 1) return launch_fwd<R, 1, false, TABLE>(p, blocks, lds, s);
    if (pol == 2) return launch_fwd<R, 2, false, TABLE>(p, blocks, lds, s);
    return launch_fwd<R, 3, false, TABLE>(p, blocks, lds, s);
}

template <typename R, int POL, bool AMP, bool ROWS>
static hipError_t launch_pair(const FwdParams<R>& p, int blocks, int threads, size_t lds, hipStream_t s) {
    // dynamic LDS above 64 KiB: raise the kernel's limit once per device
    static std::atomic<size_t> raised[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (raised[dev].load() < lds) {
        (void)hipFuncSetAttribute((const void*)&fwd_pair_kernel<R, POL, AMP, ROWS>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
        raised[dev].store(lds);
    }
    hipLaunchKernelGGL((fwd_pair_kernel<R, POL, AMP, ROWS>), dim3(blocks), dim3(threads), lds, s, p);
    return hipGetLastError();
}

// Launch shape of the pair kernel: as many workgroups per CU as the LDS holds
// (1, 2 or 4), and waves per workgroup so that the CU holds its maximum of
// resident waves.  Stacks per workgroup: enough layer steps to amortise the
// workgroup's table build (about 320 VALU instructions per material pair and
// 150 per material, against about 60 per layer step) twenty times over, more
// while the grid keeps at least 64 workgroups per resident slot (a short last
// round of workgroups), at most 32 per wave.
template <typename R, int POL, bool AMP, bool ROWS>
static tmm_status run_pair(FwdParams<R> p, int64_t B, int64_t cols, hipStream_t s) {
    const size_t lds = pair_kernel_lds_bytes<R, ROWS>(p.n_mat);
    const size_t granule = 2048;
    int per_cu = (int)(kLdsPerCU / ((lds + granule - 1) / granule * granule));
    // 1, 2 or 4 workgroups per CU, so that each holds a multiple of the four SIMDs'
    // waves (three would give five-wave workgroups that do not divide over them)
    per_cu = per_cu >= 4 ? 4 : (per_cu >= 2 ? 2 : 1);
    const int waves = pair_max_waves<R, POL, AMP>() / per_cu;
    const int64_t table_cost = ROWS ? 450 * (int64_t)p.n_mat : 320 * (int64_t)p.n_mat * p.n_mat + 150 * (int64_t)p.n_mat;
    const int64_t amortise = ceil_div(20 * table_cost, 60 * ((int64_t)p.L + 1));
    const int64_t fill = ceil_div(B * cols, 256 * (int64_t)per_cu * 64);
    int64_t chunk = amortise > fill ? amortise : fill;
    if (chunk > 32 * waves) chunk = 32 * waves;
    chunk = ceil_div(chunk, waves) * waves;
    p.chunk = (int)chunk;
    const int64_t blocks = cols * ceil_div(B, (int64_t)p.chunk);
    if (blocks > 0x7fffffff)
        return fail(TMM_ERR_UNSUPPORTED, "tmm_rt: grid of %lld workgroups is too large", (long long)blocks);
    const hipError_t e = launch_pair<R, POL, AMP, ROWS>(p, (int)blocks, waves * kWave, lds, s);
    if (e != hipSuccess) return fail(TMM_ERR_HIP, "tmm_rt: launch failed: %s", hipGetErrorString(e));
    return ok();
}

template <typename R, bool ROWS>
static tmm_status dispatch_pair(const FwdParams<R>& p, unsigned pol, bool amp, int64_t B, int64_t cols,
                                hipStream_t s) {
    if (amp) {
        if (pol == 1) return run_pair<R, 1, true, ROWS>(p, B, cols, s);
        if (pol == 2) return run_pair<R, 2, true, ROWS>(p, B, cols, s);
        return run_pair<R, 3, true, ROWS>(p, B, cols, s);
    }
    if (pol == 1) return run_pair<R, 1, false, ROWS>(p, B, cols, s);
    if (pol == 2) return run_pair<R, 2, false, ROWS>(p, B, cols, s);
    return run_pair<R, 3, false, ROWS>(p, B, cols, s);
}

// Stacks per workgroup: enough workgroups to fill 256 CUs many times over,
// and as many stacks per workgroup as that allows, to amortise the table.
static int pick_chunk(int64_t B, int64_t tiles_x_angles) {
    const int64_t target_blocks = 32768;
    int64_t chunk = ceil_div(B * tiles_x_angles, target_blocks);
    chunk = ceil_div(chunk, kWavesPerBlock) * kWavesPerBlock;
    if (chunk < kWavesPerBlock) chunk = kWavesPerBlock;
    if (chunk > 64) chunk = 64;
    return (int)chunk;
}

template <typename R>
static tmm_status run_fwd(const tmm_rt_args* a, hipStream_t s) {
    FwdParams<R> p;
    p.B = a->B;
    p.L = a->L;
    p.n_wl = a->n_wl;
    p.n_theta = a->n_theta;
    p.d = static_cast<const R*>(a->d);
    p.nk = static_cast<const R*>(a->nk);
    p.n_mat = a->n_mat;
    p.dispersive = a->dispersive;
    p.mat = a->mat;
    p.wl = static_cast<const R*>(a->wl);
    p.sin_t = static_cast<const R*>(a->sin_theta);
    p.cos_t = static_cast<const R*>(a->cos_theta);
    p.R_out = static_cast<R*>(a->R);
    p.T_out = static_cast<R*>(a->T);
    p.r_out = static_cast<R*>(a->r);
    p.t_out = static_cast<R*>(a->t);
    p.n_tiles = (int)ceil_div(a->n_wl, kWave);
    const int64_t cols = (int64_t)p.n_tiles * a->n_theta;
    const bool amp = a->r != nullptr || a->t != nullptr;
    (void)hipGetLastError();
    if (a->mat != nullptr && a->n_mat <= pair_max_mat<R>())
        return dispatch_pair<R, false>(p, a->pol_mask, amp, a->B, cols, s);
    if (a->mat != nullptr && a->n_mat <= kRowMaxMat) return dispatch_pair<R, true>(p, a->pol_mask, amp, a->B, cols, s);
    p.chunk = pick_chunk(a->B, cols);
    const int64_t blocks = cols * ceil_div(a->B, p.chunk);
    if (blocks > 0x7fffffff)
        return fail(TMM_ERR_UNSUPPORTED, "tmm_rt: grid of %lld workgroups is too large", (long long)blocks);
    const bool table = a->mat != nullptr && a->n_mat <= kMaxTableMat;
    const size_t lds = table ? table_bytes<R>(a->n_mat) : phase_tab_bytes<R>();
    const hipError_t e = table ? dispatch_pol<R, true>(p, a->pol_mask, amp, (int)blocks, lds, s)
                               : dispatch_pol<R, false>(p, a->pol_mask, amp, (int)blocks, lds, s);
    if (e != hipSuccess) return fail(TMM_ERR_HIP, "tmm_rt: launch failed: %s", hipGetErrorString(e));
    return ok();
}

tmm_status check_rt_args(const tmm_rt_args* a, const char* who, bool need_output) {
    if (!a) return fail(TMM_ERR_INVALID_ARG, "%s: args is NULL", who);
    if (a->B < 0 || a->L < 0 || a->n_wl < 0 || a->n_theta < 0)
        return fail(TMM_ERR_INVALID_ARG, "%s: negative size (B=%d L=%d n_wl=%d n_theta=%d)", who, a->B, a->L,
                    a->n_wl, a->n_theta);
    if (a->L > (1 << 20)) return fail(TMM_ERR_INVALID_ARG, "%s: L=%d exceeds 1<<20", who, a->L);
    if (a->pol_mask < 1u || a->pol_mask > 3u)
        return fail(TMM_ERR_INVALID_ARG, "%s: pol_mask must be 1 (s), 2 (p) or 3 (both), got %u", who, a->pol_mask);
    if (a->dispersive != 0 && a->dispersive != 1)
        return fail(TMM_ERR_INVALID_ARG, "%s: dispersive must be 0 or 1", who);
    if (a->flags & ~(uint32_t)TMM_CHECK_FINITE)
        return fail(TMM_ERR_INVALID_ARG, "%s: unknown flag bits 0x%x", who, a->flags & ~(uint32_t)TMM_CHECK_FINITE);
    if (a->B == 0 || a->n_wl == 0 || a->n_theta == 0) return ok();  // nothing to compute
    if (a->n_mat < 1) return fail(TMM_ERR_INVALID_ARG, "%s: n_mat must be >= 1", who);
    if (!a->nk || !a->wl || !a->sin_theta || !a->cos_theta)
        return fail(TMM_ERR_INVALID_ARG, "%s: nk, wl, sin_theta and cos_theta must be non-NULL", who);
    if (a->L > 0 && !a->d) return fail(TMM_ERR_INVALID_ARG, "%s: d is NULL with L > 0", who);
    if (!a->mat && (int64_t)a->n_mat < (int64_t)a->B * (a->L + 2))
        return fail(TMM_ERR_INVALID_ARG, "%s: without mat, nk needs B*(L+2)=%lld rows, has %d", who,
                    (long long)a->B * (a->L + 2), a->n_mat);
    const int P = (a->pol_mask == 3u) ? 2 : 1;
    const double elems = (double)a->B * P * (double)a->n_theta * (double)a->n_wl;
    if (elems > 4.0e18) return fail(TMM_ERR_INVALID_ARG, "%s: output too large", who);
    if (need_output && !a->R && !a->T && !a->r && !a->t)
        return fail(TMM_ERR_INVALID_ARG, "%s: no output requested", who);
    return ok();
}

char* last_error_buffer() {
    static thread_local char buf[512];
    return buf;
}

}  // namespace tmm

extern "C" {

const char* tmm_status_string(tmm_status s) {
    switch (s) {
        case TMM_OK: return "ok";
        case TMM_ERR_INVALID_ARG: return "invalid argument";
        case TMM_ERR_UNSUPPORTED: return "unsupported request";
        case TMM_ERR_NONFINITE: return "non-finite input value";
        case TMM_ERR_HIP: return "HIP runtime error";
        case TMM_ERR_WORKSPACE: return "workspace missing or too small";
    }
    return "unknown status";
}

const char* tmm_last_error(void) { return tmm::last_error_buffer(); }

const char* tmm_version(void) { return "0.1.0"; }

tmm_status tmm_rt(const tmm_rt_args* a, tmm_dtype dtype, void* stream) {
    using tmm::fail;
    tmm_status st = tmm::check_rt_args(a, "tmm_rt", true);
    if (st != TMM_OK) return st;
    if (dtype != TMM_F64 && dtype != TMM_F32) return fail(TMM_ERR_INVALID_ARG, "tmm_rt: unknown dtype %d", (int)dtype);
    if (a->B == 0 || a->n_wl == 0 || a->n_theta == 0) return tmm::ok();  // nothing to compute
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (a->flags & TMM_CHECK_FINITE) {
        st = dtype == TMM_F64 ? tmm::check_rt_inputs<double>(a, nullptr, 0, nullptr, 0, "tmm_rt", s)
                              : tmm::check_rt_inputs<float>(a, nullptr, 0, nullptr, 0, "tmm_rt", s);
        if (st != TMM_OK) return st;
    }
    return dtype == TMM_F64 ? tmm::run_fwd<double>(a, s) : tmm::run_fwd<float>(a, s);
}

}  // extern "C"
