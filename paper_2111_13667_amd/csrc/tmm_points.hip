// tmm_rt at an explicit list of points (gfx950): R and T of the listed
// (stack, angle, wavelength) points of a dense batch, written into arrays laid
// out as tmm_rt's outputs.  The physics and algebra are those of the dense
// kernels (Eq. (1)-(7); the division-free recursion of tmm_device.hpp and
// tmm_chain.hpp); only the mapping differs: one lane is one listed point, so
// the lanes of a wave may belong to different stacks, angles and wavelengths.
//
// Each lane therefore reads its own layer data (thickness and material id per
// step, gathered from the stack's rows) and its own media: with material ids
// and a table of at most kPtMaxMat rows, q and eta of every row at the lane's
// (wavelength, angle) go into the wave's LDS slice once per point; otherwise
// they are computed per step.  Used where only scattered points are needed --
// the surrogate's transfer-matrix fallback recomputes exactly the outputs whose
// error estimate exceeds its bound.
#include <hip/hip_runtime.h>

#include "tmm_chain.hpp"
#include "tmm_check.hpp"
#include "tmm_host.hpp"
#include "tmm_points.hpp"

namespace tmm {
namespace pts {

constexpr int kPtWaves = 4;
constexpr int kPtBlock = kPtWaves * kWave;
constexpr int kPtMaxMat = 8;

// Per-wave media slice: q and eta (in double) of every table row at each lane's
// own point; [row][q, eta][lane].
struct LaneTable {
    double2* base;
    __device__ __forceinline__ void put(int m, int lane, const Medium& md) {
        base[(2 * m) * kWave + lane] = make_double2(md.qr, md.qi);
        base[(2 * m + 1) * kWave + lane] = make_double2(md.er, md.ei);
    }
    template <typename R>
    __device__ __forceinline__ Layer<R> get(int m, int lane) const {
        const double2 a = base[(2 * m) * kWave + lane], b = base[(2 * m + 1) * kWave + lane];
        Layer<R> v;
        v.q = {(R)a.x, (R)a.y};
        v.e = {(R)b.x, (R)b.y};
        v.q2 = (R)(a.x * a.x + a.y * a.y);
        v.e2 = (R)(b.x * b.x + b.y * b.y);
        v.pr = a.x;
        v.pi = a.y;
        return v;
    }
};

constexpr size_t lane_table_bytes(int n_mat) { return (size_t)n_mat * 2 * kWave * sizeof(double2); }

template <typename R>
__device__ __forceinline__ int64_t point_index(const PtParams<R>& p, int64_t t) {
    return p.pts64 ? p.pts64[t] : (int64_t)p.pts32[t];
}

template <typename R, int POL, bool TABLE, bool AMP>
__global__ void __launch_bounds__(kPtBlock) points_kernel(PtParams<R> p) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    fill_phase_tab<R>(smem, threadIdx.x, blockDim.x);
    __syncthreads();
    const TabPhase<R> phase = phase_of<R>(smem);
    LaneTable tab;
    tab.base = reinterpret_cast<double2*>(smem + phase_tab_bytes<R>() + (size_t)wave * lane_table_bytes(p.n_mat));
    constexpr int P = (POL == 3) ? 2 : 1;
    const int64_t n = p.n_dev ? (int64_t)*p.n_dev : p.n_pts;
    const int64_t total = (int64_t)p.B * p.n_theta * p.n_wl;
    const int L = p.L, L2 = p.L + 2;
    const int64_t stride = (int64_t)gridDim.x * kPtWaves * kWave;
    for (int64_t base = ((int64_t)blockIdx.x * kPtWaves + wave) * kWave; base < n; base += stride) {
        const int64_t t = base + lane;
        const bool listed = t < n;
        int64_t f = listed ? point_index(p, t) : 0;
        const bool in_range = listed && f >= 0 && f < total;
        if (!in_range) f = 0;
        const int i = (int)(f % p.n_wl);
        const int64_t bk = f / p.n_wl;
        const int k = (int)(bk % p.n_theta);
        const int b = (int)(bk / p.n_theta);
        const double lam = (double)p.wl[i];
        const bool lam_ok = lam > 0.0 && lam < __builtin_inf();
        const double c4lam = 4.0 / lam;
        const double st = (double)p.sin_t[k], ct = (double)p.cos_t[k];
        const int32_t* mrow = p.mat ? p.mat + (int64_t)b * L2 : nullptr;
        bool bad = false;
        auto row_of = [&](int j) -> int64_t {
            if (!mrow) return (int64_t)b * L2 + j;
            const int m = mrow[j];
            bad = bad || (uint32_t)m >= (uint32_t)p.n_mat;
            return m < 0 ? 0 : (m >= p.n_mat ? p.n_mat - 1 : m);
        };
        double n0r, n0i;
        load_n(p.nk, p.dispersive, p.n_wl, row_of(0), i, n0r, n0i);
        const Ambient amb = make_ambient(n0r, n0i, st, ct);
        auto medium = [&](int j) -> Layer<R> {
            const int64_t r = row_of(j);
            if (TABLE) return tab.get<R>((int)r, lane);
            double nr, ni;
            load_n(p.nk, p.dispersive, p.n_wl, r, i, nr, ni);
            return to_layer<R>(make_medium(nr, ni, amb.kx));
        };
        if (TABLE) {
            // every lane writes and reads only its own entries: no barrier needed
            for (int m = 0; m < p.n_mat; ++m) {
                double nr, ni;
                load_n(p.nk, p.dispersive, p.n_wl, m, i, nr, ni);
                tab.put(m, lane, make_medium(nr, ni, amb.kx));
            }
        }
        const R* drow = p.d + (int64_t)b * L;
        const Layer<R> sub = medium(L + 1);
        Layer<R> nxt = sub;
        Chain<R, POL, AMP> c;
        c.init();
        constexpr int RP = RenormPeriod<R>::value;
        int since = 0;
        for (int j = L; j >= 1; --j) {
            const Layer<R> cur = medium(j);
            const R dj = drow[j - 1];
            bad = bad || bad_thickness(dj);
            c.step(cur, nxt, (double)dj * c4lam, __any(cur.pi != 0.0), phase);
            nxt = cur;
            if (++since == RP) {
                c.renorm();
                since = 0;
            }
        }
        c.renorm();
        double ns_r = 0.0, ns_i = 0.0;  // the substrate's index (t of p)
        if constexpr (AMP) load_n(p.nk, p.dispersive, p.n_wl, row_of(L + 1), i, ns_r, ns_i);
        PointOut out[2];
        finish<R, POL, AMP>(c, amb, nxt, sub, ns_r, ns_i, L, out, phase);
        if (in_range) {
            const bool valid = lam_ok && amb.ok && !bad;
            const double nan = __builtin_nan("");
            for (int q = 0; q < P; ++q) {
                const int64_t o = (((int64_t)b * P + q) * p.n_theta + k) * p.n_wl + i;
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
    }
}

template <typename R, int POL, bool TABLE, bool AMP>
static hipError_t launch_pol(const PtParams<R>& p, int64_t max_points, hipStream_t s) {
    const size_t lds = phase_tab_bytes<R>() + (TABLE ? (size_t)kPtWaves * lane_table_bytes(p.n_mat) : 0);
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess)
        n_cu = 256;
    // persistent: enough blocks to fill the chip several times, no more than the points need
    int64_t blocks = ceil_div(max_points, kPtBlock);
    const int64_t cap = (int64_t)n_cu * 8;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute((const void*)&points_kernel<R, POL, TABLE, AMP>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    }
    hipLaunchKernelGGL((points_kernel<R, POL, TABLE, AMP>), dim3((unsigned)blocks), dim3(kPtBlock), lds, s, p);
    return hipGetLastError();
}

template <typename R, bool AMP>
static hipError_t launch_amp(const PtParams<R>& p, unsigned pol_mask, int64_t max_points, hipStream_t s) {
    const bool table = p.mat != nullptr && p.n_mat <= kPtMaxMat;
    if (pol_mask == 1u)
        return table ? launch_pol<R, 1, true, AMP>(p, max_points, s) : launch_pol<R, 1, false, AMP>(p, max_points, s);
    if (pol_mask == 2u)
        return table ? launch_pol<R, 2, true, AMP>(p, max_points, s) : launch_pol<R, 2, false, AMP>(p, max_points, s);
    return table ? launch_pol<R, 3, true, AMP>(p, max_points, s) : launch_pol<R, 3, false, AMP>(p, max_points, s);
}

template <typename R>
hipError_t launch_points(const PtParams<R>& p, unsigned pol_mask, int64_t max_points, hipStream_t s) {
    return (p.r_out || p.t_out) ? launch_amp<R, true>(p, pol_mask, max_points, s)
                                : launch_amp<R, false>(p, pol_mask, max_points, s);
}

template hipError_t launch_points<double>(const PtParams<double>&, unsigned, int64_t, hipStream_t);
template hipError_t launch_points<float>(const PtParams<float>&, unsigned, int64_t, hipStream_t);

template <typename R>
static tmm_status run(const tmm_rt_args* a, const int64_t* points, int64_t n_points, hipStream_t s) {
    PtParams<R> p;
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
    p.pts64 = points;
    p.pts32 = nullptr;
    p.n_pts = n_points;
    p.n_dev = nullptr;
    (void)hipGetLastError();
    if (launch_points<R>(p, a->pol_mask, n_points, s) != hipSuccess) return check_launch("tmm_rt_points");
    return ok();
}

}  // namespace pts
}  // namespace tmm

extern "C" {

tmm_status tmm_rt_points(const tmm_rt_args* a, const int64_t* points, int64_t n_points, tmm_dtype dtype,
                         void* stream) {
    using tmm::fail;
    tmm_status st = tmm::check_rt_args(a, "tmm_rt_points", false);
    if (st != TMM_OK) return st;
    if (dtype != TMM_F64 && dtype != TMM_F32)
        return fail(TMM_ERR_INVALID_ARG, "tmm_rt_points: unknown dtype %d", (int)dtype);
    if (n_points < 0) return fail(TMM_ERR_INVALID_ARG, "tmm_rt_points: negative point count");
    if (!a->R && !a->T && !a->r && !a->t) return fail(TMM_ERR_INVALID_ARG, "tmm_rt_points: no output requested");
    if (n_points > 0 && !points) return fail(TMM_ERR_INVALID_ARG, "tmm_rt_points: points is NULL");
    if (n_points == 0 || a->B == 0 || a->n_wl == 0 || a->n_theta == 0) return tmm::ok();
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (a->flags & TMM_CHECK_FINITE) {
        st = dtype == TMM_F64 ? tmm::check_rt_inputs<double>(a, nullptr, 0, nullptr, 0, "tmm_rt_points", s)
                              : tmm::check_rt_inputs<float>(a, nullptr, 0, nullptr, 0, "tmm_rt_points", s);
        if (st != TMM_OK) return st;
    }
    return dtype == TMM_F64 ? tmm::pts::run<double>(a, points, n_points, s)
                            : tmm::pts::run<float>(a, points, n_points, s);
}

}  // extern "C"
