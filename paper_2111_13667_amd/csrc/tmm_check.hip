// Opt-in validation of the device-resident inputs of tmm_rt / tmm_rt_grad
// (flag TMM_CHECK_FINITE).
//
// Without the flag the kernels never look at a value's validity beyond what
// they need: a non-finite or out-of-range value in device memory turns the
// affected outputs into NaN.  With the flag, one grid-stride kernel scans every
// input array the call will read and ORs what it finds into a status word; the
// host reads the word back (one stream synchronisation) before anything is
// launched, and reports TMM_ERR_NONFINITE for a NaN or infinity, or
// TMM_ERR_INVALID_ARG for a finite value outside its documented range
// (negative thickness, non-positive wavelength, material id outside the table,
// sin/cos of an angle outside [0, pi/2], an absorbing ambient at oblique
// incidence -- the conditions of the paper's problem statement, section
// "Physical Background": real incidence angle in a lossless ambient, Eq. (3)).
//
// The status words live in a small static device array (no allocation); each
// call takes the next of kCheckSlots words, so checks overlapping on one device
// race only when more than kCheckSlots of them are in flight at once.
#include <atomic>
#include <mutex>

#include "tmm_check.hpp"
#include "tmm_host.hpp"

namespace tmm {

constexpr int kCheckSlots = 64;
constexpr int kCheckMaxDevices = 64;

enum : unsigned {
    kBadNonFinite = 1u,   // a NaN or infinity anywhere
    kBadRange = 2u,       // a finite value outside its documented range
    kOblique = 4u,        // some sin(theta) != 0
    kLossyAmbient = 8u,   // some ambient row with Im n != 0 at some wavelength
};

static __device__ unsigned check_words[kCheckSlots];

template <typename R>
__device__ __forceinline__ bool fin(R x) {
    return __builtin_isfinite(x);
}

__global__ void check_reset(unsigned* word) {
    *word = 0u;
}

// One grid-stride pass over every input element.  The element index space is
// the concatenation of: d [B*L], nk [rows*cols*2], mat [B*(L+2)], wl [n_wl],
// sin/cos [n_theta] (pairs), and the extra arrays of the gradient entry point.
template <typename R>
__global__ void check_inputs(CheckArgs<R> c, unsigned* word) {
    const int64_t n_d = (int64_t)c.B * c.L;
    const int64_t n_nk = (int64_t)c.nk_rows * c.nk_cols;
    const int64_t n_mat = c.mat ? (int64_t)c.B * (c.L + 2) : 0;
    const int64_t n_amb = (int64_t)c.B;
    const int64_t e0 = n_d, e1 = e0 + n_nk, e2 = e1 + n_mat, e3 = e2 + c.n_wl, e4 = e3 + c.n_theta,
                  e5 = e4 + n_amb, e6 = e5 + c.n_extra0, e7 = e6 + c.n_extra1;
    unsigned bad = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < e7; t += stride) {
        if (t < e0) {
            const R v = c.d[t];
            bad |= !fin(v) ? kBadNonFinite : (v < R(0) ? kBadRange : 0u);
        } else if (t < e1) {
            const int64_t k = t - e0;
            if (!fin(c.nk[2 * k]) || !fin(c.nk[2 * k + 1])) bad |= kBadNonFinite;
        } else if (t < e2) {
            const int32_t m = c.mat[t - e1];
            if (m < 0 || m >= c.n_mat) bad |= kBadRange;
        } else if (t < e3) {
            const R v = c.wl[t - e2];
            bad |= !fin(v) ? kBadNonFinite : (v <= R(0) ? kBadRange : 0u);
        } else if (t < e4) {
            const R s = c.sin_t[t - e3], co = c.cos_t[t - e3];
            if (!fin(s) || !fin(co)) {
                bad |= kBadNonFinite;
            } else {
                if (s < R(0) || s > R(1) || co < R(0) || co > R(1)) bad |= kBadRange;
                if (s != R(0)) bad |= kOblique;
            }
        } else if (t < e5) {
            // the ambient row of stack b at every wavelength of the table
            const int64_t b = t - e4;
            const int64_t row = c.mat ? (int64_t)c.mat[b * (c.L + 2)] : b * (c.L + 2);
            if (row >= 0 && row < c.nk_rows) {
                for (int64_t i = 0; i < c.nk_cols; ++i) {
                    const R im = c.nk[2 * (row * c.nk_cols + i) + 1];
                    if (fin(im) && im != R(0)) {
                        bad |= kLossyAmbient;
                        break;
                    }
                }
            }
        } else if (t < e6) {
            if (!fin(c.extra0[t - e5])) bad |= kBadNonFinite;
        } else {
            if (!fin(c.extra1[t - e6])) bad |= kBadNonFinite;
        }
    }
    // one atomic per wave
    for (int off = 32; off >= 1; off >>= 1) bad |= __shfl_xor(bad, off);
    if ((threadIdx.x & 63) == 0 && bad) atomicOr(word, bad);
}

// Device address of the status words, per device (looked up once).
static unsigned* check_words_on(int dev) {
    static std::mutex mu;
    static unsigned* addr[kCheckMaxDevices] = {};
    std::lock_guard<std::mutex> g(mu);
    if (dev < 0 || dev >= kCheckMaxDevices) return nullptr;
    if (!addr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(check_words)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        addr[dev] = static_cast<unsigned*>(p);
    }
    return addr[dev];
}

template <typename R>
tmm_status check_device_inputs(const CheckArgs<R>& c, const char* who, hipStream_t s) {
    static std::atomic<unsigned> next{0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TMM_ERR_HIP, "%s: no device", who);
    unsigned* words = check_words_on(dev);
    if (!words) return fail(TMM_ERR_HIP, "%s: input check: status words not found on device %d", who, dev);
    unsigned* word = words + (next.fetch_add(1u) % kCheckSlots);
    (void)hipGetLastError();
    hipLaunchKernelGGL(check_reset, dim3(1), dim3(1), 0, s, word);
    hipLaunchKernelGGL(check_inputs<R>, dim3(1024), dim3(256), 0, s, c, word);
    unsigned host = 0u;
    hipError_t e = hipMemcpyAsync(&host, word, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(TMM_ERR_HIP, "%s: input check: %s", who, hipGetErrorString(e));
    if (host & kBadNonFinite)
        return fail(TMM_ERR_NONFINITE, "%s: an input holds NaN or infinity (TMM_CHECK_FINITE)", who);
    if (host & kBadRange)
        return fail(TMM_ERR_INVALID_ARG,
                    "%s: an input value is out of range: negative thickness, wavelength <= 0, material id "
                    "outside [0, n_mat) or an angle outside [0, pi/2] (TMM_CHECK_FINITE)",
                    who);
    if ((host & kOblique) && (host & kLossyAmbient))
        return fail(TMM_ERR_INVALID_ARG, "%s: absorbing ambient at oblique incidence (TMM_CHECK_FINITE)", who);
    return ok();
}

template <typename R>
tmm_status check_rt_inputs(const tmm_rt_args* a, const R* extra0, int64_t n_extra0, const R* extra1,
                           int64_t n_extra1, const char* who, hipStream_t s) {
    CheckArgs<R> c;
    c.B = a->B;
    c.L = a->L;
    c.n_wl = a->n_wl;
    c.n_theta = a->n_theta;
    c.d = static_cast<const R*>(a->d);
    c.nk = static_cast<const R*>(a->nk);
    c.nk_rows = a->n_mat;
    c.nk_cols = a->dispersive ? a->n_wl : 1;
    c.n_mat = a->n_mat;
    c.mat = a->mat;
    c.wl = static_cast<const R*>(a->wl);
    c.sin_t = static_cast<const R*>(a->sin_theta);
    c.cos_t = static_cast<const R*>(a->cos_theta);
    c.extra0 = extra0;
    c.n_extra0 = extra0 ? n_extra0 : 0;
    c.extra1 = extra1;
    c.n_extra1 = extra1 ? n_extra1 : 0;
    return check_device_inputs<R>(c, who, s);
}

template tmm_status check_rt_inputs<double>(const tmm_rt_args*, const double*, int64_t, const double*, int64_t,
                                            const char*, hipStream_t);
template tmm_status check_rt_inputs<float>(const tmm_rt_args*, const float*, int64_t, const float*, int64_t,
                                           const char*, hipStream_t);

}  // namespace tmm
