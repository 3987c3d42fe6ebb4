// Learned surrogate of the transfer-matrix method: an ensemble of MLPs
// (thicknesses -> R spectrum) trained and evaluated with hand-written BF16
// MFMA kernels (FP32 accumulation, FP32 master weights, Adam), plus the
// TMM fallback that recomputes every stack whose ensemble spread exceeds a
// bound.  The paper motivates this use of fast TMM (sections "Core
// functionality speedup and dataset generation" and App. A.2: generating
// datasets for machine learning); the network itself is this project's.
//
// Network per member: x (n_in thicknesses, normalised, zero-padded to a
// multiple of 128) -> n_layers x [Linear(n_hidden) + GELU] -> Linear(n_out).
// Weights W_l [out][in] in FP32 (master) plus BF16 copies W [out][in] and
// Wt [in][out]; activations BF16 (plus transposed copies for the weight
// gradients), pre-activations FP32, outputs FP32.  All members run in the
// same launches (grid z = member).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "tmm_host.hpp"
#include "tmm_mlp_kernels.hpp"
#include "tmm_points.hpp"

#include "tmm_surrogate.h"

namespace tmm {
namespace mlp {

// ----------------------------------------------------------------------------
// Elementwise / reduction kernels.

// x [B][n_in] fp32 -> Xb [Bt][in_pad] bf16 and Xt [in_pad][Bt] bf16 of
// (x - shift) * scale; rows >= B and columns >= n_in are zero.
__global__ void prep_input(const float* x, int B, int n_in, int in_pad, int Bt, float shift, float scale,
                           __bf16* Xb, __bf16* Xt) {
    const int64_t n = (int64_t)Bt * in_pad;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(t / in_pad), k = (int)(t % in_pad);
        float v = 0.0f;
        if (m < B && k < n_in) v = (x[(int64_t)m * n_in + k] - shift) * scale;
        const __bf16 h = (__bf16)v;
        Xb[t] = h;
        Xt[(int64_t)k * Bt + m] = h;
    }
}

// Tiled transpose helper for [rows][cols] -> [cols][rows] bf16 via LDS.
constexpr int kTile = 64;

// Objective: the mean over the batch of the summed squared error over the
// outputs, sum_o (Y - T)^2 / B (its gradient scale keeps Adam's epsilon far
// below the gradients).  dY = 2 (Y - T) / B for rows < B (0 beyond), bf16
// [m][n] and [n][m]; loss[e] += sum (Y - T)^2 / (B n_out), the mean squared
// error per output (reported only: each block writes its partial sum to
// part[e][block], sum_parts adds them in a fixed order).  grid (n_out/64, Bt/64), block 256: the
// block's 64 x 64 target tile is read once and kept in registers while the
// members are processed in turn.  Thread t owns rows t/16 + 16 s (s = 0..3),
// columns 4 (t % 16) .. + 3; the transposed copy goes through LDS, each
// thread writing 16 consecutive rows of one column (32 bytes).
__global__ void loss_grad(const float* Y, const float* T, int B, int Bt, int n_out, int E, int64_t strideY,
                          __bf16* dY, __bf16* dYt, int64_t strideD, float* part) {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
    __shared__ __align__(16) __bf16 tile[kTile][kTile + 8];
    __shared__ float red[4];
    const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
    const int64_t nblk = (int64_t)gridDim.x * gridDim.y, blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int c4 = (threadIdx.x & 15) * 4, r0 = threadIdx.x >> 4;
    const float inv = 1.0f / ((float)B * (float)n_out);
    const float ginv = 2.0f / (float)B;
    float4 tv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int m = m0 + r0 + 16 * q;
        tv[q] = m < B ? *reinterpret_cast<const float4*>(T + (int64_t)m * n_out + n0 + c4) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const int tc = threadIdx.x >> 2, tr = (threadIdx.x & 3) * 16;  // transposed: column, first row
    for (int e = 0; e < E; ++e) {
        float acc = 0.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 + 16 * q, m = m0 + r;
            float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
            if (m < B) {
                const float4 y = *reinterpret_cast<const float4*>(Y + e * strideY + (int64_t)m * n_out + n0 + c4);
                const float4 df = make_float4(y.x - tv[q].x, y.y - tv[q].y, y.z - tv[q].z, y.w - tv[q].w);
                acc += (df.x * df.x + df.y * df.y + df.z * df.z + df.w * df.w) * inv;
                g = make_float4(df.x * ginv, df.y * ginv, df.z * ginv, df.w * ginv);
            }
            const bf16x4 h = {(__bf16)g.x, (__bf16)g.y, (__bf16)g.z, (__bf16)g.w};
            *reinterpret_cast<bf16x4*>(dY + e * strideD + (int64_t)m * n_out + n0 + c4) = h;
            *reinterpret_cast<bf16x4*>(&tile[r][c4]) = h;
        }
        __syncthreads();
        bf16x8 lo, hi;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            lo[i] = tile[tr + i][tc];
            hi[i] = tile[tr + 8 + i][tc];
        }
        __bf16* dst = dYt + e * strideD + (int64_t)(n0 + tc) * Bt + m0 + tr;
        *reinterpret_cast<bf16x8*>(dst) = lo;
        *reinterpret_cast<bf16x8*>(dst + 8) = hi;
        if (part) {
            for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        }
        __syncthreads();  // the tile (and red) are rewritten by the next member
        if (part && threadIdx.x == 0) part[e * nblk + blk] = (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// loss[e] = sum over blocks of part[e][block], in a fixed order.  grid (E), block 256.
__global__ void sum_parts(const float* part, int64_t nblk, float* loss) {
    __shared__ float red[256];
    const float* p = part + (int64_t)blockIdx.x * nblk;
    float acc = 0.0f;
    for (int64_t i = threadIdx.x; i < nblk; i += blockDim.x) acc += p[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (unsigned st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[blockIdx.x] = red[0];
}

// db[e][o] = sum_m dZt[e][o][m]; one wave per row.  grid (ceil(out*E/4)), block 256.
__global__ void bias_grad(const __bf16* dZt, int out, int Bt, int E, int64_t strideD, float* db,
                          int64_t strideDb) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= out * E) return;
    const int e = row / out, o = row % out;
    const __bf16* p = dZt + e * strideD + (int64_t)o * Bt;
    float s = 0.0f;
    for (int m = lane; m < Bt; m += 64) s += (float)p[m];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) db[e * strideDb + o] = s;
}

// Adam on one weight matrix per member, [out][in] fp32; refreshes the BF16
// copies W [out][in] and Wt [in][out] (transposed through LDS).  step = 0
// only refreshes the copies.  grid (in/64, out/64, E), block 256.
__global__ void adam_weights(float* W, float* Mo, float* V, const float* G, __bf16* Wb, __bf16* Wt, int out,
                             int in, int64_t strideW, int64_t strideWb, int step, float lr, float b1,
                             float b2, float eps, float wd) {
    __shared__ __bf16 tile[kTile][kTile + 2];
    const int e = blockIdx.z;
    const int o0 = blockIdx.y * kTile, i0 = blockIdx.x * kTile;
    const float c1 = step > 0 ? 1.0f / (1.0f - powf(b1, (float)step)) : 0.0f;
    const float c2 = step > 0 ? 1.0f / (1.0f - powf(b2, (float)step)) : 0.0f;
    for (int t = threadIdx.x; t < kTile * kTile; t += blockDim.x) {
        const int r = t / kTile, c = t % kTile;
        const int64_t idx = e * strideW + (int64_t)(o0 + r) * in + (i0 + c);
        float w = W[idx];
        if (step > 0) {
            const float g = G[idx];
            const float m = b1 * Mo[idx] + (1.0f - b1) * g;
            const float v = b2 * V[idx] + (1.0f - b2) * g * g;
            Mo[idx] = m;
            V[idx] = v;
            w -= lr * ((m * c1) / (sqrtf(v * c2) + eps) + wd * w);
            W[idx] = w;
        }
        const __bf16 h = (__bf16)w;
        Wb[e * strideWb + (int64_t)(o0 + r) * in + (i0 + c)] = h;
        tile[r][c] = h;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kTile * kTile; t += blockDim.x) {
        const int c = t / kTile, r = t % kTile;
        Wt[e * strideWb + (int64_t)(i0 + c) * out + (o0 + r)] = tile[r][c];
    }
}

// Adam on a bias vector per member (no weight decay).
__global__ void adam_bias(float* b, float* Mo, float* V, const float* G, int n, int E, int64_t stride, int step,
                          float lr, float b1, float b2, float eps) {
    const int64_t total = (int64_t)n * E;
    const float c1 = 1.0f / (1.0f - powf(b1, (float)step));
    const float c2 = 1.0f / (1.0f - powf(b2, (float)step));
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(t / n), o = (int)(t % n);
        const int64_t idx = e * stride + o;
        const float g = G[idx];
        const float m = b1 * Mo[idx] + (1.0f - b1) * g;
        const float v = b2 * V[idx] + (1.0f - b2) * g * g;
        Mo[idx] = m;
        V[idx] = v;
        b[idx] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
    }
}

// Counter-based uniform in [-1, 1) (splitmix64 finaliser of seed ^ index).
__device__ __forceinline__ float hash_uniform(uint64_t seed, uint64_t i) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)((z >> 40) * (1.0 / 16777216.0)) * 2.0f - 1.0f;
}

// W ~ U(-a, a) for columns < in_used, 0 beyond; a per member layer.
__global__ void init_weights(float* W, int out, int in, int in_used, int E, int64_t stride, float a, uint64_t seed) {
    const int64_t total = (int64_t)out * in * E;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(t / ((int64_t)out * in));
        const int64_t r = t % ((int64_t)out * in);
        const int c = (int)(r % in);
        W[e * stride + r] = c < in_used ? a * hash_uniform(seed + 7919ull * e, (uint64_t)r) : 0.0f;
    }
}

__global__ void fill_f32(float* x, int64_t n, float v) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) x[t] = v;
}

// mean and spread over members: Y [E][Bt][n_out] -> mean, sigma [B][n_out]
// (rows < B); sigma is the sample standard deviation (0 for one member).
__global__ void ensemble_stats(const float* Y, int E, int B, int n_out, int64_t strideY, float* mean, float* sigma) {
    // one pass, four consecutive outputs per thread (n_out is a multiple of 128);
    // sums of the differences to member 0 keep the variance free of cancellation
    const int64_t total4 = (int64_t)B * n_out / 4;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total4; t += (int64_t)gridDim.x * blockDim.x) {
        const float4 y0 = reinterpret_cast<const float4*>(Y)[t];
        float4 s1 = make_float4(0.f, 0.f, 0.f, 0.f), s2 = s1;
        for (int e = 1; e < E; ++e) {
            const float4 y = reinterpret_cast<const float4*>(Y + e * strideY)[t];
            const float4 dl = make_float4(y.x - y0.x, y.y - y0.y, y.z - y0.z, y.w - y0.w);
            s1.x += dl.x; s1.y += dl.y; s1.z += dl.z; s1.w += dl.w;
            s2.x += dl.x * dl.x; s2.y += dl.y * dl.y; s2.z += dl.z * dl.z; s2.w += dl.w * dl.w;
        }
        const float inv = 1.0f / (float)E;
        reinterpret_cast<float4*>(mean)[t] =
            make_float4(y0.x + s1.x * inv, y0.y + s1.y * inv, y0.z + s1.z * inv, y0.w + s1.w * inv);
        if (sigma) {
            const float c = E > 1 ? 1.0f / (float)(E - 1) : 0.0f;
            auto sd = [&](float a, float b) { return sqrtf(fmaxf(b - a * a * inv, 0.0f) * c); };
            reinterpret_cast<float4*>(sigma)[t] = make_float4(sd(s1.x, s2.x), sd(s1.y, s2.y), sd(s1.z, s2.z), sd(s1.w, s2.w));
        }
    }
}

// Fallback selection, one workgroup of 256 threads per stack row b.  A unit is
// one (angle k, wavelength i) of the row, u = k * n_wl + i, with its P outputs
// at sigma[b][q * units + u]; it is flagged when some output has
// scale * sigma_w > bound (or a NaN sigma_w), sigma_w being the largest sigma of
// the output's (k, q) spectrum within win wavelengths of i.  A row whose units are all flagged is
// appended to stacks (recomputed by the dense kernel); otherwise its flagged
// units are appended to points as b * units + u (recomputed one by one).  Order
// within the lists is unspecified.  counts[0] = stacks, counts[1] = points.
__global__ void flag_units(const float* sigma, int units, int n_wl, int win, int P, float scale, float bound,
                           int* stacks, uint32_t* points, int* counts) {
    __shared__ int s_cnt;
    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const float* sg = sigma + (int64_t)b * units * P;
    auto flagged = [&](int u) {
        const int i = u % n_wl;
        const int lo = i - win > 0 ? i - win : 0, hi = i + win < n_wl - 1 ? i + win : n_wl - 1;
        bool f = false;
        for (int q = 0; q < P; ++q) {
            const float* row = sg + (int64_t)q * units + (u - i);
            // a NaN anywhere in the window flags the unit (fmaxf would drop it)
            float m = 0.0f;
            bool nan = false;
            for (int j = lo; j <= hi; ++j) {
                const float v = row[j];
                nan = nan || (v != v);
                m = fmaxf(m, v);
            }
            f = f || nan || !(scale * m <= bound);
        }
        return f;
    };
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    int cnt = 0;
    for (int u = threadIdx.x; u < units; u += blockDim.x) cnt += flagged(u) ? 1 : 0;
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if (lane == 0 && cnt) atomicAdd(&s_cnt, cnt);
    __syncthreads();
    const int total = s_cnt;
    if (total == 0) return;
    if (total == units) {
        if (threadIdx.x == 0) stacks[atomicAdd(&counts[0], 1)] = b;
        return;
    }
    // wave-level compaction: one counter update per wave and 64 units
    for (int u0 = threadIdx.x - lane; u0 < units; u0 += blockDim.x) {
        const int u = u0 + lane;
        const bool f = u < units && flagged(u);
        const unsigned long long m = __ballot(f);
        if (!m) continue;
        int base = 0;
        if (lane == 0) base = atomicAdd(&counts[1], __popcll(m));
        base = __shfl(base, 0, 64);
        if (f) {
            const int below = __popcll(m & ((1ull << lane) - 1ull));
            points[base + below] = (uint32_t)((int64_t)b * units + u);
        }
    }
}

__global__ void gather_stacks(const float* x, const int32_t* mat, const int* list, int n, int n_in, int L2,
                              float* dc, int32_t* matc) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * (n_in + L2); t += gridDim.x * blockDim.x) {
        const int i = t / (n_in + L2), j = t % (n_in + L2);
        const int b = list[i];
        if (j < n_in)
            dc[(int64_t)i * n_in + j] = x[(int64_t)b * n_in + j];
        else
            matc[(int64_t)i * L2 + (j - n_in)] = mat[(int64_t)b * L2 + (j - n_in)];
    }
}

__global__ void scatter_outputs(const float* Rc, const int* list, int n, int n_out, float* out) {
    const int64_t total = (int64_t)n * n_out;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / n_out), o = (int)(t % n_out);
        out[(int64_t)list[i] * n_out + o] = Rc[t];
    }
}

__global__ void zero_int(int* x, int n) {
    if (blockIdx.x == 0 && (int)threadIdx.x < n) x[threadIdx.x] = 0;
}

__global__ void copy_rows(const float* src, float* dst, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) dst[t] = src[t];
}

}  // namespace mlp
}  // namespace tmm

// ----------------------------------------------------------------------------
// The handle.

struct tmm_surrogate {
    tmm_surrogate_config cfg;
    int in_pad, Bt, E, NL;  // NL = number of linear layers = n_layers + 1
    std::vector<int> din, dout;
    std::vector<int64_t> woff, boff;  // per-member offsets (elements) of each layer
    int64_t wsz, bsz;                 // per-member total weights / biases
    int step;
    // parameters (all members, member stride wsz / bsz)
    float *W, *Wm, *Wv, *Wg;
    float *b, *bm, *bv, *bg;
    __bf16 *Wb, *Wt;
    // activations
    __bf16 *Xb, *Xt;
    std::vector<float*> Z;          // hidden pre-activations [E][Bt][H]
    std::vector<__bf16*> H, Ht;     // hidden activations [E][Bt][H], [E][H][Bt]
    float* Y;                       // [E][Bt][n_out]
    __bf16 *dY, *dYt;               // [E][Bt][n_out], [E][n_out][Bt]
    __bf16 *dZa, *dZat, *dZb, *dZbt;  // ping-pong hidden gradients
    float *mean_buf, *sigma_buf;    // [Bt][n_out]
    int* list;         // [Bt] stacks recomputed whole by the fallback
    uint32_t* plist;   // [Bt * n_out] units recomputed one by one
    int* count;        // [2]: stacks, units
    float* dc;         // [Bt][n_in] gathered thicknesses
    int32_t* matc;     // [Bt][n_in + 2] gathered material ids
    float* Rc;         // [Bt][n_out] dense fallback output
    float* loss_part;  // [E][blocks of loss_grad] per-block partial losses
};

namespace {

using tmm::fail;
using tmm::ok;

void free_all(tmm_surrogate* h) {
    void* ptrs[] = {h->W, h->Wm, h->Wv, h->Wg, h->b, h->bm, h->bv, h->bg, h->Wb, h->Wt, h->Xb, h->Xt,
                    h->Y, h->dY, h->dYt, h->dZa, h->dZat, h->dZb, h->dZbt, h->mean_buf, h->sigma_buf,
                    h->list, h->plist, h->count, h->dc, h->matc, h->Rc, h->loss_part};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (float* p : h->Z)
        if (p) (void)hipFree(p);
    for (__bf16* p : h->H)
        if (p) (void)hipFree(p);
    for (__bf16* p : h->Ht)
        if (p) (void)hipFree(p);
}

template <typename T>
bool dalloc(T** p, size_t n) {
    *p = nullptr;
    return hipMalloc((void**)p, n * sizeof(T)) == hipSuccess;
}

unsigned grid1(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g > 65535) g = 65535;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// Launch one batched NT GEMM (all members) with the given epilogue.  Every
// dimension is a multiple of 128.  Automatic tile (tile = 0): 256 x 256 (eight
// waves of 128 x 64) where it still gives at least four workgroups per CU, else
// 256 x 128 (eight waves of 64 x 64), else 128 x 128 (four waves of 64 x 64).
// tile = 1, 2, 3 forces one of the three where it divides M and N.
template <int EPI>
void gemm(hipStream_t s, int E, const tmm::mlp::GemmArgs& g, int tile) {
    const bool fit256 = g.M % 256 == 0 && g.N % 256 == 0, fit128 = g.M % 256 == 0;
    if ((tile == 1 && !fit256) || (tile == 2 && !fit128)) tile = 0;
    if (tile == 0) tile = fit256 && (int64_t)(g.M / 256) * (g.N / 256) * E >= 1024 ? 1 : fit128 ? 2 : 3;
    if (tile == 1) {
        hipLaunchKernelGGL((tmm::mlp::gemm_nt_bf16<EPI, 128, 64, 2, 4>), dim3(g.N / 256, g.M / 256, E), dim3(512), 0,
                           s, g);
    } else if (tile == 2) {
        hipLaunchKernelGGL((tmm::mlp::gemm_nt_bf16<EPI, 64, 64, 4, 2>), dim3(g.N / 128, g.M / 256, E), dim3(512), 0, s,
                           g);
    } else {
        hipLaunchKernelGGL((tmm::mlp::gemm_nt_bf16<EPI, 64, 64, 2, 2>), dim3(g.N / 128, g.M / 128, E), dim3(256), 0, s,
                           g);
    }
}

tmm::mlp::GemmArgs gargs(int M, int N, int K, const __bf16* A, int lda, int64_t sA, const __bf16* B, int ldb,
                         int64_t sB) {
    tmm::mlp::GemmArgs g;
    memset(&g, 0, sizeof(g));
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.lda = lda;
    g.strideA = sA;
    g.B = B;
    g.ldb = ldb;
    g.strideB = sB;
    return g;
}

// Forward of all members on the prepared input (Xb, Xt).  train: keep Z, H, Ht.
void forward(tmm_surrogate* h, hipStream_t s, bool train) {
    const int E = h->E, Bt = h->Bt, Hd = h->cfg.n_hidden;
    const __bf16* in = h->Xb;
    int in_dim = h->in_pad;
    int64_t in_stride = 0;  // the input is shared by all members
    for (int l = 0; l < h->NL; ++l) {
        const int out = h->dout[l];
        tmm::mlp::GemmArgs g = gargs(Bt, out, in_dim, in, in_dim, in_stride, h->Wb + h->woff[l], in_dim, h->wsz);
        g.bias = h->b + h->boff[l];
        g.strideBias = h->bsz;
        if (l < h->NL - 1) {
            const int64_t sH = (int64_t)Bt * Hd;
            g.outH = h->H[l];
            g.ldh = Hd;
            g.strideOutH = sH;
            if (train) {
                g.outF = h->Z[l];
                g.ldo = Hd;
                g.strideOutF = sH;
                g.outHt = h->Ht[l];
                g.ldt = Bt;
                g.strideOutHt = sH;
                gemm<tmm::mlp::EPI_BIAS_GELU>(s, E, g, h->cfg.gemm_tile);
            } else {
                gemm<tmm::mlp::EPI_BIAS_GELU_H>(s, E, g, h->cfg.gemm_tile);
            }
            in = h->H[l];
            in_dim = Hd;
            in_stride = sH;
        } else {
            g.outF = h->Y;
            g.ldo = out;
            g.strideOutF = (int64_t)Bt * out;
            gemm<tmm::mlp::EPI_BIAS_F32>(s, E, g, h->cfg.gemm_tile);
        }
    }
}

// Backward of all members after forward(train = true) and loss_grad: fills Wg, bg.
void backward(tmm_surrogate* h, hipStream_t s) {
    const int E = h->E, Bt = h->Bt, Hd = h->cfg.n_hidden;
    const __bf16* dZ = h->dY;
    const __bf16* dZt = h->dYt;
    int64_t sdz = (int64_t)Bt * h->cfg.n_out;
    bool use_a = true;
    for (int l = h->NL - 1; l >= 0; --l) {
        const int out = h->dout[l], in = h->din[l];
        // dW_l = dZt [out][Bt] x Xt_l [in][Bt]^T
        const __bf16* Xt = l == 0 ? h->Xt : h->Ht[l - 1];
        const int64_t sXt = l == 0 ? 0 : (int64_t)Bt * Hd;
        tmm::mlp::GemmArgs g = gargs(out, in, Bt, dZt, Bt, sdz, Xt, Bt, sXt);
        g.outF = h->Wg + h->woff[l];
        g.ldo = in;
        g.strideOutF = h->wsz;
        gemm<tmm::mlp::EPI_F32>(s, E, g, h->cfg.gemm_tile);
        hipLaunchKernelGGL(tmm::mlp::bias_grad, dim3((out * E + 3) / 4), dim3(256), 0, s, dZt, out, Bt, E, sdz,
                           h->bg + h->boff[l], h->bsz);
        if (l > 0) {
            // dZ_{l-1} = (dZ_l [Bt][out] x Wt_l [in][out]^T) * gelu'(Z_{l-1})
            __bf16* nz = use_a ? h->dZa : h->dZb;
            __bf16* nzt = use_a ? h->dZat : h->dZbt;
            tmm::mlp::GemmArgs g2 = gargs(Bt, in, out, dZ, out, sdz, h->Wt + h->woff[l], out, h->wsz);
            g2.zin = h->Z[l - 1];
            g2.ldz = Hd;
            g2.strideZin = (int64_t)Bt * Hd;
            g2.outH = nz;
            g2.ldh = Hd;
            g2.strideOutH = (int64_t)Bt * Hd;
            g2.outHt = nzt;
            g2.ldt = Bt;
            g2.strideOutHt = (int64_t)Bt * Hd;
            gemm<tmm::mlp::EPI_DGELU>(s, E, g2, h->cfg.gemm_tile);
            dZ = nz;
            dZt = nzt;
            sdz = (int64_t)Bt * Hd;
            use_a = !use_a;
        }
    }
}

void publish_weights(tmm_surrogate* h, hipStream_t s, bool update, float lr) {
    const tmm_surrogate_config& c = h->cfg;
    for (int l = 0; l < h->NL; ++l) {
        const int out = h->dout[l], in = h->din[l];
        dim3 grid(in / tmm::mlp::kTile, out / tmm::mlp::kTile, h->E);
        hipLaunchKernelGGL(tmm::mlp::adam_weights, grid, dim3(256), 0, s, h->W + h->woff[l], h->Wm + h->woff[l],
                           h->Wv + h->woff[l], h->Wg + h->woff[l], h->Wb + h->woff[l], h->Wt + h->woff[l], out, in,
                           h->wsz, h->wsz, update ? h->step : 0, lr, c.beta1, c.beta2, c.eps, c.weight_decay);
    }
    if (update)
        for (int l = 0; l < h->NL; ++l)
            hipLaunchKernelGGL(tmm::mlp::adam_bias, dim3(grid1((int64_t)h->dout[l] * h->E)), dim3(256), 0, s,
                               h->b + h->boff[l], h->bm + h->boff[l], h->bv + h->boff[l], h->bg + h->boff[l],
                               h->dout[l], h->E, h->bsz, h->step, lr, c.beta1, c.beta2, c.eps);
}

tmm_status prep(tmm_surrogate* h, const float* x, int B, hipStream_t s) {
    hipLaunchKernelGGL(tmm::mlp::prep_input, dim3(grid1((int64_t)h->Bt * h->in_pad)), dim3(256), 0, s, x, B,
                       h->cfg.n_in, h->in_pad, h->Bt, h->cfg.in_shift, h->cfg.in_scale, h->Xb, h->Xt);
    return ok();
}

tmm_status check_handle(const tmm_surrogate* h, const char* who) {
    if (!h) return fail(TMM_ERR_INVALID_ARG, "%s: handle is NULL", who);
    return ok();
}

}  // namespace

extern "C" {

tmm_status tmm_surrogate_create(const tmm_surrogate_config* c, tmm_surrogate** out) {
    if (!c || !out) return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_create: NULL argument");
    *out = nullptr;
    if (c->n_in < 1 || c->n_hidden < 128 || c->n_hidden % 128 || c->n_layers < 1 || c->n_out < 128 ||
        c->n_out % 128 || c->n_members < 1 || c->max_batch < 128 || c->max_batch % 128)
        return fail(TMM_ERR_INVALID_ARG,
                    "tmm_surrogate_create: need n_in >= 1, n_hidden and n_out multiples of 128, n_layers >= 1, "
                    "n_members >= 1, max_batch a multiple of 128");
    if ((int64_t)c->max_batch * c->n_out >= ((int64_t)1 << 32))
        return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_create: max_batch * n_out must stay below 2^32");
    if (c->gemm_tile < 0 || c->gemm_tile > 3)
        return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_create: gemm_tile must be 0 (automatic), 1, 2 or 3");
    if (c->sigma_window < 0 || c->sigma_window > 4096)
        return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_create: sigma_window must be in 0 .. 4096");
    if (!(c->in_scale == c->in_scale) || !(c->lr >= 0.0f) || !(c->beta1 >= 0.0f && c->beta1 < 1.0f) ||
        !(c->beta2 >= 0.0f && c->beta2 < 1.0f) || !(c->eps > 0.0f))
        return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_create: bad optimiser or input scaling parameters");
    tmm_surrogate* h = new tmm_surrogate();
    memset((void*)&h->cfg, 0, sizeof(h->cfg));
    h->cfg = *c;
    h->in_pad = (int)tmm::ceil_div(c->n_in, 128) * 128;
    h->Bt = c->max_batch;
    h->E = c->n_members;
    h->NL = c->n_layers + 1;
    h->step = 0;
    h->W = h->Wm = h->Wv = h->Wg = h->b = h->bm = h->bv = h->bg = nullptr;
    h->Wb = h->Wt = h->Xb = h->Xt = nullptr;
    h->Y = nullptr;
    h->dY = h->dYt = h->dZa = h->dZat = h->dZb = h->dZbt = nullptr;
    h->mean_buf = h->sigma_buf = nullptr;
    h->list = h->count = nullptr;
    h->plist = nullptr;
    h->dc = nullptr;
    h->matc = nullptr;
    h->Rc = nullptr;
    h->loss_part = nullptr;
    int64_t wo = 0, bo = 0;
    for (int l = 0; l < h->NL; ++l) {
        const int in = l == 0 ? h->in_pad : c->n_hidden;
        const int o = l == h->NL - 1 ? c->n_out : c->n_hidden;
        h->din.push_back(in);
        h->dout.push_back(o);
        h->woff.push_back(wo);
        h->boff.push_back(bo);
        wo += (int64_t)in * o;
        bo += o;
    }
    h->wsz = wo;
    h->bsz = bo;
    const int64_t E = h->E, Bt = h->Bt, Hd = c->n_hidden, No = c->n_out;
    bool okk = dalloc(&h->W, wo * E) && dalloc(&h->Wm, wo * E) && dalloc(&h->Wv, wo * E) && dalloc(&h->Wg, wo * E) &&
               dalloc(&h->b, bo * E) && dalloc(&h->bm, bo * E) && dalloc(&h->bv, bo * E) && dalloc(&h->bg, bo * E) &&
               dalloc(&h->Wb, wo * E) && dalloc(&h->Wt, wo * E) && dalloc(&h->Xb, Bt * h->in_pad) &&
               dalloc(&h->Xt, Bt * h->in_pad) && dalloc(&h->Y, E * Bt * No) && dalloc(&h->dY, E * Bt * No) &&
               dalloc(&h->dYt, E * Bt * No) && dalloc(&h->dZa, E * Bt * Hd) && dalloc(&h->dZat, E * Bt * Hd) &&
               dalloc(&h->dZb, E * Bt * Hd) && dalloc(&h->dZbt, E * Bt * Hd) && dalloc(&h->mean_buf, Bt * No) &&
               dalloc(&h->sigma_buf, Bt * No) && dalloc(&h->list, Bt) && dalloc(&h->count, 2) &&
               dalloc(&h->plist, Bt * No) && dalloc(&h->dc, Bt * c->n_in) &&
               dalloc(&h->matc, Bt * (c->n_in + 2)) && dalloc(&h->Rc, Bt * No) &&
               dalloc(&h->loss_part, E * (No / tmm::mlp::kTile) * (Bt / tmm::mlp::kTile));
    for (int l = 0; okk && l < c->n_layers; ++l) {
        float* z = nullptr;
        __bf16 *a = nullptr, *at = nullptr;
        okk = dalloc(&z, E * Bt * Hd) && dalloc(&a, E * Bt * Hd) && dalloc(&at, E * Bt * Hd);
        h->Z.push_back(z);
        h->H.push_back(a);
        h->Ht.push_back(at);
    }
    if (!okk) {
        free_all(h);
        delete h;
        return fail(TMM_ERR_HIP, "tmm_surrogate_create: device allocation failed");
    }
    // initial weights: U(-a, a), a = sqrt(6 / fan_in) (hidden) and sqrt(3 / fan_in) (output); zero biases
    hipStream_t s = nullptr;
    for (int l = 0; l < h->NL; ++l) {
        const int in_used = l == 0 ? c->n_in : h->din[l];
        const float a = sqrtf((l == h->NL - 1 ? 3.0f : 6.0f) / (float)in_used);
        hipLaunchKernelGGL(tmm::mlp::init_weights, dim3(grid1(h->wsz)), dim3(256), 0, s, h->W + h->woff[l],
                           h->dout[l], h->din[l], in_used, h->E, h->wsz, a, c->seed + 1000003ull * l);
    }
    hipLaunchKernelGGL(tmm::mlp::fill_f32, dim3(grid1(wo * E)), dim3(256), 0, s, h->Wm, wo * E, 0.0f);
    hipLaunchKernelGGL(tmm::mlp::fill_f32, dim3(grid1(wo * E)), dim3(256), 0, s, h->Wv, wo * E, 0.0f);
    hipLaunchKernelGGL(tmm::mlp::fill_f32, dim3(grid1(bo * E)), dim3(256), 0, s, h->b, bo * E, 0.0f);
    hipLaunchKernelGGL(tmm::mlp::fill_f32, dim3(grid1(bo * E)), dim3(256), 0, s, h->bm, bo * E, 0.0f);
    hipLaunchKernelGGL(tmm::mlp::fill_f32, dim3(grid1(bo * E)), dim3(256), 0, s, h->bv, bo * E, 0.0f);
    publish_weights(h, s, false, 0.0f);
    if (hipDeviceSynchronize() != hipSuccess || hipGetLastError() != hipSuccess) {
        free_all(h);
        delete h;
        return fail(TMM_ERR_HIP, "tmm_surrogate_create: initialisation failed");
    }
    *out = h;
    return ok();
}

tmm_status tmm_surrogate_destroy(tmm_surrogate* h) {
    if (!h) return ok();
    (void)hipDeviceSynchronize();
    free_all(h);
    delete h;
    return ok();
}

size_t tmm_surrogate_param_count(const tmm_surrogate* h) {
    return h ? (size_t)(h->wsz + h->bsz) : 0;
}

tmm_status tmm_surrogate_export(const tmm_surrogate* h, float* host, size_t n_floats) {
    tmm_status st = check_handle(h, "tmm_surrogate_export");
    if (st != TMM_OK) return st;
    const size_t per = (size_t)(h->wsz + h->bsz);
    if (!host || n_floats < per * h->E)
        return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_export: need %zu floats", per * h->E);
    if (hipDeviceSynchronize() != hipSuccess) return fail(TMM_ERR_HIP, "tmm_surrogate_export: sync failed");
    for (int e = 0; e < h->E; ++e) {
        if (hipMemcpy(host + per * e, h->W + (size_t)h->wsz * e, h->wsz * sizeof(float), hipMemcpyDeviceToHost) !=
                hipSuccess ||
            hipMemcpy(host + per * e + h->wsz, h->b + (size_t)h->bsz * e, h->bsz * sizeof(float),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return fail(TMM_ERR_HIP, "tmm_surrogate_export: copy failed");
    }
    return ok();
}

tmm_status tmm_surrogate_import(tmm_surrogate* h, const float* host, size_t n_floats) {
    tmm_status st = check_handle(h, "tmm_surrogate_import");
    if (st != TMM_OK) return st;
    const size_t per = (size_t)(h->wsz + h->bsz);
    if (!host || n_floats < per * h->E)
        return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_import: need %zu floats", per * h->E);
    if (hipDeviceSynchronize() != hipSuccess) return fail(TMM_ERR_HIP, "tmm_surrogate_import: sync failed");
    for (int e = 0; e < h->E; ++e) {
        if (hipMemcpy(h->W + (size_t)h->wsz * e, host + per * e, h->wsz * sizeof(float), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(h->b + (size_t)h->bsz * e, host + per * e + h->wsz, h->bsz * sizeof(float),
                      hipMemcpyHostToDevice) != hipSuccess)
            return fail(TMM_ERR_HIP, "tmm_surrogate_import: copy failed");
    }
    h->step = 0;
    const int64_t E = h->E;
    hipLaunchKernelGGL(tmm::mlp::fill_f32, dim3(grid1(h->wsz * E)), dim3(256), 0, 0, h->Wm, h->wsz * E, 0.0f);
    hipLaunchKernelGGL(tmm::mlp::fill_f32, dim3(grid1(h->wsz * E)), dim3(256), 0, 0, h->Wv, h->wsz * E, 0.0f);
    hipLaunchKernelGGL(tmm::mlp::fill_f32, dim3(grid1(h->bsz * E)), dim3(256), 0, 0, h->bm, h->bsz * E, 0.0f);
    hipLaunchKernelGGL(tmm::mlp::fill_f32, dim3(grid1(h->bsz * E)), dim3(256), 0, 0, h->bv, h->bsz * E, 0.0f);
    publish_weights(h, nullptr, false, 0.0f);
    if (hipDeviceSynchronize() != hipSuccess) return fail(TMM_ERR_HIP, "tmm_surrogate_import: publish failed");
    return tmm::check_launch("tmm_surrogate_import");
}

static tmm_status grads_common(tmm_surrogate* h, const float* x, const float* y, int32_t B, float* loss,
                               hipStream_t s, const char* who) {
    tmm_status st = check_handle(h, who);
    if (st != TMM_OK) return st;
    if (!x || !y) return fail(TMM_ERR_INVALID_ARG, "%s: x and y must be non-NULL", who);
    if (B < 1 || B > h->Bt) return fail(TMM_ERR_INVALID_ARG, "%s: batch %d outside [1, %d]", who, B, h->Bt);
    (void)hipGetLastError();
    prep(h, x, B, s);
    forward(h, s, true);
    dim3 grid(h->cfg.n_out / tmm::mlp::kTile, h->Bt / tmm::mlp::kTile);
    hipLaunchKernelGGL(tmm::mlp::loss_grad, grid, dim3(256), 0, s, h->Y, y, (int)B, h->Bt, h->cfg.n_out, h->E,
                       (int64_t)h->Bt * h->cfg.n_out, h->dY, h->dYt, (int64_t)h->Bt * h->cfg.n_out,
                       loss ? h->loss_part : nullptr);
    if (loss)
        hipLaunchKernelGGL(tmm::mlp::sum_parts, dim3(h->E), dim3(256), 0, s, h->loss_part,
                           (int64_t)grid.x * grid.y, loss);
    backward(h, s);
    return tmm::check_launch(who);
}

tmm_status tmm_surrogate_train_step(tmm_surrogate* h, const float* x, const float* y, int32_t B, float lr,
                                    float* loss, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (h && !(lr >= 0.0f)) return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_train_step: lr must be >= 0");
    tmm_status st = grads_common(h, x, y, B, loss, s, "tmm_surrogate_train_step");
    if (st != TMM_OK) return st;
    h->step += 1;
    publish_weights(h, s, true, lr);
    return tmm::check_launch("tmm_surrogate_train_step");
}

tmm_status tmm_surrogate_gradients(tmm_surrogate* h, const float* x, const float* y, int32_t B, float* grads,
                                   void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!grads) return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_gradients: grads is NULL");
    tmm_status st = grads_common(h, x, y, B, nullptr, s, "tmm_surrogate_gradients");
    if (st != TMM_OK) return st;
    const int64_t per = h->wsz + h->bsz;
    for (int e = 0; e < h->E; ++e) {
        hipLaunchKernelGGL(tmm::mlp::copy_rows, dim3(grid1(h->wsz)), dim3(256), 0, s, h->Wg + h->wsz * e,
                           grads + per * e, h->wsz);
        hipLaunchKernelGGL(tmm::mlp::copy_rows, dim3(grid1(h->bsz)), dim3(256), 0, s, h->bg + h->bsz * e,
                           grads + per * e + h->wsz, h->bsz);
    }
    return tmm::check_launch("tmm_surrogate_gradients");
}

tmm_status tmm_surrogate_predict(tmm_surrogate* h, const float* x, int32_t B, float* mean, float* sigma,
                                 float* members, void* stream) {
    tmm_status st = check_handle(h, "tmm_surrogate_predict");
    if (st != TMM_OK) return st;
    if (!x || (!mean && !members)) return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_predict: NULL argument");
    if (B < 0) return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_predict: negative batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int No = h->cfg.n_out;
    (void)hipGetLastError();
    for (int b0 = 0; b0 < B; b0 += h->Bt) {
        const int nb = B - b0 < h->Bt ? B - b0 : h->Bt;
        prep(h, x + (int64_t)b0 * h->cfg.n_in, nb, s);
        forward(h, s, false);
        if (mean)
            hipLaunchKernelGGL(tmm::mlp::ensemble_stats, dim3(grid1((int64_t)nb * No / 4)), dim3(256), 0, s, h->Y, h->E,
                               nb, No, (int64_t)h->Bt * No, mean + (int64_t)b0 * No,
                               sigma ? sigma + (int64_t)b0 * No : nullptr);
        if (members)
            for (int e = 0; e < h->E; ++e)
                hipLaunchKernelGGL(tmm::mlp::copy_rows, dim3(grid1((int64_t)nb * No)), dim3(256), 0, s,
                                   h->Y + (int64_t)e * h->Bt * No, members + ((int64_t)e * B + b0) * No,
                                   (int64_t)nb * No);
    }
    return tmm::check_launch("tmm_surrogate_predict");
}

tmm_status tmm_surrogate_predict_fallback(tmm_surrogate* h, const float* x, int32_t B, const tmm_rt_args* tmpl,
                                          float err_scale, float bound, float* out, int64_t* n_fallback,
                                          void* stream) {
    tmm_status st = check_handle(h, "tmm_surrogate_predict_fallback");
    if (st != TMM_OK) return st;
    if (!x || !out || !tmpl) return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_predict_fallback: NULL argument");
    const int No = h->cfg.n_out;
    const int P = tmpl->pol_mask == 3u ? 2 : 1;
    if (tmpl->L != h->cfg.n_in || !tmpl->mat || tmpl->B != B || (int64_t)P * tmpl->n_theta * tmpl->n_wl != No)
        return fail(TMM_ERR_INVALID_ARG,
                    "tmm_surrogate_predict_fallback: the template must describe the same B stacks with "
                    "L = n_in layers, material ids, and P * n_theta * n_wl = n_out");
    if (!(err_scale >= 0.0f) || !(bound >= 0.0f))
        return fail(TMM_ERR_INVALID_ARG, "tmm_surrogate_predict_fallback: err_scale and bound must be >= 0");
    {
        tmm_rt_args tc = *tmpl;  // the template's own d and outputs are ignored
        tc.d = x;
        tc.R = out;
        tc.T = tc.r = tc.t = nullptr;
        tc.flags = 0;
        st = tmm::check_rt_args(&tc, "tmm_surrogate_predict_fallback", true);
        if (st != TMM_OK) return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int L2 = tmpl->L + 2;
    const int units = tmpl->n_theta * tmpl->n_wl;
    int64_t replaced = 0;
    (void)hipGetLastError();
    for (int b0 = 0; b0 < B; b0 += h->Bt) {
        const int nb = B - b0 < h->Bt ? B - b0 : h->Bt;
        const float* xc = x + (int64_t)b0 * h->cfg.n_in;
        float* oc = out + (int64_t)b0 * No;
        const int32_t* mc = tmpl->mat + (int64_t)b0 * L2;
        prep(h, xc, nb, s);
        forward(h, s, false);
        hipLaunchKernelGGL(tmm::mlp::ensemble_stats, dim3(grid1((int64_t)nb * No / 4)), dim3(256), 0, s, h->Y, h->E, nb,
                           No, (int64_t)h->Bt * No, oc, h->sigma_buf);
        hipLaunchKernelGGL(tmm::mlp::zero_int, dim3(1), dim3(64), 0, s, h->count, 2);
        hipLaunchKernelGGL(tmm::mlp::flag_units, dim3(nb), dim3(256), 0, s, h->sigma_buf, units, tmpl->n_wl,
                           h->cfg.sigma_window, P, err_scale, bound, h->list, h->plist, h->count);
        int cnt[2] = {0, 0};
        if (hipMemcpyAsync(cnt, h->count, sizeof(cnt), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(TMM_ERR_HIP, "tmm_surrogate_predict_fallback: count readback failed");
        const int nf = cnt[0], npt = cnt[1];
        replaced += (int64_t)nf * No + (int64_t)npt * P;
        if (nf > 0) {
            // stacks flagged everywhere: the dense kernel on the gathered stacks
            hipLaunchKernelGGL(tmm::mlp::gather_stacks, dim3(grid1((int64_t)nf * (h->cfg.n_in + L2))), dim3(256), 0, s,
                               xc, mc, h->list, nf, h->cfg.n_in, L2, h->dc, h->matc);
            tmm_rt_args a = *tmpl;
            a.B = nf;
            a.d = h->dc;
            a.mat = h->matc;
            a.R = h->Rc;
            a.T = nullptr;
            a.r = nullptr;
            a.t = nullptr;
            a.flags = 0;
            st = tmm_rt(&a, TMM_F32, stream);
            if (st != TMM_OK) return st;
            hipLaunchKernelGGL(tmm::mlp::scatter_outputs, dim3(grid1((int64_t)nf * No)), dim3(256), 0, s, h->Rc,
                               h->list, nf, No, oc);
        }
        if (npt > 0) {
            // the flagged points of the other stacks, written in place into out
            tmm::pts::PtParams<float> p;
            p.B = nb;
            p.L = tmpl->L;
            p.n_wl = tmpl->n_wl;
            p.n_theta = tmpl->n_theta;
            p.d = xc;
            p.nk = static_cast<const float*>(tmpl->nk);
            p.n_mat = tmpl->n_mat;
            p.dispersive = tmpl->dispersive;
            p.mat = mc;
            p.wl = static_cast<const float*>(tmpl->wl);
            p.sin_t = static_cast<const float*>(tmpl->sin_theta);
            p.cos_t = static_cast<const float*>(tmpl->cos_theta);
            p.R_out = oc;
            p.T_out = nullptr;
            p.r_out = p.t_out = nullptr;
            p.pts64 = nullptr;
            p.pts32 = h->plist;
            p.n_pts = npt;
            p.n_dev = nullptr;
            if (tmm::pts::launch_points<float>(p, tmpl->pol_mask, npt, s) != hipSuccess)
                return tmm::check_launch("tmm_surrogate_predict_fallback");
        }
    }
    if (n_fallback) *n_fallback = replaced;
    return tmm::check_launch("tmm_surrogate_predict_fallback");
}

}  // extern "C"
