// BF16 MFMA kernels of the learned surrogate (gfx950).
//
// Every matrix product of the MLP is written as  C[M][N] = sum_k A[m][k] B[n][k]
// with both operands stored row-major and contiguous along the reduction index
// k, so every global-to-LDS copy is a straight 16-byte move:
//   forward   Y  = X  W^T      A = X  [batch][in],    B = W  [out][in]
//   dX        dH = dZ W        A = dZ [batch][out],   B = Wt [in][out]   (transposed weight copy)
//   dW        dW = dZ^T X      A = dZt [out][batch],  B = Xt [in][batch] (transposed activations)
// The transposed copies are written by the producers (optimizer, forward and
// backward epilogues), not by separate transposes.
//
// Tile: NWM x NWN waves, each owning WM x WN outputs (WM/32 x WN/32 blocks of
// the 32x32x16 BF16 MFMA, FP32 accumulation), so a workgroup covers
// (NWM WM) x (NWN WN).  64 reduction steps per LDS stage (double-buffered, rows
// padded by 16 bytes against bank conflicts; up to 144 KiB of LDS).  The large
// shapes use eight waves (two per SIMD, 128 x 64 or 64 x 64 per wave): while
// one wave of a SIMD waits on LDS, global memory or its epilogue, the other
// keeps the matrix unit busy.  MFMA operand layout used: lane l supplies
// row/column (l mod 32) and 8 consecutive reduction indices starting at
// 8 (l / 32); accumulator element r of lane l is
// C[8 (r/4) + 4 (l/32) + r mod 4][l mod 32].  (Any consistent permutation of the
// 16 reduction indices gives the same sum.)
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace tmm {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte chunk

constexpr int kBK = 64;
constexpr int kLdsRow = kBK + 8;  // padded row (bf16 elements): 144 B = 9 x 16 B, no ds_read_b128 bank conflicts
constexpr int kChunksPerRow = kBK / 8;  // 16-byte chunks per tile row

enum Epilogue : int {
    EPI_F32 = 0,        // C fp32 [m][n]
    EPI_BIAS_GELU = 1,  // Z = C + bias (fp32 [m][n]); H = gelu(Z) bf16 [m][n] and [n][m]
    EPI_BIAS_F32 = 2,   // Y = C + bias (fp32 [m][n])
    EPI_DGELU = 3,      // dZ = C * gelu'(Zprev[m][n]) bf16 [m][n] and [n][m]
    EPI_BIAS_GELU_H = 4 // H = gelu(C + bias) bf16 [m][n] only (inference)
};

struct GemmArgs {
    int M, N, K;
    const __bf16* A;  // [M][lda]
    const __bf16* B;  // [N][ldb]
    int lda, ldb;
    int64_t strideA, strideB;  // per ensemble member (blockIdx.z), elements
    const float* bias;         // [N] (EPI_BIAS_*), stride strideBias
    int64_t strideBias;
    const float* zin;          // EPI_DGELU: pre-activations [M][ldz]
    int ldz;
    int64_t strideZin;
    float* outF;               // fp32 output [M][ldo]
    int ldo;
    int64_t strideOutF;
    __bf16* outH;              // bf16 output [M][ldh]
    int ldh;
    int64_t strideOutH;
    __bf16* outHt;             // bf16 transposed output [N][ldt]
    int ldt;
    int64_t strideOutHt;
};

// erf without branches (gen_poly.py fits, coefficients lowest degree first;
// max abs error 1.2e-7 in FP32):
//   |x| < 0.875:  erf(x) = x * P(x^2)
//   otherwise:    erf(|x|) = 1 - 2^Q(min(|x|, 4))  with Q ~ log2 erfc
// (erfc(4) = 1.5e-8, below half an ulp of 1).  Both pieces are evaluated and one
// is selected, so a wave never splits into two paths.
constexpr float kErfSmall[6] = {1.128379107e+00f, -3.761255443e-01f, 1.128249690e-01f,
                                -2.679294720e-02f, 5.034370814e-03f, -6.214585155e-04f};
constexpr float kErfcLog2[9] = {4.546713317e-04f,  -1.630561113e+00f, -9.115559459e-01f,
                                -1.588001102e-01f, 3.811602667e-02f,  -6.867640652e-03f,
                                8.615075494e-04f,  -6.653598393e-05f, 2.367627530e-06f};
__device__ __forceinline__ float erf_fit(float x) {
    const float a = fabsf(x), s = a * a;
    float p = kErfSmall[5];
#pragma unroll
    for (int i = 4; i >= 0; --i) p = fmaf(p, s, kErfSmall[i]);
    const float t = fminf(a, 4.0f);
    float q = kErfcLog2[8];
#pragma unroll
    for (int i = 7; i >= 0; --i) q = fmaf(q, t, kErfcLog2[i]);
    const float r = a < 0.875f ? a * p : 1.0f - __builtin_amdgcn_exp2f(q);
    return copysignf(r, x);
}
__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + erf_fit(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
    const float cdf = 0.5f * (1.0f + erf_fit(z * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * __expf(-0.5f * z * z);
    return cdf + z * pdf;
}

// One K stage of a tile: global -> registers (chunk s of this thread is row
// r0 + RPP s, RPP = threads / 8 rows per pass of the workgroup, so its address is
// the thread's base plus s passes), and registers -> LDS (the same rows at the
// padded pitch).
template <int C, int RPP>
__device__ __forceinline__ void stage_load(u32x4 (&r)[C], const __bf16* base, int64_t ld, int kt) {
#pragma unroll
    for (int s = 0; s < C; ++s)
        r[s] = *reinterpret_cast<const u32x4*>(base + (int64_t)s * RPP * ld + kt * kBK);
}
template <int C, int RPP>
__device__ __forceinline__ void stage_store(const u32x4 (&r)[C], __bf16* lds) {
#pragma unroll
    for (int s = 0; s < C; ++s) *reinterpret_cast<u32x4*>(lds + s * RPP * kLdsRow) = r[s];
}

template <int EPI, int WM, int WN, int NWM, int NWN>
__global__ void __launch_bounds__(64 * NWM * NWN) gemm_nt_bf16(GemmArgs g) {
    constexpr int NT = 64 * NWM * NWN;                  // threads
    constexpr int BM = NWM * WM, BN = NWN * WN;
    constexpr int FM = WM / 32, FN = WN / 32;           // MFMA blocks per wave
    constexpr int RPP = NT / kChunksPerRow;             // tile rows per pass of the workgroup
    constexpr int CA = BM * kChunksPerRow / NT;         // 16-byte chunks per thread and stage
    constexpr int CB = BN * kChunksPerRow / NT;
    static_assert(CA * NT == BM * kChunksPerRow && CB * NT == BN * kChunksPerRow, "tile not covered");
    __shared__ __align__(16) __bf16 As[2][BM * kLdsRow];
    __shared__ __align__(16) __bf16 Bs[2][BN * kLdsRow];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int z = blockIdx.z;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const __bf16* A = g.A + z * g.strideA + (int64_t)m0 * g.lda;
    const __bf16* B = g.B + z * g.strideB + (int64_t)n0 * g.ldb;

    // global -> register staging: chunk c = tid + 256 s is row c / 8, columns 8 (c % 8) .. + 7;
    // the row offsets are fixed for the whole loop.  Two register sets: the loads of
    // stage kt + 2 are issued while stage kt is multiplied, so each load has two
    // stages of MFMA work to arrive before it is written to LDS.
    u32x4 ra0[CA], rb0[CB], ra1[CA], rb1[CB];
    const int r0 = tid / kChunksPerRow, c0 = (tid % kChunksPerRow) * 8;
    const __bf16* const a0 = A + (int64_t)r0 * g.lda + c0;
    const __bf16* const b0 = B + (int64_t)r0 * g.ldb + c0;
    const int l0 = r0 * kLdsRow + c0;
    auto load = [&](u32x4 (&ra)[CA], u32x4 (&rb)[CB], int kt) __attribute__((always_inline)) {
        stage_load<CA, RPP>(ra, a0, g.lda, kt);
        stage_load<CB, RPP>(rb, b0, g.ldb, kt);
    };
    auto store = [&](const u32x4 (&ra)[CA], const u32x4 (&rb)[CB], int buf) __attribute__((always_inline)) {
        stage_store<CA, RPP>(ra, &As[buf][l0]);
        stage_store<CB, RPP>(rb, &Bs[buf][l0]);
    };

    f32x16 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    const int wm = (wave / NWN) * WM, wn = (wave % NWN) * WN;
    const int fr = lane & 31, fk = (lane >> 5) * 8;
    // One LDS stage: four 16-deep MFMA steps.
    auto compute = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 16) {
            bf16x8 af[FM], bfr[FN];
#pragma unroll
            for (int a = 0; a < FM; ++a)
                af[a] = *reinterpret_cast<const bf16x8*>(&As[buf][(wm + 32 * a + fr) * kLdsRow + kk + fk]);
#pragma unroll
            for (int b = 0; b < FN; ++b)
                bfr[b] = *reinterpret_cast<const bf16x8*>(&Bs[buf][(wn + 32 * b + fr) * kLdsRow + kk + fk]);
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
            // scheduling hint: alternate the fragment reads with the first MFMAs
#pragma unroll
            for (int i = 0; i < FM + FN; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
            }
            __builtin_amdgcn_sched_group_barrier(0x008, FM * FN - FM - FN, 0);
        }
    };
    // K is a multiple of 2 kBK (every dimension is a multiple of 128); stage indices
    // past the end are clamped (those loads and stores are harmless repeats).
    const int KT = g.K / kBK;
    load(ra0, rb0, 0);
    store(ra0, rb0, 0);
    load(ra1, rb1, 1 < KT ? 1 : 0);
    __syncthreads();
    for (int kt = 0; kt < KT; kt += 2) {
        // stage kt in LDS buffer 0, stage kt + 1 in set 1
        load(ra0, rb0, kt + 2 < KT ? kt + 2 : KT - 1);
        compute(0);
        store(ra1, rb1, 1);  // buffer 1 was last read before the previous barrier
        __syncthreads();
        // stage kt + 1 in LDS buffer 1, stage kt + 2 in set 0
        load(ra1, rb1, kt + 3 < KT ? kt + 3 : KT - 1);
        compute(1);
        store(ra0, rb0, 0);
        __syncthreads();
    }

    // epilogue: lane owns column n of every block and rows 8 q + 4 (lane / 32) + 0..3, q = 0..3
#pragma unroll
    for (int a = 0; a < FM; ++a) {
#pragma unroll
        for (int b = 0; b < FN; ++b) {
            const int n = n0 + wn + 32 * b + (lane & 31);
            float bias = 0.0f;
            if (EPI == EPI_BIAS_GELU || EPI == EPI_BIAS_F32 || EPI == EPI_BIAS_GELU_H)
                bias = g.bias[z * g.strideBias + n];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int mb = m0 + wm + 32 * a + 8 * q + 4 * (lane >> 5);
                __bf16 ht[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = mb + i;
                    const float v = acc[a][b][4 * q + i];
                    if (EPI == EPI_F32) {
                        g.outF[z * g.strideOutF + (int64_t)m * g.ldo + n] = v;
                    } else if (EPI == EPI_BIAS_F32) {
                        g.outF[z * g.strideOutF + (int64_t)m * g.ldo + n] = v + bias;
                    } else if (EPI == EPI_BIAS_GELU) {
                        const float zz = v + bias;
                        g.outF[z * g.strideOutF + (int64_t)m * g.ldo + n] = zz;
                        ht[i] = (__bf16)gelu(zz);
                        g.outH[z * g.strideOutH + (int64_t)m * g.ldh + n] = ht[i];
                    } else if (EPI == EPI_BIAS_GELU_H) {
                        g.outH[z * g.strideOutH + (int64_t)m * g.ldh + n] = (__bf16)gelu(v + bias);
                    } else {  // EPI_DGELU
                        const float zz = g.zin[z * g.strideZin + (int64_t)m * g.ldz + n];
                        ht[i] = (__bf16)(v * gelu_grad(zz));
                        g.outH[z * g.strideOutH + (int64_t)m * g.ldh + n] = ht[i];
                    }
                }
                if (EPI == EPI_BIAS_GELU || EPI == EPI_DGELU) {
                    // rows mb .. mb + 3 of the transposed copy are consecutive: one 8-byte store
                    __bf16 __attribute__((ext_vector_type(4))) v4 = {ht[0], ht[1], ht[2], ht[3]};
                    *reinterpret_cast<decltype(v4)*>(&g.outHt[z * g.strideOutHt + (int64_t)n * g.ldt + mb]) = v4;
                }
            }
        }
    }
}

}  // namespace mlp
}  // namespace tmm
