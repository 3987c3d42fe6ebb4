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
// Tile: 128 x 128 outputs per 256-thread workgroup, 32 reduction steps per LDS
// stage, four waves each owning a 64 x 64 quadrant = 2 x 2 blocks of the
// 32x32x16 BF16 MFMA (FP32 accumulation).  MFMA operand layout used: lane l
// supplies row/column (l mod 32) and 8 consecutive reduction indices starting
// at 8 (l / 32); accumulator element r of lane l is C[8 (r/4) + 4 (l/32) + r mod 4][l mod 32].
// (Any consistent permutation of the 16 reduction indices gives the same sum.)
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace tmm {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBM = 128, kBN = 128, kBK = 32;
constexpr int kLdsRow = kBK + 8;  // padded row (bf16 elements) against bank conflicts
constexpr int kGemmThreads = 256;

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

__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
    const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * __expf(-0.5f * z * z);
    return cdf + z * pdf;
}

template <int EPI>
__global__ void __launch_bounds__(kGemmThreads) gemm_nt_bf16(GemmArgs g) {
    __shared__ __align__(16) __bf16 As[2][kBM * kLdsRow];
    __shared__ __align__(16) __bf16 Bs[2][kBN * kLdsRow];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int z = blockIdx.z;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const __bf16* A = g.A + z * g.strideA + (int64_t)m0 * g.lda;
    const __bf16* B = g.B + z * g.strideB + (int64_t)n0 * g.ldb;

    // global -> register staging: each thread moves 2 chunks of 8 bf16 for A and B
    // chunk c = tid + 256 s (s = 0, 1): row c / 4, columns 8 (c % 4) .. + 7
    uint4 ra[2], rb[2];
    auto gload = [&](int kt) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int c = tid + kGemmThreads * s;
            const int row = c >> 2, col = (c & 3) * 8;
            ra[s] = *reinterpret_cast<const uint4*>(A + (int64_t)row * g.lda + kt * kBK + col);
            rb[s] = *reinterpret_cast<const uint4*>(B + (int64_t)row * g.ldb + kt * kBK + col);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int c = tid + kGemmThreads * s;
            const int row = c >> 2, col = (c & 3) * 8;
            *reinterpret_cast<uint4*>(&As[buf][row * kLdsRow + col]) = ra[s];
            *reinterpret_cast<uint4*>(&Bs[buf][row * kLdsRow + col]) = rb[s];
        }
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int fr = lane & 31, fk = (lane >> 5) * 8;
    const int KT = g.K / kBK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < KT; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < KT) gload(kt + 1);
#pragma unroll
        for (int kk = 0; kk < kBK; kk += 16) {
            bf16x8 af[2], bfr[2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                af[a] = *reinterpret_cast<const bf16x8*>(&As[buf][(wm + 32 * a + fr) * kLdsRow + kk + fk]);
#pragma unroll
            for (int b = 0; b < 2; ++b)
                bfr[b] = *reinterpret_cast<const bf16x8*>(&Bs[buf][(wn + 32 * b + fr) * kLdsRow + kk + fk]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        }
        if (kt + 1 < KT) {
            sstore(buf ^ 1);
            __syncthreads();
        }
    }

    // epilogue
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int n = n0 + wn + 32 * b + (lane & 31);
            float bias = 0.0f;
            if (EPI == EPI_BIAS_GELU || EPI == EPI_BIAS_F32 || EPI == EPI_BIAS_GELU_H)
                bias = g.bias[z * g.strideBias + n];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wm + 32 * a + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const float v = acc[a][b][r];
                if (EPI == EPI_F32) {
                    g.outF[z * g.strideOutF + (int64_t)m * g.ldo + n] = v;
                } else if (EPI == EPI_BIAS_F32) {
                    g.outF[z * g.strideOutF + (int64_t)m * g.ldo + n] = v + bias;
                } else if (EPI == EPI_BIAS_GELU) {
                    const float zz = v + bias;
                    g.outF[z * g.strideOutF + (int64_t)m * g.ldo + n] = zz;
                    const __bf16 h = (__bf16)gelu(zz);
                    g.outH[z * g.strideOutH + (int64_t)m * g.ldh + n] = h;
                    g.outHt[z * g.strideOutHt + (int64_t)n * g.ldt + m] = h;
                } else if (EPI == EPI_BIAS_GELU_H) {
                    g.outH[z * g.strideOutH + (int64_t)m * g.ldh + n] = (__bf16)gelu(v + bias);
                } else {  // EPI_DGELU
                    const float zz = g.zin[z * g.strideZin + (int64_t)m * g.ldz + n];
                    const __bf16 h = (__bf16)(v * gelu_grad(zz));
                    g.outH[z * g.strideOutH + (int64_t)m * g.ldh + n] = h;
                    g.outHt[z * g.strideOutHt + (int64_t)n * g.ldt + m] = h;
                }
            }
        }
    }
}

}  // namespace mlp
}  // namespace tmm
