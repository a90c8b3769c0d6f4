// Device helpers of the learned initialiser shared by the training kernels and
// the fragment kernel: BF16 conversion, tanh, the PCG hash and MLP inference.
#pragma once
#include <hip/hip_runtime.h>

#include "ivr_mlp.h"

namespace ivr {

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ float tanh_fast(float x) { return 1.0f - 2.0f / (__expf(2.0f * x) + 1.0f); }

// PCG hash (Jarzynski & Olano, "Hash Functions for GPU Rendering", JCGT 2020).
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}
__device__ __forceinline__ float u01(uint32_t h) { return float(h >> 8) * (1.0f / 16777216.0f); }

// p = MLP_q(x) from block q's BF16 weights; x in world coordinates.
__device__ __forceinline__ void mlp_infer(const uint16_t *wball, const float *normall, int q,
                                          const float (&x)[3], float (&p)[3]) {
    const uint16_t *wb = wball + (size_t)q * kMlpWbStride;
    const float *nm = normall + 12 * q;
    const float xh[3] = {(x[0] - nm[6]) * nm[3], (x[1] - nm[7]) * nm[4], (x[2] - nm[8]) * nm[5]};
    float h1[kMlpH];
#pragma unroll
    for (int n = 0; n < kMlpH; ++n)
        h1[n] = tanh_fast(bf2f(wb[kOffB1 + n]) + xh[0] * bf2f(wb[kOffW1 + n]) +
                          xh[1] * bf2f(wb[kOffW1 + 64 + n]) + xh[2] * bf2f(wb[kOffW1 + 128 + n]));
    float y[3] = {bf2f(wb[kOffB3]), bf2f(wb[kOffB3 + 1]), bf2f(wb[kOffB3 + 2])};
    for (int n = 0; n < kMlpH; ++n) {
        float z = bf2f(wb[kOffB2 + n]);
#pragma unroll
        for (int k = 0; k < kMlpH; ++k) z += h1[k] * bf2f(wb[kOffW2 + k * 64 + n]);
        const float h2 = tanh_fast(z);
#pragma unroll
        for (int c = 0; c < 3; ++c) y[c] += h2 * bf2f(wb[kOffW3 + n * 3 + c]);
    }
    p[0] = y[0]; p[1] = y[1]; p[2] = y[2];
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// MLP of one block (wave-uniform q) for the 64 points of a wave: layer 1 and 3
// per lane on the VALU, the 64x64 layer as a 64-row GEMM on
// v_mfma_f32_16x16x16_bf16 (lane l holds A[l%16][4(l/16)+j], B[4(l/16)+j][l%16],
// D[4(l/16)+j][l%16]).  sA: 64*72 BF16 and sY: 64*4 floats of LDS owned by the
// wave.  Every lane of the wave must execute this.
__device__ __forceinline__ void mlp_infer_wave(const uint16_t *wball, const float *normall, int q,
                                               const float (&x)[3], float (&p)[3], uint16_t *sA,
                                               float *sY) {
    const int l = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int lr16 = l & 15, lg = l >> 4;
    const uint16_t *wb = wball + (size_t)q * kMlpWbStride;
    const float *nm = normall + 12 * q;
    const float xh[3] = {(x[0] - nm[6]) * nm[3], (x[1] - nm[7]) * nm[4], (x[2] - nm[8]) * nm[5]};
    uint32_t *row = reinterpret_cast<uint32_t *>(sA + l * 72);
#pragma unroll
    for (int n = 0; n < kMlpH; n += 2) {
        const float h0 = tanh_fast(bf2f(wb[kOffB1 + n]) + xh[0] * bf2f(wb[kOffW1 + n]) +
                                   xh[1] * bf2f(wb[kOffW1 + 64 + n]) + xh[2] * bf2f(wb[kOffW1 + 128 + n]));
        const float h1 = tanh_fast(bf2f(wb[kOffB1 + n + 1]) + xh[0] * bf2f(wb[kOffW1 + n + 1]) +
                                   xh[1] * bf2f(wb[kOffW1 + 64 + n + 1]) + xh[2] * bf2f(wb[kOffW1 + 128 + n + 1]));
        row[n >> 1] = (uint32_t)f2bf(h0) | ((uint32_t)f2bf(h1) << 16);
    }
    __syncthreads();
    f32x4 acc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rb][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
        bf16x4 a[4], b[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
            a[rb] = *reinterpret_cast<const bf16x4 *>(sA + (rb * 16 + lr16) * 72 + ks * 16 + 4 * lg);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
            b[ct] = *reinterpret_cast<const bf16x4 *>(wb + kOffW2T + (ct * 16 + lr16) * 64 + ks * 16 + 4 * lg);
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                acc[rb][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[rb], b[ct], acc[rb][ct], 0, 0, 0);
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float y[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const int n = ct * 16 + lr16;
                const float h2 = tanh_fast(acc[rb][ct][j] + bf2f(wb[kOffB2 + n]));
#pragma unroll
                for (int c = 0; c < 3; ++c) y[c] += h2 * bf2f(wb[kOffW3 + n * 3 + c]);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float v = y[c];
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 4);
                v += __shfl_xor(v, 8);
                y[c] = v;
            }
            if (lr16 == 0) {
                const int r = rb * 16 + 4 * lg + j;
                sY[r * 4] = y[0]; sY[r * 4 + 1] = y[1]; sY[r * 4 + 2] = y[2];
            }
        }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) p[c] = sY[l * 4 + c] + bf2f(wb[kOffB3 + c]);
    __syncthreads();
}

}  // namespace ivr
