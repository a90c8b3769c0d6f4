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
// for inference: the hardware reciprocal (about 1 ulp) instead of a division
__device__ __forceinline__ float tanh_infer(float x) {
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * x) + 1.0f);
}

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

// The network's guess of the parameter point of world point x in block q, out
// of line: the integrator calls it only to seed a rare Newton restart.
__device__ __attribute__((noinline)) void mlp_seed_at(const uint16_t *wball, const float *normall, int q,
                                                      float x0, float x1, float x2, float *p) {
    const float x[3] = {x0, x1, x2};
    float r[3];
    mlp_infer(wball, normall, q, x, r);
    p[0] = r[0]; p[1] = r[1]; p[2] = r[2];
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// The MLP for the 64 rows of a wave, each row (lane) with its own block q (ok:
// the row is a query).  Layers 1 and 3 run per lane on the VALU with the row's
// own weights (16-byte loads); the 64x64 layer runs on v_mfma_f32_16x16x16_bf16
// once per distinct block among the rows, each row keeping its block's result.
// LDS owned by the wave: sA 64*72 BF16 (layer-1 activations), sZ 64*65 floats
// (layer-2 pre-activations), sQ 64 ints.  Every lane of the wave must execute it.
__device__ __forceinline__ void mlp_infer_rows(const uint16_t *wball, const float *normall, int q, bool ok,
                                               const float (&x)[3], float (&p)[3], uint16_t *sA, float *sZ,
                                               int *sQ) {
    const int l = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int lr16 = l & 15, lg = l >> 4;
    const int qq = ok ? q : 0;
    const uint16_t *wq = wball + (size_t)qq * kMlpWbStride;
    const float *nm = normall + 12 * qq;
    const float xh[3] = {(x[0] - nm[6]) * nm[3], (x[1] - nm[7]) * nm[4], (x[2] - nm[8]) * nm[5]};
    sQ[l] = ok ? q : -1;
    uint32_t *row = reinterpret_cast<uint32_t *>(sA + l * 72);
#pragma unroll 1
    for (int n0 = 0; n0 < kMlpH; n0 += 8) {
        const uint4 w0 = *reinterpret_cast<const uint4 *>(wq + kOffW1 + n0);
        const uint4 w1 = *reinterpret_cast<const uint4 *>(wq + kOffW1 + 64 + n0);
        const uint4 w2 = *reinterpret_cast<const uint4 *>(wq + kOffW1 + 128 + n0);
        const uint4 b1 = *reinterpret_cast<const uint4 *>(wq + kOffB1 + n0);
        const uint32_t a0[4] = {w0.x, w0.y, w0.z, w0.w}, a1[4] = {w1.x, w1.y, w1.z, w1.w};
        const uint32_t a2[4] = {w2.x, w2.y, w2.z, w2.w}, bb[4] = {b1.x, b1.y, b1.z, b1.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            float v[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int sh = 16 * s;
                v[s] = tanh_infer(bf2f((uint16_t)(bb[h] >> sh)) + xh[0] * bf2f((uint16_t)(a0[h] >> sh)) +
                                 xh[1] * bf2f((uint16_t)(a1[h] >> sh)) + xh[2] * bf2f((uint16_t)(a2[h] >> sh)));
            }
            row[(n0 >> 1) + h] = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
        }
    }
    __syncthreads();
    unsigned long long todo = __ballot(ok);
    while (todo) {
        const int b = __builtin_amdgcn_readfirstlane(__shfl(qq, __builtin_ctzll(todo)));
        const uint16_t *wb = wball + (size_t)b * kMlpWbStride;
        f32x4 acc[4][4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[rb][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            bf16x4 a[4], bm[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
                a[rb] = *reinterpret_cast<const bf16x4 *>(sA + (rb * 16 + lr16) * 72 + ks * 16 + 4 * lg);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
                bm[ct] = *reinterpret_cast<const bf16x4 *>(wb + kOffW2T + (ct * 16 + lr16) * 64 + ks * 16 + 4 * lg);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    acc[rb][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[rb], bm[ct], acc[rb][ct], 0, 0, 0);
        }
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = rb * 16 + 4 * lg + j;
                if (sQ[r] == b) {
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct) sZ[r * 65 + ct * 16 + lr16] = acc[rb][ct][j];
                }
            }
        todo &= ~__ballot(ok && q == b);
    }
    __syncthreads();
    float y[3] = {bf2f(wq[kOffB3]), bf2f(wq[kOffB3 + 1]), bf2f(wq[kOffB3 + 2])};
#pragma unroll 1
    for (int n0 = 0; n0 < kMlpH; n0 += 8) {
        const uint4 b2 = *reinterpret_cast<const uint4 *>(wq + kOffB2 + n0);
        const uint32_t bb[4] = {b2.x, b2.y, b2.z, b2.w};
        uint32_t w3[12];
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const uint4 t = *reinterpret_cast<const uint4 *>(wq + kOffW3 + 3 * n0 + 8 * v);
            w3[4 * v] = t.x; w3[4 * v + 1] = t.y; w3[4 * v + 2] = t.z; w3[4 * v + 3] = t.w;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float h2 = tanh_infer(sZ[l * 65 + n0 + i] + bf2f((uint16_t)(bb[i >> 1] >> (16 * (i & 1)))));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int e = 3 * i + c;   // element of the 24 BF16 of W3 rows n0..n0+7
                y[c] += h2 * bf2f((uint16_t)(w3[e >> 1] >> (16 * (e & 1))));
            }
        }
    }
    p[0] = y[0]; p[1] = y[1]; p[2] = y[2];
    __syncthreads();
}

}  // namespace ivr
