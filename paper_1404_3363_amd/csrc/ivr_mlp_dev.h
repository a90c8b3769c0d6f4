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
    const uint16_t *wb = wball + (size_t)q * kMlpStride;
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

}  // namespace ivr
