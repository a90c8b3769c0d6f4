// Per-block learned initialiser: a 3 -> 64 -> 64 -> 3 tanh MLP approximating the
// inverse geometry map F^-1 on the block's image, trained on (F(p), p) pairs that
// the forward map generates.  Parameter layout (floats), per block:
//   W1[3][64] | b1[64] | W2[64][64] (row = input unit) | b2[64] | W3[64][3] | b3[3]
// Inputs are the world point normalised by the block's box to [-1, 1]^3.
#pragma once
#include <stdint.h>

namespace ivr {

constexpr int kMlpIn = 3, kMlpH = 64, kMlpOut = 3;
constexpr int kOffW1 = 0, kOffB1 = 192, kOffW2 = 256, kOffB2 = 4352, kOffW3 = 4416, kOffB3 = 4608;
constexpr int kMlpParams = 4611;
constexpr int kMlpStride = 4624;       // per-block stride of the FP32 arrays (16-float aligned)
constexpr int kOffW2T = 4624;          // BF16 inference copy: W2 transposed, [n_out][k_in]
constexpr int kMlpWbStride = 8720;     // per-block stride of the BF16 inference weights
constexpr int kMlpBatch = 128;         // minibatch per training step and block
constexpr int kMlpSmall = 515;         // parameters outside W2

struct MlpState {
    float *w;            // FP32 master weights      [npatch][kMlpStride]
    float *m, *v;        // Adam moments              [npatch][kMlpStride]
    uint16_t *wb;        // BF16 weights (inference)  [npatch][kMlpWbStride]
    float *norm;         // per block: lo[3], inv_half_extent[3], centre[3], pad
};

struct MlpTrainParams {
    int32_t steps, samples, log_every, npatch;
    int32_t batch;   // live rows of the kMlpBatch computed (the rest carry no gradient)
    float lr, beta1, beta2, eps;
    uint32_t seed;
};

}  // namespace ivr
