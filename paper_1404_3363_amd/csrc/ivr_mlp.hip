// Learned initialiser kernels (gfx950): forward-map sampling, BF16 MFMA training
// (forward, backward, Adam with FP32 master weights) and inference.
//
// Training layout, one workgroup of 4 waves per block, 128 rows computed per
// step (a smaller minibatch leaves the rows past it without gradient):
//   layer 1 (3 -> 64) and layer 3 (64 -> 3) are thin and run on the VALU;
//   layer 2 (64 -> 64) forward Z2 = H1 W2, and backward dW2 = H1^T dZ2 and
//   dH1 = dZ2 W2^T run on v_mfma_f32_16x16x16_bf16 with FP32 accumulation.
// MFMA operand layout (16x16x16, wave64): lane l holds A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16] and D[4(l/16)+j][l%16], j = 0..3.
#include <hip/hip_runtime.h>

#include "ivr_internal.h"
#include "ivr_mlp.h"
#include "ivr_mlp_dev.h"
#include "ivr_spline.h"

namespace ivr {


// ------------------------------------------------------------------ samples

template <int P, bool RAT>
__device__ __forceinline__ void forward_map(const Model &m, const DevPatch &Pd, const float (&p)[3],
                                            float (&x)[3]) {
    const PatchView<float> pv = view_of<float>(Pd);
    const Arrays<float> ar = arrays_of(m, 0.0f);
    float J[3][3], rho, g[3];
    eval_volume<P, RAT, 0>(pv, ar, p, x, J, rho, g);
}

// (x_hat, p) pairs: p ~ U[0,1]^3 from the hash of (seed, block, sample), x = F(p)
// normalised by the block's box.  Grid: (ceil(n/256), npatch).
__global__ __launch_bounds__(256) void k_mlp_samples(Model m, MlpState st, int n, uint32_t seed,
                                                     float4 *xs, float4 *ps) {
    const int q = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const DevPatch &Pd = m.patches[q];
    float p[3], x[3];
    const uint32_t base = pcg_hash(seed ^ pcg_hash((uint32_t)q * 0x9E3779B9u));
#pragma unroll
    for (int c = 0; c < 3; ++c) p[c] = u01(pcg_hash(base ^ pcg_hash((uint32_t)i * 3u + (uint32_t)c)));
    switch (Pd.deg * 2 + Pd.rational) {
    case 2: forward_map<1, false>(m, Pd, p, x); break;
    case 3: forward_map<1, true>(m, Pd, p, x); break;
    case 4: forward_map<2, false>(m, Pd, p, x); break;
    case 5: forward_map<2, true>(m, Pd, p, x); break;
    case 6: forward_map<3, false>(m, Pd, p, x); break;
    default: forward_map<3, true>(m, Pd, p, x); break;
    }
    const float *nm = st.norm + 12 * q;
    const size_t o = (size_t)q * n + i;
    xs[o] = make_float4((x[0] - nm[6]) * nm[3], (x[1] - nm[7]) * nm[4], (x[2] - nm[8]) * nm[5], 0.f);
    ps[o] = make_float4(p[0], p[1], p[2], 0.f);
}

// ------------------------------------------------------------------ training

constexpr int LDP = 72;   // padded LDS row (bf16 elements), 144 bytes

__device__ __forceinline__ bf16x4 lds4(const uint16_t *base) {
    return *reinterpret_cast<const bf16x4 *>(base);
}
__device__ __forceinline__ float red16(float v) {   // sum over the 16 lanes of a group
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}
__device__ __forceinline__ float red_groups(float v) {   // sum over the 4 groups of 16
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// MODE 0: tp.steps Adam steps on minibatches drawn from (xs, ps).
// MODE 1: one forward/backward on the 128 rows (gc_x, gc_p) with the block's
//         current weights; writes the gradient (kMlpParams) and the loss to gc_out.
template <int MODE>
__global__ __launch_bounds__(256) void k_mlp_train(MlpState st, MlpTrainParams tp, const float4 *xs,
                                                   const float4 *ps, float *loss_log, int nlog,
                                                   const float *gc_x, const float *gc_p, float *gc_out) {
    __shared__ uint16_t sH1[kMlpBatch * LDP];
    __shared__ uint16_t sdZ2[kMlpBatch * LDP];
    __shared__ uint16_t sW2[kMlpH * LDP];    // [k_in][n_out]
    __shared__ uint16_t sW2T[kMlpH * LDP];   // [n_out][k_in]
    __shared__ float sX[kMlpBatch * 3], sP[kMlpBatch * 3];
    __shared__ float sW1[192], sb1[64], sb2[64], sW3[192], sb3[4];
    __shared__ float gW1[192], gb1[64], gb2[64], gW3[192], gb3[4];
    __shared__ float sLoss;

    const int q = blockIdx.x, tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int lr16 = l & 15, lg = l >> 4;
    float *W = st.w + (size_t)q * kMlpStride;
    float *Mo = st.m + (size_t)q * kMlpStride;
    float *Vo = st.v + (size_t)q * kMlpStride;

    for (int i = tid; i < 192; i += 256) { sW1[i] = W[kOffW1 + i]; sW3[i] = W[kOffW3 + i]; gW1[i] = 0.f; gW3[i] = 0.f; }
    for (int i = tid; i < 64; i += 256) { sb1[i] = W[kOffB1 + i]; sb2[i] = W[kOffB2 + i]; gb1[i] = 0.f; gb2[i] = 0.f; }
    if (tid < 4) { sb3[tid] = tid < 3 ? W[kOffB3 + tid] : 0.f; gb3[tid] = 0.f; }
    for (int i = tid; i < 64 * 64; i += 256) {
        const int k = i >> 6, n = i & 63;
        const uint16_t b = f2bf(W[kOffW2 + i]);
        sW2[k * LDP + n] = b;
        sW2T[n * LDP + k] = b;
    }
    __syncthreads();

    const int steps = MODE ? 1 : tp.steps;
    for (int step = 0; step < steps; ++step) {
        // minibatch
        if (tid < kMlpBatch) {
            float x[3], p[3];
            if (MODE) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    x[c] = tid < tp.batch ? gc_x[tid * 3 + c] : 0.f;
                    p[c] = tid < tp.batch ? gc_p[tid * 3 + c] : 0.f;
                }
            } else {
                const uint32_t h = pcg_hash(tp.seed ^ pcg_hash((uint32_t)(q * 7919 + step) * 131u + (uint32_t)tid));
                const size_t o = (size_t)q * tp.samples + (h % (uint32_t)tp.samples);
                const float4 xv = xs[o], pv = ps[o];
                x[0] = xv.x; x[1] = xv.y; x[2] = xv.z; p[0] = pv.x; p[1] = pv.y; p[2] = pv.z;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) { sX[tid * 3 + c] = x[c]; sP[tid * 3 + c] = p[c]; }
        }
        if (tid == 0) sLoss = 0.f;
        __syncthreads();
        // layer 1: H1 = tanh(X W1 + b1)
        for (int e = tid; e < kMlpBatch * 64; e += 256) {
            const int i = e >> 6, n = e & 63;
            const float z = sb1[n] + sX[i * 3] * sW1[n] + sX[i * 3 + 1] * sW1[64 + n] + sX[i * 3 + 2] * sW1[128 + n];
            sH1[i * LDP + n] = f2bf(tanh_fast(z));
        }
        __syncthreads();
        // layer 2 forward (MFMA): wave w owns rows 32w .. 32w+31
        f32x4 acc[2][4];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[rb][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            bf16x4 a[2], b[4];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) a[rb] = lds4(&sH1[(32 * w + rb * 16 + lr16) * LDP + ks * 16 + 4 * lg]);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) b[ct] = lds4(&sW2T[(ct * 16 + lr16) * LDP + ks * 16 + 4 * lg]);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    acc[rb][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[rb], b[ct], acc[rb][ct], 0, 0, 0);
        }
        float h2[2][4][4];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                for (int j = 0; j < 4; ++j) h2[rb][ct][j] = tanh_fast(acc[rb][ct][j] + sb2[ct * 16 + lr16]);
        // layer 3, loss, dY = 2 (Y - P) / B
        float dy[2][4][3], lossp = 0.f;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = 32 * w + rb * 16 + 4 * lg + j;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float s = 0.f;
#pragma unroll
                    for (int ct = 0; ct < 4; ++ct) s += h2[rb][ct][j] * sW3[(ct * 16 + lr16) * 3 + c];
                    // rows past the minibatch (batch < kMlpBatch) carry no gradient
                    const float e = i < tp.batch ? red16(s) + sb3[c] - sP[i * 3 + c] : 0.f;
                    dy[rb][j][c] = e * (2.0f / (float)tp.batch);
                    lossp += e * e;
                }
            }
        if (lr16 == 0) atomicAdd(&sLoss, lossp);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float g = 0.f;
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int j = 0; j < 4; ++j) g += h2[rb][ct][j] * dy[rb][j][c];
                g = red_groups(g);
                if (lg == 0) atomicAdd(&gW3[(ct * 16 + lr16) * 3 + c], g);
            }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float g = 0.f;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int j = 0; j < 4; ++j) g += dy[rb][j][c];
            g = red_groups(g);
            if (l == 0) atomicAdd(&gb3[c], g);
        }
        // dZ2 = (dY W3^T) * (1 - H2^2), stored as BF16 rows; db2
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int n = ct * 16 + lr16;
            float g = 0.f;
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float dh = dy[rb][j][0] * sW3[n * 3] + dy[rb][j][1] * sW3[n * 3 + 1] + dy[rb][j][2] * sW3[n * 3 + 2];
                    const float dz = dh * (1.0f - h2[rb][ct][j] * h2[rb][ct][j]);
                    sdZ2[(32 * w + rb * 16 + 4 * lg + j) * LDP + n] = f2bf(dz);
                    g += dz;
                }
            g = red_groups(g);
            if (lg == 0) atomicAdd(&gb2[n], g);
        }
        __syncthreads();
        // dW2 = H1^T dZ2 (MFMA, K = batch): wave w owns input rows 16w .. 16w+15
        f32x4 gw2[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) gw2[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kMlpBatch / 16; ++ks) {
            bf16x4 a, b[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) a[j] = (short)sH1[(ks * 16 + 4 * lg + j) * LDP + 16 * w + lr16];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                for (int j = 0; j < 4; ++j) b[ct][j] = (short)sdZ2[(ks * 16 + 4 * lg + j) * LDP + ct * 16 + lr16];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) gw2[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[ct], gw2[ct], 0, 0, 0);
        }
        // dH1 = dZ2 W2^T (MFMA), dZ1 = dH1 * (1 - H1^2); dW1, db1
        f32x4 acc3[2][4];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc3[rb][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            bf16x4 a[2], b[4];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) a[rb] = lds4(&sdZ2[(32 * w + rb * 16 + lr16) * LDP + ks * 16 + 4 * lg]);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) b[ct] = lds4(&sW2[(ct * 16 + lr16) * LDP + ks * 16 + 4 * lg]);
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    acc3[rb][ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[rb], b[ct], acc3[rb][ct], 0, 0, 0);
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int n = ct * 16 + lr16;
            float gb = 0.f, gw[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int i = 32 * w + rb * 16 + 4 * lg + j;
                    const float h1 = bf2f(sH1[i * LDP + n]);
                    const float dz1 = acc3[rb][ct][j] * (1.0f - h1 * h1);
                    gb += dz1;
#pragma unroll
                    for (int c = 0; c < 3; ++c) gw[c] += sX[i * 3 + c] * dz1;
                }
            gb = red_groups(gb);
#pragma unroll
            for (int c = 0; c < 3; ++c) gw[c] = red_groups(gw[c]);
            if (lg == 0) {
                atomicAdd(&gb1[n], gb);
#pragma unroll
                for (int c = 0; c < 3; ++c) atomicAdd(&gW1[c * 64 + n], gw[c]);
            }
        }
        __syncthreads();

        if (MODE) {
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    gc_out[kOffW2 + (16 * w + 4 * lg + j) * 64 + ct * 16 + lr16] = gw2[ct][j];
            for (int i = tid; i < 192; i += 256) { gc_out[kOffW1 + i] = gW1[i]; gc_out[kOffW3 + i] = gW3[i]; }
            for (int i = tid; i < 64; i += 256) { gc_out[kOffB1 + i] = gb1[i]; gc_out[kOffB2 + i] = gb2[i]; }
            if (tid < 3) gc_out[kOffB3 + tid] = gb3[tid];
            if (tid == 0) gc_out[kMlpParams] = sLoss / (float)tp.batch;
            return;
        }
        // Adam on the FP32 master weights
        const float t = float(step + 1);
        const float bc1 = 1.0f - __powf(tp.beta1, t), bc2 = 1.0f - __powf(tp.beta2, t);
        auto adam = [&](int idx, float g) {
            const float mm = tp.beta1 * Mo[idx] + (1.0f - tp.beta1) * g;
            const float vv = tp.beta2 * Vo[idx] + (1.0f - tp.beta2) * g * g;
            Mo[idx] = mm;
            Vo[idx] = vv;
            const float nw = W[idx] - tp.lr * (mm / bc1) / (sqrtf(vv / bc2) + tp.eps);
            W[idx] = nw;
            return nw;
        };
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = 16 * w + 4 * lg + j, n = ct * 16 + lr16;
                const uint16_t b = f2bf(adam(kOffW2 + k * 64 + n, gw2[ct][j]));
                sW2[k * LDP + n] = b;
                sW2T[n * LDP + k] = b;
            }
        for (int s = tid; s < kMlpSmall; s += 256) {
            if (s < 192) sW1[s] = adam(kOffW1 + s, gW1[s]);
            else if (s < 256) sb1[s - 192] = adam(kOffB1 + s - 192, gb1[s - 192]);
            else if (s < 320) sb2[s - 256] = adam(kOffB2 + s - 256, gb2[s - 256]);
            else if (s < 512) sW3[s - 320] = adam(kOffW3 + s - 320, gW3[s - 320]);
            else sb3[s - 512] = adam(kOffB3 + s - 512, gb3[s - 512]);
        }
        __syncthreads();
        if (tid == 0 && tp.log_every > 0 && step % tp.log_every == 0 && step / tp.log_every < nlog)
            loss_log[(size_t)q * nlog + step / tp.log_every] = sLoss / (float)tp.batch;
        for (int i = tid; i < 192; i += 256) { gW1[i] = 0.f; gW3[i] = 0.f; }
        for (int i = tid; i < 64; i += 256) { gb1[i] = 0.f; gb2[i] = 0.f; }
        if (tid < 4) gb3[tid] = 0.f;
        __syncthreads();
    }
    if (MODE == 0) {
        uint16_t *wb = st.wb + (size_t)q * kMlpWbStride;
        for (int i = tid; i < kMlpParams; i += 256) wb[i] = f2bf(W[i]);
        for (int i = tid; i < 64 * 64; i += 256) wb[kOffW2T + (i & 63) * 64 + (i >> 6)] = f2bf(W[kOffW2 + i]);
    }
}

// ------------------------------------------------------------------ inference

__global__ __launch_bounds__(256) void k_mlp_infer(MlpState st, const int *patch, const float *x, int n,
                                                   float *p) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float xv[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    float pv[3];
    mlp_infer(st.wb, st.norm, patch[i], xv, pv);
    p[3 * i] = pv[0]; p[3 * i + 1] = pv[1]; p[3 * i + 2] = pv[2];
}

// held-out error: max over coordinates |MLP(F(p)) - p| per sample, from the
// normalised inputs (grid like k_mlp_samples)
__global__ __launch_bounds__(256) void k_mlp_heldout(MlpState st, int n, const float4 *xs, const float4 *ps,
                                                     float *err) {
    const int q = blockIdx.y;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float *nm = st.norm + 12 * q;
    const size_t o = (size_t)q * n + i;
    const float4 xv = xs[o], pv = ps[o];
    // back to world coordinates for the common inference path
    const float x[3] = {xv.x / nm[3] + nm[6], xv.y / nm[4] + nm[7], xv.z / nm[5] + nm[8]};
    float p[3];
    mlp_infer(st.wb, st.norm, q, x, p);
    err[o] = fmaxf(fabsf(p[0] - pv.x), fmaxf(fabsf(p[1] - pv.y), fabsf(p[2] - pv.z)));
}

// ------------------------------------------------------------------ launchers

hipError_t launch_mlp_samples(const Model &m, const MlpState &st, int npatch, int n, uint32_t seed,
                              float4 *xs, float4 *ps, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_samples, dim3((n + 255) / 256, npatch), dim3(256), 0, s, m, st, n, seed, xs, ps);
    return hipGetLastError();
}

hipError_t launch_mlp_train(const MlpState &st, const MlpTrainParams &tp, const float4 *xs,
                            const float4 *ps, float *loss_log, int nlog, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_train<0>, dim3(tp.npatch), dim3(256), 0, s, st, tp, xs, ps, loss_log, nlog,
                       (const float *)nullptr, (const float *)nullptr, (float *)nullptr);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpState &st, const MlpTrainParams &tp, const float *x, const float *p,
                           float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_train<1>, dim3(1), dim3(256), 0, s, st, tp, (const float4 *)nullptr,
                       (const float4 *)nullptr, (float *)nullptr, 0, x, p, out);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const MlpState &st, const int *patch, const float *x, int n, float *p,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_infer, dim3((n + 255) / 256), dim3(256), 0, s, st, patch, x, n, p);
    return hipGetLastError();
}

hipError_t launch_mlp_heldout(const MlpState &st, int npatch, int n, const float4 *xs, const float4 *ps,
                              float *err, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_heldout, dim3((n + 255) / 256, npatch), dim3(256), 0, s, st, n, xs, ps, err);
    return hipGetLastError();
}

}  // namespace ivr
