// Launchers of the gfx950 kernels (defined in ivr_kernels.hip, called by ivr_api.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "ivr_mlp.h"
#include "ivr_types.h"

namespace ivr {

hipError_t launch_fragments(bool fp64, const Model &m, const FrameParams &fp, void *segs,
                            uint32_t seg_cap, uint32_t *queues, uint32_t queue_stride,
                            uint32_t class_mask, QueueState *qs, uint2 *pixseg, float *depth,
                            unsigned long long *ctr, hipStream_t st);

hipError_t launch_integrate(bool fp64, int klass, const Model &m, const FrameParams &fp,
                            const void *segs, const uint32_t *queue, const QueueState *qs,
                            uint32_t *qnext, float4 *results, unsigned long long *ctr, int n_cu,
                            hipStream_t st);

hipError_t launch_mlp_samples(const Model &m, const MlpState &st, int npatch, int n, uint32_t seed,
                              float4 *xs, float4 *ps, hipStream_t s);
hipError_t launch_mlp_train(const MlpState &st, const MlpTrainParams &tp, const float4 *xs,
                            const float4 *ps, float *loss_log, int nlog, hipStream_t s);
hipError_t launch_mlp_grad(const MlpState &st, const MlpTrainParams &tp, const float *x, const float *p,
                           float *out, hipStream_t s);
hipError_t launch_mlp_infer(const MlpState &st, const int *patch, const float *x, int n, float *p,
                            hipStream_t s);
hipError_t launch_mlp_heldout(const MlpState &st, int npatch, int n, const float4 *xs, const float4 *ps,
                              float *err, hipStream_t s);

hipError_t launch_merge(const FrameParams &fp, const uint2 *pixseg, const float4 *results,
                        float *rgba, hipStream_t st);

}  // namespace ivr
