// Launchers of the gfx950 kernels (defined in ivr_kernels.hip, called by ivr_api.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "ivr_mlp.h"
#include "ivr_types.h"

namespace ivr {

hipError_t launch_fragments(bool fp64, bool mlp, const Model &m, const ViewRec *views, int n_views,
                            uint32_t n_tiles, const LaunchCfg &lc, void *segs, uint32_t seg_cap,
                            uint2 *seg_kr, uint32_t *pcount, QueueState *qs, uint2 *pixseg,
                            const CandLists &mq, unsigned long long *ctr, int n_cu, hipStream_t st);

hipError_t launch_block_sort(const QueueState *qs, uint32_t seg_cap, const uint2 *seg_kr,
                             const uint32_t *pperm, int nperm, const uint32_t *pcount, uint32_t *pbase,
                             uint32_t *pcur, uint32_t *order, int n_cu, hipStream_t st);

// field: IVR_FIELD_*; the derived fields (with the ODE or root-finding
// interior method only) run launch_integrate_field, in their own unit.
// diag: the instrumented integrator that records the pixel accuracy (views'
// dp buffers; scalar field, ODE or RF), also in that unit.
hipError_t launch_integrate(bool fp64, int method, int field, bool diag, int klass, const Model &m,
                            const ViewRec *views, int n_views, void *segs, const IntegrateArgs &a,
                            unsigned long long *ctr, int n_cu, const LaunchCfg &lc, hipStream_t st);
hipError_t launch_integrate_field(bool fp64, int method, int field, bool diag, int klass, const Model &m,
                                  const ViewRec *views, int n_views, void *segs, const IntegrateArgs &a,
                                  unsigned long long *ctr, int n_cu, const LaunchCfg &lc, hipStream_t st);
// CIEDE2000 of two premultiplied RGBA images over bg (per pixel into out if
// given; the summary accumulated into *sum, which the caller clears)
hipError_t launch_delta_e(const float *a, const float *b, uint64_t n, const double (&bg)[3], double threshold,
                          float *out, DeltaESum *sum, int n_cu, hipStream_t st);
// zeroes the views' dp buffers (before an instrumented integrator)
hipError_t launch_dp_clear(const ViewRec *views, int n_views, uint32_t n_pixels, hipStream_t st);

hipError_t launch_merge(const ViewRec *views, int n_views, uint32_t n_pixels, const uint2 *pixseg,
                        const void *segs, bool fp64, const QueueState *qs, uint32_t *totals, hipStream_t st);

hipError_t launch_clear(QueueState *qs, unsigned long long *ctr, bool collect, uint32_t *pcount, int npatch,
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

}  // namespace ivr
