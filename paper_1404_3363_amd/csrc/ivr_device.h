// Wave-level helpers and the pixel ray shared by the fragment kernel and the
// integrator.
#pragma once
#include <hip/hip_runtime.h>

#include "ivr_types.h"

namespace ivr {

using u32 = uint32_t;
using u64 = unsigned long long;

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ int rank_in(u64 mask) {
    return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
}

// sum over the wave, result in every lane
__device__ __forceinline__ u64 wave_sum(u64 v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ void flush_counter(u64 *ctr, int idx, u64 v) {
    const u64 s = wave_sum(v);
    if (lane_id() == 0 && s) atomicAdd(ctr + idx, s);
}

// Ray through the centre of pixel (px, py), computed in FP64.
__device__ __forceinline__ void ray_dir(const FrameParams &fp, int px, int py, double (&d)[3]) {
    const double sx = (2.0 * (px + 0.5) / fp.width - 1.0) * fp.tan_half * fp.aspect;
    const double sy = (1.0 - 2.0 * (py + 0.5) / fp.height) * fp.tan_half;
    double n2 = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        d[q] = fp.fwd[q] + sx * fp.right[q] + sy * fp.up[q];
        n2 += d[q] * d[q];
    }
    const double inv = 1.0 / sqrt(n2);
#pragma unroll
    for (int q = 0; q < 3; ++q) d[q] *= inv;
}

}  // namespace ivr
