// The integrator kernel (Secs. "ODE Based Algorithm", "Root Finding Based
// Algorithm", "Quadrature of volume render integral") and its launch
// templates.  Included by the translation units that instantiate it: the
// stored-scalar variants with the other kernels, the derived-field variants
// in their own unit.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ivr.h"
#include "ivr_internal.h"
#include "ivr_device.h"
#include "ivr_mlp_dev.h"
#include "ivr_spline.h"

namespace ivr {

// Integrator-internal bits of a segment's flags (not reported): a drift restart
// happened since the last accepted RK step; the exit lies on the cutting plane
// (no parameter point: the last step's end is sampled); that end sample is due.
constexpr uint32_t kJustRestarted = 1u << 31;
constexpr uint32_t kExitOnPlane = 1u << 30;
constexpr uint32_t kEndSample = 1u << 29;
constexpr uint32_t kSecondSeed = 1u << 28;   // this Newton restarted from its second seed
constexpr uint32_t kPublicFlags = 0xFFFFu;

__device__ __forceinline__ float pow_fifth(float x) { return exp2f(0.2f * __log2f(x)); }
__device__ __forceinline__ double pow_fifth(double x) { return pow(x, 0.2); }

// Runge-Kutta-Fehlberg 4(5): stages, 5th-order weights (propagated) and the
// difference of the 5th- and 4th-order weights (error estimate).
template <typename R>
struct RKF {
    static constexpr R a21 = R(1) / R(4);
    static constexpr R a31 = R(3) / R(32), a32 = R(9) / R(32);
    static constexpr R a41 = R(1932) / R(2197), a42 = R(-7200) / R(2197), a43 = R(7296) / R(2197);
    static constexpr R a51 = R(439) / R(216), a52 = R(-8), a53 = R(3680) / R(513),
                       a54 = R(-845) / R(4104);
    static constexpr R a61 = R(-8) / R(27), a62 = R(2), a63 = R(-3544) / R(2565),
                       a64 = R(1859) / R(4104), a65 = R(-11) / R(40);
    static constexpr R b1 = R(16) / R(135), b3 = R(6656) / R(12825), b4 = R(28561) / R(56430),
                       b5 = R(-9) / R(50), b6 = R(2) / R(55);
    static constexpr R e1 = R(1) / R(360), e3 = R(-128) / R(4275), e4 = R(-2197) / R(75240),
                       e5 = R(1) / R(50), e6 = R(2) / R(55);
};

// The fixed-step explicit family (IVR_INTERIOR_RK1 .. RKF5, in that order):
// stages, the lower triangle of a, and b, by Butcher tableau.
struct RkTableau {
    int stages;
    double a[6][6];
    double b[6];
};
static __constant__ RkTableau kRkFamily[6] = {
    {1, {{0}}, {1}},                                                            // explicit Euler
    {2, {{0}, {0.5}}, {0, 1}},                                                  // midpoint
    {3, {{0}, {0.5}, {-1, 2}}, {1.0 / 6, 2.0 / 3, 1.0 / 6}},                    // Kutta, third order
    {4, {{0}, {0.5}, {0, 0.5}, {0, 0, 1}}, {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6}},  // classic fourth order
    {4, {{0}, {1.0 / 3}, {-1.0 / 3, 1}, {1, -1, 1}}, {1.0 / 8, 3.0 / 8, 3.0 / 8, 1.0 / 8}},  // 3/8 rule
    {6,
     {{0},
      {1.0 / 4},
      {3.0 / 32, 9.0 / 32},
      {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197},
      {439.0 / 216, -8, 3680.0 / 513, -845.0 / 4104},
      {-8.0 / 27, 2, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40}},
     {16.0 / 135, 0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55}}};  // Fehlberg, fifth order

// METHOD kOde: the ray preimage ODE by adaptive RKF45 (Sec. "ODE Based
// Algorithm"); kRootFinding: every sample's preimage by Newton (Sec. "Root
// Finding Based Algorithm"), seeded from the previous sample along J^-1 d.
// kFixedRK: a fixed-step explicit method of the family above; kImplicitEuler:
// implicit Euler with the exact Jacobian of its Newton (Eq. (JacG)).
constexpr int kOde = 0, kRootFinding = 1, kFixedRK = 2, kImplicitEuler = 3;

// FIELD: the value sampled along the ray.  0: the block's scalar spline rho;
// otherwise a field derived from the maps at each sample (IVR_FIELD_*), with
// its parameter gradient g (for d rho/ds = g . W, as for the scalar field):
// 1: the parametrisation quality q = det J / |J|_F (Eq. (paramQuality)),
//    d q = (d det |J|_F - det d|J|_F) / |J|_F^2 with d det = sum cof(J) : dJ,
//    d|J|_F = J : dJ / |J|_F and dJ/dp_a from the Hessian of phi;
// 2: von Mises of the displacement spline u (Eq. (vonMises), with the squares
//    and root the printed formula lacks) of e = (Y + Y^T)/2, Y = J_u J^-1 the
//    Jacobian of u o phi^-1 (the transpose of the paper's J_phi^T X = J_u^T,
//    which e symmetrises away); vm = sqrt(Q/2),
//    Q = (e11-e22)^2 + (e22-e33)^2 + (e33-e11)^2 + 6 (e12^2 + e23^2 + e31^2),
//    dY/dp_a = (dJ_u/dp_a - Y dJ/dp_a) J^-1, d vm = dQ / (4 vm).
// u is stored as (w u, w) per control point, so one rational evaluation serves
// B-spline (w = 1) and NURBS blocks.  J: J_phi at p (for J^-1 d at an exit).
// Packed Hessian slot of d^2 / dp_j dp_a.
__device__ __forceinline__ constexpr int hslot(int j, int a) {
    return j == a ? j : (j + a == 1 ? 3 : (j + a == 2 ? 4 : 5));
}

template <int P, bool RAT, int FIELD, typename R>
__device__ __forceinline__ R derived_field(const PatchView<R> &pv, const Arrays<R> &ar,
                                           const typename CpType<R>::T *disp, const R (&p)[3], R (&g)[3],
                                           R (&J)[3][3]) {
    R x[3], H[3][6];
    eval_volume_h<P, RAT, R, false>(pv, ar, p, x, J, H);
    // cofactors C[i][j] of J (adj(J) = C^T), det
    R C[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            C[i][j] = J[i1][j1] * J[i2][j2] - J[i1][j2] * J[i2][j1];
        }
    const R det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    if constexpr (FIELD == 1) {
        R fro2 = R(0);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) fro2 += J[i][j] * J[i][j];
        const R fro = sqrt(fro2);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            R ddet = R(0), dfro = R(0);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const R dJ = H[i][hslot(j, a)];
                    ddet += C[i][j] * dJ;
                    dfro += J[i][j] * dJ;
                }
            dfro /= fro;
            g[a] = (ddet * fro - det * dfro) / fro2;
        }
        return det / fro;
    } else {
        Arrays<R> ad = ar;
        ad.cp = disp;
        R u[3], Ju[3][3], Hu[3][6];
        eval_volume_h<P, true, R, false>(pv, ad, p, u, Ju, Hu);
        // J^-1 = C^T / det
        R Ji[3][3];
        const R idet = R(1) / det;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Ji[i][j] = C[j][i] * idet;
        R Y[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) Y[i][j] = Ju[i][0] * Ji[0][j] + Ju[i][1] * Ji[1][j] + Ju[i][2] * Ji[2][j];
        const R e00 = Y[0][0], e11 = Y[1][1], e22 = Y[2][2];
        const R e01 = R(0.5) * (Y[0][1] + Y[1][0]), e12 = R(0.5) * (Y[1][2] + Y[2][1]),
                e20 = R(0.5) * (Y[2][0] + Y[0][2]);
        const R d01 = e00 - e11, d12 = e11 - e22, d20 = e22 - e00;
        const R Q = d01 * d01 + d12 * d12 + d20 * d20 + R(6) * (e01 * e01 + e12 * e12 + e20 * e20);
        const R vm = sqrt(R(0.5) * Q);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // dY_a = (dJu_a - Y dJ_a) J^-1
            R T[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    T[i][k] = Hu[i][hslot(k, a)] - (Y[i][0] * H[0][hslot(k, a)] + Y[i][1] * H[1][hslot(k, a)] +
                                                    Y[i][2] * H[2][hslot(k, a)]);
            R dY[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) dY[i][j] = T[i][0] * Ji[0][j] + T[i][1] * Ji[1][j] + T[i][2] * Ji[2][j];
            const R f01 = R(0.5) * (dY[0][1] + dY[1][0]), f12 = R(0.5) * (dY[1][2] + dY[2][1]),
                    f20 = R(0.5) * (dY[2][0] + dY[0][2]);
            const R dQ = R(2) * (d01 * (dY[0][0] - dY[1][1]) + d12 * (dY[1][1] - dY[2][2]) +
                                 d20 * (dY[2][2] - dY[0][0])) +
                         R(12) * (e01 * f01 + e12 * f12 + e20 * f20);
            g[a] = vm > R(0) ? dQ / (R(4) * vm) : R(0);
        }
        return vm;
    }
}

// Distance of point g to the boundary of the frustum of pixel (row*width + col)
// of view fv: the smallest distance to its four side planes through the eye
// (Sec. "Root Finding Based Algorithm": the pixel-accurate Newton stop).
template <typename R>
__device__ __forceinline__ R frustum_distance(const FrameParams &fv, uint32_t pixel, const R (&g)[3]) {
    const int px = (int)(pixel % (uint32_t)fv.width), py = (int)(pixel / (uint32_t)fv.width);
    const R th = R(fv.tan_half), as = R(fv.aspect);
    R v[3], fw[3], rt[3], up[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v[c] = g[c] - R(fv.eye[c]);
        fw[c] = R(fv.fwd[c]);
        rt[c] = R(fv.right[c]);
        up[c] = R(fv.up[c]);
    }
    R dmin = R(INFINITY);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        // e = 0, 1: the planes x = const (they contain up); 2, 3: y = const
        R a[3], n[3];
        if (e < 2) {
            const R xe = (R(2) * R(px + e) / R(fv.width) - R(1)) * th * as;
#pragma unroll
            for (int c = 0; c < 3; ++c) a[c] = fw[c] + xe * rt[c];
            cross3(a, up, n);
        } else {
            const R ye = (R(1) - R(2) * R(py + e - 2) / R(fv.height)) * th;
#pragma unroll
            for (int c = 0; c < 3; ++c) a[c] = fw[c] + ye * up[c];
            cross3(rt, a, n);
        }
        dmin = fmin(dmin, fabs(dot3(v, n)) / sqrt(dot3(n, n)));
    }
    return dmin;
}

// Three waves per SIMD: the FP32 kernels fit in 168 VGPRs without spilling.
//
// Each workgroup works on one block at a time: with LDS, the block's control
// points (and w*rho for NURBS) are staged in LDS, so every evaluation reads its
// (p+1)^3 points from there instead of gathering them through the vector L1.
// The workgroup starts at the block holding its share of the class's segments,
// its waves refill their lanes from that block's cursor (one atomic per wave),
// and when the block has no segments left it drains and moves on to the next
// block with work, cyclically in class order.
// DIAG: the pixel-accuracy record of the views with a dp buffer.
template <int P, bool RAT, typename R, bool LDS, int METHOD, int FIELD = 0, bool DIAG = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_integrate(
    Model m, const ViewRec *views, int n_views, Seg<R> *segs, const u32 *order, const u32 *pperm,
    int q_begin, int q_end, const u32 *pbase, const u32 *pcount, u32 *pcur, int max_cp, u64 *ctr) {
    using K = RKF<R>;
    // LDS: per-view transfer functions and step bounds (a lane's segment may
    // belong to any view of the batch), then the staged block
    extern __shared__ __align__(16) unsigned char smem_raw[];
    ViewLds *vls = reinterpret_cast<ViewLds *>(smem_raw);
    float4 *lds_cp = reinterpret_cast<float4 *>(smem_raw + sizeof(ViewLds) * n_views);
    float *lds_rho = reinterpret_cast<float *>(lds_cp + max_cp);
    float *lds_tab = lds_rho + (RAT ? (max_cp + 3) / 4 * 4 : 0);   // 16-byte aligned
    __shared__ int s_q;
    view_stage(views, n_views, vls);
    const FrameParams fp = views[0].fp;   // the batch's options (uniform)
    const R tol = sizeof(R) == 4 ? R(fp.rk_tol) : R(fp.rk_told);
    const R cperp = sizeof(R) == 4 ? R(fp.c_perp) : R(fp.c_perpd);
    const R early = sizeof(R) == 4 ? R(fp.early_term) : R(fp.early_termd);
    const R dthr = sizeof(R) == 4 ? R(fp.det_thr) : R(fp.det_thrd);     // FP64 solves below it
    const R dsing = sizeof(R) == 4 ? R(fp.det_sing) : R(fp.det_singd);  // singular J below it
    const int nq = q_end - q_begin;
    if (threadIdx.x == 0) {
        // the block that holds segment S0 + (S1 - S0) * blockIdx / gridDim
        const u32 S0 = pbase[pperm[q_begin]];
        const u32 S1 = pbase[pperm[q_end - 1]] + pcount[pperm[q_end - 1]];
        int q = -1;
        if (S1 > S0) {
            const u32 target = S0 + (u32)(((unsigned long long)(S1 - S0) * blockIdx.x) / gridDim.x);
            int lo = q_begin, hi = q_end;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pbase[pperm[mid]] <= target) lo = mid;
                else hi = mid;
            }
            q = lo;
        }
        s_q = q;
    }
    __syncthreads();
    int q = s_q;

    bool active = false;
    u32 sid = 0;
    int vid = 0;                  // view of the lane's segment
    R hmax = 0, hmin = 0, vscale = 0;
    R p[3] = {0, 0, 0}, gin[3] = {0, 0, 0}, d[3] = {0, 0, 0};
    R s = 0, L = 0, Lend = 0, h = 0, h_prev = 0, rho_prev = 0, m_prev = 0, rho_out = 0, m_out = 0;
    R C[3] = {0, 0, 0}, A = 0;
    bool pending = false, fresh = false, rejected = false;
    int iters = 0;
    // Eq. (degeneracyfix) state: shrink > 0 (the attempt) while Newton seeks the
    // preimage of the entry moved delta along the ray; gin is then that point (it
    // stays on the ray, so V keeps its meaning)
    // shrink < 0: a drift restart, Newton on phi(p) = gin.  gin is the ray point at
    // the current arc length s (V_perp only takes its distance from the ray, so
    // any ray point serves; it moves with every accepted step).  fl: IVR_FLAG_*
    // bits of the lane's segment.
    int shrink = 0, newton_it = 0;
    R delta = 0, rho_in = 0;
    u32 fl = 0;
    // root finding with the frustum stop: the current sample's tolerance
    R rf_tol = R(0);
    // pixel-accuracy record (DIAG): the segment's largest Delta P, the ray
    // parameter of its last sample (the entry's first) and of its exit, pixel
    float dg_dp = 0.f;
    R dg_t = R(0), dg_tout = R(0);
    u32 dg_pix = 0, c_dpo = 0, c_ord = 0;
    // frequent events are counted per lane and summed per wave at the end; rare
    // ones (iteration cap, singular ends, restarts) with one atomic each
    u32 c_steps = 0, c_rej = 0, c_samp = 0, c_w = 0, c_fp64 = 0, c_sub = 0;
    auto count_rare = [&](int idx) __attribute__((always_inline)) {
        if (fp.collect) atomicAdd(ctr + idx, 1ull);
    };
    // drift threshold relative to the scale (0: no check); per lane it is at least
    // twice the restart Newton's own tolerance, so that a converged restart never
    // triggers another
    const R drel_set = sizeof(R) == 4 ? R(fp.drift_tol) : R(fp.drift_told);
    const R drel = drel_set > R(0) ? fmax(drel_set, sizeof(R) == 4 ? R(4e-6) : R(2e-12)) : R(0);

    for (;;) {   // blocks
        if (threadIdx.x == 0) {
            // from q on, cyclically in class order, the first block with segments left
            int found = -1;
            if (q >= 0)
                for (int t = 0; t < nq; ++t) {
                    const int qq = q_begin + (q - q_begin + t) % nq;
                    const u32 pp = pperm[qq];
                    if (__hip_atomic_load(&pcur[pp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
                        pbase[pp] + pcount[pp]) {
                        found = qq;
                        break;
                    }
                }
            s_q = found;
        }
        __syncthreads();
        q = s_q;
        if (q < 0) break;
        const u32 blk = pperm[q];
        const u32 pend = pbase[blk] + pcount[blk];
        PatchView<R> pv = view_of<R>(m.patches[blk]);
        Arrays<R> ar = arrays_of(m, R(0));
        const typename CpType<R>::T *disp_arr = nullptr;
        if constexpr (FIELD != 0) {
            if constexpr (sizeof(R) == 4) disp_arr = m.disp32;
            else disp_arr = m.disp64;
        }
        if constexpr (LDS) {
            const int ncp = pv.n[0] * pv.n[1] * pv.n[2];
            for (int i = threadIdx.x; i < ncp; i += blockDim.x) {
                lds_cp[i] = m.cp32[pv.cp_off + i];
                if (RAT) lds_rho[i] = m.rho32[pv.cp_off + i];
            }
            const DevPatch &Pb = m.patches[blk];
            for (int i = threadIdx.x; i < Pb.btab_len; i += blockDim.x) lds_tab[i] = m.btab[Pb.btab_off + i];
            pv.cp_off = 0;
            ar.cp = reinterpret_cast<const typename CpType<R>::T *>(lds_cp);
            ar.rho = reinterpret_cast<const R *>(lds_rho);
            ar.tab = lds_tab;
        }
        __syncthreads();
        bool queue_empty = false;
        for (;;) {   // segments of the block
        // refill idle lanes from the block's cursor (one atomic per wave)
        const u64 need = __ballot(!active);
        if (need && !queue_empty) {
            const int leader = __ffsll((long long)need) - 1;
            u32 b = 0;
            if (lane_id() == leader) b = atomicAdd(&pcur[blk], (u32)__popcll(need));
            b = __shfl(b, leader);
            if (b + (u32)__popcll(need) >= pend) queue_empty = true;
            if (!active) {
                const u32 qi = b + (u32)rank_in(need);
                if (qi < pend) {
                    sid = order[qi];
                    const Seg<R> sg = segs[sid];
                    vid = (int)(sg.patch >> kViewShift);
                    const FrameParams &fv = views[vid].fp;
                    const int pxl = (int)(sg.pixel % (u32)fv.width), pyl = (int)(sg.pixel / (u32)fv.width);
                    double dd[3];
                    ray_dir(fv, pxl, pyl, dd);
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        d[q] = R(dd[q]);
                        gin[q] = R(fv.eye[q] + double(sg.t_in) * dd[q]);
                        p[q] = sg.p_in[q];
                    }
                    hmax = sizeof(R) == 4 ? R(vls[vid].h_max) : R(fv.h_maxd);
                    hmin = sizeof(R) == 4 ? R(vls[vid].h_min) : R(fv.h_mind);
                    vscale = sizeof(R) == 4 ? R(vls[vid].scale) : R(fv.scaled);
                    L = sg.t_out - sg.t_in;
                    if constexpr (DIAG) {
                        dg_dp = 0.f;
                        dg_t = R(sg.t_in);
                        dg_tout = R(sg.t_out);
                        dg_pix = sg.pixel;
                    }
                    s = R(0);
                    h = L < hmax ? L : hmax;
                    rho_out = sg.rho_out;
                    m_out = sg.drho_out;
                    if constexpr (FIELD != 0) {
                        // the derived field at the exit and d rho/ds = g . J^-1 d
                        // there (a singular exit keeps its marker)
                        if (isfinite(sg.p_out[0])) {
                            const R po[3] = {sg.p_out[0], sg.p_out[1], sg.p_out[2]};
                            R go[3], Jo[3][3], Wo[3];
                            rho_out = derived_field<P, RAT, FIELD, R>(pv, ar, disp_arr, po, go, Jo);
                            const R c0[3] = {Jo[0][0], Jo[1][0], Jo[2][0]}, c1[3] = {Jo[0][1], Jo[1][1], Jo[2][1]},
                                    c2[3] = {Jo[0][2], Jo[1][2], Jo[2][2]};
                            solve_cols(c0, c1, c2, d, Wo);
                            if (isfinite(m_out)) m_out = dot3(go, Wo);
                        }
                    }
                    // singular J at the exit (flagged by a NaN slope): stop 1e-4 of
                    // the chord short of it and close with the exit's rho
                    Lend = isfinite(m_out) ? L : L - R(1e-4) * L;
                    if (!isfinite(m_out)) count_rare(C_DEGENERATE);
                    // next to a singular face p' and rho vary like sqrt of the
                    // distance: half the step bound on such a segment
                    if (!isfinite(m_out)) hmax *= R(0.5);
                    C[0] = C[1] = C[2] = A = R(0);
                    pending = false;
                    fresh = true;
                    rejected = false;
                    iters = 0;
                    shrink = 0;
                    fl = isfinite(m_out) ? 0u : (u32)IVR_FLAG_DEGENERATE;
                    if (!isfinite(sg.p_out[0])) fl |= kExitOnPlane;
                    // an entry on a clip plane has no parameter point: Newton finds
                    // it (Sec. "Cutting and Near Clip Planes", Eq. (F)) from the block
                    // centre, or from the block's network with MLP seeds, before the
                    // ODE starts
                    if (!isfinite(sg.p_in[0])) {
                        p[0] = p[1] = p[2] = R(0.5);
                        shrink = -2;
                        newton_it = 0;
                        if (fv.seed_mode == IVR_SEED_MLP) {
                            float pm[3];
                            mlp_seed_at(m.mlp_wb, m.mlp_norm, blk, float(gin[0]), float(gin[1]), float(gin[2]), pm);
                            if (isfinite(pm[0] + pm[1] + pm[2])) {
#pragma unroll
                                for (int c = 0; c < 3; ++c) p[c] = clamp01(R(pm[c]));
                                count_rare(C_MLP_RESTARTS);
                            }
                        }
                    }
                    active = true;
                }
            }
        }
        if (__ballot(active) == 0) break;
        if (!active) continue;

        bool done = false;
        // stage 1 at the current point; also samples rho and d rho/ds there.  While
        // shrinking, the same evaluation gives the Newton step J^-1 (gin - phi(p)).
        R k1[3], k2[3], k3[3], k4[3], k5[3], k6[3], rho_cur = R(0), grho[3], res2 = R(0), xw[3], wt[3];
        const bool shrinking = shrink != 0;
        const R det1 = eval_W<P, RAT, FIELD == 0 ? 2 : 0, R, LDS, METHOD == kRootFinding>(
            pv, ar, p, gin, d, cperp, dthr, k1, rho_cur, grho, c_fp64, shrinking, res2, xw, wt);
        ++c_w;
        // a derived field and its parameter gradient at p
        if constexpr (FIELD != 0) {
            R Jd[3][3];
            rho_cur = derived_field<P, RAT, FIELD, R>(pv, ar, disp_arr, p, grho, Jd);
        }
        const R m_cur = dot3(grho, k1);
        // Eq. (deltaP) and the depth order for a sample at phi(p) = xg (DIAG)
        auto diag_sample = [&](const R (&xg)[3]) __attribute__((always_inline)) {
            if constexpr (DIAG) {
                const FrameParams &fv = views[vid].fp;
                R v[3], z = R(0), sx = R(0), sy = R(0), t = R(0);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    v[c] = xg[c] - R(fv.eye[c]);
                    z += v[c] * R(fv.fwd[c]);
                    sx += v[c] * R(fv.right[c]);
                    sy += v[c] * R(fv.up[c]);
                    t += v[c] * d[c];
                }
                const R th = R(fv.tan_half), as = R(fv.aspect);
                const R X = (sx / (z * th * as) + R(1)) * R(0.5) * R(fv.width);
                const R Y = (R(1) - sy / (z * th)) * R(0.5) * R(fv.height);
                const R cx = R(dg_pix % (u32)fv.width) + R(0.5), cy = R(dg_pix / (u32)fv.width) + R(0.5);
                const R dp = R(2) * fmax(fabs(X - cx), fabs(Y - cy));
                dg_dp = fmaxf(dg_dp, float(dp));
                c_dpo += dp > R(1) ? 1u : 0u;
                if (t < dg_t) {
                    fl |= IVR_FLAG_DEPTH_ORDER;
                    ++c_ord;
                }
                dg_t = t;
            }
        };
        // Root finding: the next sample.  Its step follows the same bounds as the
        // ODE's (h_max, rho's change); its preimage is predicted along W = J^-1 d
        // and found by Newton (shrink -3); the last interval closes with the exit.
        auto rf_advance = [&](const R (&Wd)[3], R m_here) __attribute__((always_inline)) {
            const R dn_ds = fabs(m_here) * R(sizeof(R) == 4 ? double(vls[vid].inv_ranged)
                                                             : views[vid].fp.tf_inv_ranged);
            const R hf = R(fp.rho_step) / (dn_ds + R(1e-30));
            R hh = hmax < hf ? hmax : (hf > hmin ? hf : hmin);
            hh = hh < Lend - s ? hh : Lend - s;
            ++c_steps;
            if (Lend - s - hh <= R(1e-6) * L && !(fl & kExitOnPlane)) {
                const R hl = hh + (L - Lend);
                const R mo = isfinite(m_out) ? m_out : (rho_out - rho_prev) / hl;
                composite(fp, views[vid].fp, vls[vid], rho_prev, m_prev, rho_out, mo, hl, C, A, c_sub);
                ++c_samp;
                done = true;
                return;
            }
            if (Lend - s - hh <= R(1e-6) * L) fl |= kEndSample;   // the exit lies on the cutting plane
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                p[c] = clamp01(p[c] + hh * Wd[c]);
                gin[c] += hh * d[c];
            }
            s += hh;
            h_prev = hh;
            shrink = -3;
            newton_it = 0;
            if (fp.newton_stop == IVR_NEWTON_STOP_FRUSTUM) rf_tol = frustum_distance(views[vid].fp, segs[sid].pixel, gin);
            if (++iters >= 20000) {
                count_rare(C_RK_ITER_CAP);
                fl |= IVR_FLAG_ITER_CAP;
                done = true;
            }
        };
        if (shrinking && shrink < 0) {
            // drift restart (-1) or entry on a clip plane (-2): Newton on
            // phi(p) = gin (Eqs. (F), (newtonsmethod)), iterates clamped to P; once
            // converged the point is sampled (again)
            const R tolx = (sizeof(R) == 4 ? R(2e-6) : R(1e-12)) * vscale;
            if (METHOD == kRootFinding && shrink == -3) {
                // the frustum stop: within the distance of the sample to the
                // boundary of its pixel's frustum (never below tolx)
                const R tol_s = fp.newton_stop == IVR_NEWTON_STOP_FRUSTUM ? fmax(tolx, rf_tol) : tolx;
                if (res2 <= tol_s * tol_s || newton_it >= 12 || !isfinite(k1[0] + k1[1] + k1[2])) {
                    // the sample: rho and d rho/ds = grad rho . J^-1 d at the preimage
                    // (where Newton stopped if it did not converge: counted, flagged)
                    if (!(res2 <= tol_s * tol_s)) {
                        fl |= IVR_FLAG_RESTART_FAIL;
                        count_rare(C_RESTART_FAIL);
                    }
                    shrink = 0;
                    const R m_t = dot3(grho, wt);
                    composite(fp, views[vid].fp, vls[vid], rho_prev, m_prev, rho_cur, m_t, h_prev, C, A, c_sub);
                    ++c_samp;
                    diag_sample(xw);
                    rho_prev = rho_cur;
                    m_prev = m_t;
                    if (A >= R(1) - early || (fl & kEndSample)) done = true;
                    else rf_advance(wt, m_t);
                } else {
                    ++newton_it;
#pragma unroll
                    for (int c = 0; c < 3; ++c) p[c] = clamp01(p[c] + k1[c]);
                }
            } else if (res2 <= tolx * tolx) {
                shrink = 0;
            } else if (++newton_it < (shrink == -2 ? 24 : 12) && isfinite(k1[0] + k1[1] + k1[2])) {
#pragma unroll
                for (int c = 0; c < 3; ++c) p[c] = clamp01(p[c] + k1[c]);
            } else if (fp.seed_mode == IVR_SEED_MLP && !(fl & kSecondSeed)) {
                // with MLP seeds a second seed: the block's network for a drift
                // restart (which started from the drifted point), the block centre for
                // an entry on a plane (which started from the network)
                fl |= kSecondSeed;
                newton_it = 0;
                if (shrink == -1) {
                    float pm[3];
                    mlp_seed_at(m.mlp_wb, m.mlp_norm, blk, float(gin[0]), float(gin[1]), float(gin[2]), pm);
#pragma unroll
                    for (int c = 0; c < 3; ++c) p[c] = isfinite(pm[0] + pm[1] + pm[2]) ? clamp01(R(pm[c])) : R(0.5);
                    count_rare(C_MLP_RESTARTS);
                } else {
                    p[0] = p[1] = p[2] = R(0.5);
                }
            } else {
                // a drift restart goes on from where Newton stopped (no further
                // restarts); an entry that Newton cannot find leaves the segment empty
                done = shrink == -2;
                shrink = 0;
                fl |= IVR_FLAG_RESTART_FAIL;
                count_rare(C_RESTART_FAIL);
            }
        } else if (shrinking) {
            // Eq. (degeneracyfix): Newton on phi(p) = gin, iterates clamped to P
            const R tolx = (sizeof(R) == 4 ? R(2e-6) : R(1e-12)) * vscale;
            if (res2 <= tolx * tolx && fabs(det1) >= dsing) {
                // the sliver [0, delta]: rho linear from the entry to the new entry
                const R sl = (rho_cur - rho_in) / delta;
                composite(fp, views[vid].fp, vls[vid], rho_in, sl, rho_cur, sl, delta, C, A, c_sub);
                ++c_samp;
                s = delta;             // gin is the ray point at arc length delta
                shrink = 0;
                fresh = true;          // restart the ODE from the new entry
            } else if (++newton_it < 16 && isfinite(k1[0] + k1[1] + k1[2])) {
#pragma unroll
                for (int c = 0; c < 3; ++c) p[c] = clamp01(p[c] + k1[c]);
            } else if (shrink < 3) {
                // grow delta tenfold and seed again
                const Seg<R> &sg = segs[sid];
                ++shrink;
                delta *= R(10);
                R dp[3], nrm;
#pragma unroll
                for (int c = 0; c < 3; ++c) dp[c] = sg.p_out[c] - sg.p_in[c];
                nrm = sqrt(dot3(dp, dp));
                const R eps = sqrt(delta / L);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    gin[c] += R(0.9) * delta * d[c];   // from the previous delta to this one
                    p[c] = clamp01(sg.p_in[c] + eps * (nrm > R(0) ? dp[c] : R(0.5) - sg.p_in[c]));
                }
                newton_it = 0;
            } else {
                // no regular point near the entry: rho linear over the whole chord
                const R sl = (rho_out - rho_in) / L;
                composite(fp, views[vid].fp, vls[vid], rho_in, sl, rho_out, sl, L, C, A, c_sub);
                ++c_samp;
                done = true;
            }
        } else if (fresh) {
            fresh = false;
            if (!(L > R(1e-7) * vscale)) {
                done = true;   // empty chord
            } else if (s == R(0) && !(fabs(det1) >= dsing)) {
                // Eq. (degeneracyfix): J_phi singular at the entry.  Move the entry
                // delta = 1e-4 L along the ray (tenfold more, up to twice, if Newton
                // fails) and find its preimage by Newton from
                // x0 = p_in + eps (p_out - p_in)/|p_out - p_in|, eps = sqrt(delta/L)
                // |p_out - p_in| (the offset of a map whose normal derivative vanishes
                // to first order at the face)
                count_rare(C_DEGENERATE);
                fl |= IVR_FLAG_DEGENERATE;
                rho_in = rho_cur;
                hmax *= R(0.5);
                const Seg<R> &sg = segs[sid];
                shrink = 1;
                newton_it = 0;
                delta = R(1e-4) * L;
                R dp[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) dp[c] = sg.p_out[c] - sg.p_in[c];
                const R nrm = sqrt(dot3(dp, dp));
                const R eps = sqrt(delta / L);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    gin[c] += delta * d[c];
                    p[c] = clamp01(sg.p_in[c] + eps * (nrm > R(0) ? dp[c] : R(0.5) - sg.p_in[c]));
                }
                // with MLP seeds the first Newton of the restart starts from the
                // block's network at the new entry (the offset above if that fails)
                if (fp.seed_mode == IVR_SEED_MLP) {
                    float pm[3];
                    mlp_seed_at(m.mlp_wb, m.mlp_norm, blk, float(gin[0]), float(gin[1]), float(gin[2]), pm);
                    if (isfinite(pm[0] + pm[1] + pm[2])) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) p[c] = clamp01(R(pm[c]));
                        count_rare(C_MLP_RESTARTS);
                    }
                }
            }
            rho_prev = rho_cur;
            m_prev = m_cur;
        } else if (pending) {
            // The RK steps keep phi(p) on the ray only up to their error (and, with
            // c = 0, nothing pulls it back): when phi(p) lies more than drift_tol
            // from the ray point at arc length s, that point is found again by
            // Newton (seeded by the block's network with MLP seeds) before it is
            // sampled.
            R e2 = R(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) e2 += (xw[c] - gin[c]) * (xw[c] - gin[c]);
            // at most one restart between two RK steps (kJustRestarted)
            const R dtol = drel * vscale;
            if (e2 > dtol * dtol && drel > R(0) && !(fl & (IVR_FLAG_RESTART_FAIL | kJustRestarted))) {
                // Newton from the drifted point, which lies close to the preimage
                shrink = -1;
                fl = (fl | kJustRestarted | IVR_FLAG_DRIFT_RESTART) & ~kSecondSeed;
                newton_it = 0;
                count_rare(C_DRIFT_RESTARTS);
            } else {
                composite(fp, views[vid].fp, vls[vid], rho_prev, m_prev, rho_cur, m_cur, h_prev, C, A, c_sub);
                ++c_samp;
                diag_sample(xw);
                rho_prev = rho_cur;
                m_prev = m_cur;
                pending = false;
                if (A >= R(1) - early || (fl & kEndSample)) done = true;
            }
        }
        if (METHOD == kRootFinding && !done && !shrinking && !shrink) {
            rf_advance(k1, m_cur);   // from the entry (or a shrunk entry): W = J^-1 d there
        } else if (METHOD != kRootFinding && !done && !shrinking && !shrink) {
            // rho's change per step is bounded (its interpolation between samples);
            // the transfer function's frequencies are the supersampling's.  The
            // fixed-step methods start every step from h_max.
            const R dn_ds = fabs(m_cur) * R(sizeof(R) == 4 ? double(vls[vid].inv_ranged)
                                                            : views[vid].fp.tf_inv_ranged);
            const R hf = R(fp.rho_step) / (dn_ds + R(1e-30));
            if constexpr (METHOD != kOde) h = hmax;
            h = h < hf ? h : (hf > hmin ? hf : hmin);
            const R hh = (h < Lend - s) ? h : (Lend - s);
            // fixed steps: a step that ends on the exit fragment takes no stages;
            // the exit's rho closes the segment (as for root finding)
            bool closed = false;
            if constexpr (METHOD != kOde) {
                if (Lend - s - hh <= R(1e-6) * L && !(fl & kExitOnPlane)) {
                    const R hl = hh + (L - Lend);
                    const R mo = isfinite(m_out) ? m_out : (rho_out - rho_prev) / hl;
                    composite(fp, views[vid].fp, vls[vid], rho_prev, m_prev, rho_out, mo, hl, C, A, c_sub);
                    ++c_samp;
                    ++c_steps;
                    done = true;
                    closed = true;
                }
            }
            if (!closed) {
            R err = R(0), p5[3];
            if constexpr (METHOD == kOde) {
            R q[3], dummy, dg[3], dr2, dx[3];
#define IVR_STAGE(KOUT, EXPR)                                                              \
    _Pragma("unroll") for (int c = 0; c < 3; ++c) q[c] = clamp01(p[c] + hh * (EXPR));      \
    eval_W<P, RAT, 0, R, LDS>(pv, ar, q, gin, d, cperp, dthr, KOUT, dummy, dg, c_fp64, false, dr2, dx, dx); \
    ++c_w;
            IVR_STAGE(k2, K::a21 * k1[c])
            IVR_STAGE(k3, K::a31 * k1[c] + K::a32 * k2[c])
            IVR_STAGE(k4, K::a41 * k1[c] + K::a42 * k2[c] + K::a43 * k3[c])
            IVR_STAGE(k5, K::a51 * k1[c] + K::a52 * k2[c] + K::a53 * k3[c] + K::a54 * k4[c])
            IVR_STAGE(k6, K::a61 * k1[c] + K::a62 * k2[c] + K::a63 * k3[c] + K::a64 * k4[c] +
                              K::a65 * k5[c])
#undef IVR_STAGE
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                p5[c] = p[c] + hh * (K::b1 * k1[c] + K::b3 * k3[c] + K::b4 * k4[c] + K::b5 * k5[c] +
                                     K::b6 * k6[c]);
                const R e = fabs(hh * (K::e1 * k1[c] + K::e3 * k3[c] + K::e4 * k4[c] +
                                       K::e5 * k5[c] + K::e6 * k6[c]));
                err = (e > err || e != e) ? e : err;   // a non-finite stage rejects the step
            }
            } else if constexpr (METHOD == kFixedRK) {
                // the batch's tableau (uniform): stage i at p + hh sum_j a_ij k_j,
                // clamped to P; the step's end p + hh sum_i b_i k_i
                const RkTableau &tb = kRkFamily[fp.interior - IVR_INTERIOR_RK1];
                const int S = tb.stages;
                R kk[6][3];
#pragma unroll
                for (int c = 0; c < 3; ++c) kk[0][c] = k1[c];
#pragma unroll
                for (int i = 1; i < 6; ++i) {
                    if (i < S) {
                        R q[3], dummy, dg[3], dr2, dx[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            R acc = R(0);
#pragma unroll
                            for (int j = 0; j < i; ++j) acc += R(tb.a[i][j]) * kk[j][c];
                            q[c] = clamp01(p[c] + hh * acc);
                        }
                        eval_W<P, RAT, 0, R, LDS>(pv, ar, q, gin, d, cperp, dthr, kk[i], dummy, dg, c_fp64, false,
                                                  dr2, dx, dx);
                        ++c_w;
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    R acc = R(0);
#pragma unroll
                    for (int i = 0; i < 6; ++i)
                        if (i < S) acc += R(tb.b[i]) * kk[i][c];
                    p5[c] = p[c] + hh * acc;
                }
                err = isfinite(p5[0] + p5[1] + p5[2]) ? R(0) : R(NAN);
            } else {
                // Eq. (implicitEuler): Newton on G(z) = z - hh W(p + z) (Eq.
                // (newtonimpliciteuler)) from the explicit Euler predictor; each
                // update solves (J_phi J_G) dz = -J_phi G with, at q = p + z,
                //   J_phi J_G = H_phi (hh W(q)) + (I - hh J_V) J_phi,  J_V = c (d d^T - I),
                //   J_phi G   = J_phi z - hh V(phi(q))
                // (Eqs. (newtonimpliciteulerReformulated), (JacG)); iterates projected
                // onto P
                // Newton converges quadratically: once an update is below tolz the
                // point is at rounding level (FP32: updates below 1e-5 leave ~1e-10)
                const R tolz = sizeof(R) == 4 ? R(1e-5) : R(1e-12);
                const R hc = hh * cperp;
                R z[3] = {hh * k1[0], hh * k1[1], hh * k1[2]};
                bool conv = false;
#pragma unroll 1
                for (int it = 0; it < 16 && !conv; ++it) {
                    R q[3], xq[3], Jq[3][3], Hq[3][6];
#pragma unroll
                    for (int c = 0; c < 3; ++c) q[c] = clamp01(p[c] + z[c]);
                    eval_volume_h<P, RAT, R, LDS>(pv, ar, q, xq, Jq, Hq);
                    ++c_w;
                    R r[3] = {gin[0] - xq[0], gin[1] - xq[1], gin[2] - xq[2]}, hV[3];
                    const R rd = dot3(r, d);
#pragma unroll
                    for (int c = 0; c < 3; ++c) hV[c] = hh * (d[c] + cperp * (r[c] - rd * d[c]));
                    R ju[3] = {Jq[0][0], Jq[1][0], Jq[2][0]}, jv[3] = {Jq[0][1], Jq[1][1], Jq[2][1]},
                      jw[3] = {Jq[0][2], Jq[1][2], Jq[2][2]}, hw[3];
                    solve_cols(ju, jv, jw, hV, hw);
                    // columns of J_phi J_G; (d^T J_phi) for the J_V term
                    R dJ[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) dJ[a] = d[0] * Jq[0][a] + d[1] * Jq[1][a] + d[2] * Jq[2][a];
                    R M[3][3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const R *Hi = Hq[i];
                        // packed (uu, vv, ww, uv, uw, vw) applied to hw, column by column
                        M[i][0] = (R(1) + hc) * Jq[i][0] - hc * d[i] * dJ[0] + Hi[0] * hw[0] + Hi[3] * hw[1] + Hi[4] * hw[2];
                        M[i][1] = (R(1) + hc) * Jq[i][1] - hc * d[i] * dJ[1] + Hi[3] * hw[0] + Hi[1] * hw[1] + Hi[5] * hw[2];
                        M[i][2] = (R(1) + hc) * Jq[i][2] - hc * d[i] * dJ[2] + Hi[4] * hw[0] + Hi[5] * hw[1] + Hi[2] * hw[2];
                    }
                    R rhs[3], dz[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) rhs[i] = hV[i] - (Jq[i][0] * z[0] + Jq[i][1] * z[1] + Jq[i][2] * z[2]);
                    const R m0[3] = {M[0][0], M[1][0], M[2][0]}, m1[3] = {M[0][1], M[1][1], M[2][1]},
                            m2[3] = {M[0][2], M[1][2], M[2][2]};
                    solve_cols(m0, m1, m2, rhs, dz);
                    if (!isfinite(dz[0] + dz[1] + dz[2])) break;
                    // the iterate projected onto P (a step that would leave P stops
                    // on its boundary); converged once it moves by at most tolz
                    R mv = R(0);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const R zn = clamp01(p[c] + z[c] + dz[c]) - p[c];
                        mv = fmax(mv, fabs(zn - z[c]));
                        z[c] = zn;
                    }
                    conv = mv <= tolz;
                }
                if (!conv) {
                    fl |= IVR_FLAG_RESTART_FAIL;
                    count_rare(C_RESTART_FAIL);
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) p5[c] = p[c] + z[c];
                err = isfinite(p5[0] + p5[1] + p5[2]) ? R(0) : R(NAN);
            }
            ++c_steps;
            const bool finite = isfinite(err);
            const bool accept = METHOD != kOde || (err <= tol) || (hh <= hmin);
            if (accept) {
                s += hh;
                fl &= ~kJustRestarted;
                if (!finite) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) p5[c] = p[c];   // at h_min: hold p
                }
                if (Lend - s <= R(1e-6) * L && (fl & kExitOnPlane)) {
                    // last step ends on the cutting plane: its end is sampled
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        p[c] = clamp01(isfinite(err) ? p5[c] : p[c]);
                        gin[c] += hh * d[c];
                    }
                    pending = true;
                    h_prev = hh;
                    fl |= kEndSample;
                } else if (Lend - s <= R(1e-6) * L) {
                    // last step ends on the exit fragment (or, at a singular exit,
                    // 1e-4 of the chord short of it): close with the exit's rho
                    const R hl = hh + (L - Lend);
                    const R mo = isfinite(m_out) ? m_out : (rho_out - rho_prev) / hl;
                    composite(fp, views[vid].fp, vls[vid], rho_prev, m_prev, rho_out, mo, hl, C, A, c_sub);
                    ++c_samp;
                    done = true;
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        p[c] = clamp01(p5[c]);
                        gin[c] += hh * d[c];
                    }
                    pending = true;
                    h_prev = hh;
                }
            } else {
                ++c_rej;
            }
            // step-size control for a 4(5) pair; no growth on the attempt after a
            // rejection (the error estimate just proved the step too long).  The
            // fixed-step methods take h_max again at the next step.
            if constexpr (METHOD == kOde) {
            R fac = R(2.5);
            if (!finite) {
                fac = R(0.2);
            } else if (err > R(0)) {
                fac = R(0.8) * pow_fifth(tol / err);
                fac = fac < R(0.2) ? R(0.2) : (fac > R(2.5) ? R(2.5) : fac);
            }
            if (accept && rejected && fac > R(1)) fac = R(1);
            rejected = !accept;
            h = hh * fac;
            h = h > hmax ? hmax : h;
            h = h < hmin ? hmin : h;
            }
            if (++iters >= 20000 && !done) {
                count_rare(C_RK_ITER_CAP);
                fl |= IVR_FLAG_ITER_CAP;
                done = true;
            }
            }
        }
        if (done) {
            // the result (C, alpha) over the first 16 bytes of the segment's own
            // record (read at the refill; only its pixel is needed after this)
            *reinterpret_cast<float4 *>(segs + sid) = make_float4(float(C[0]), float(C[1]), float(C[2]), float(A));
            active = false;
            if constexpr (DIAG) {
                if (dg_tout < dg_t) {   // the exit before the last sample
                    fl |= IVR_FLAG_DEPTH_ORDER;
                    ++c_ord;
                }
                float *dpv = views[vid].dp;
                if (dpv) atomicMax(reinterpret_cast<unsigned int *>(dpv + dg_pix), __float_as_uint(dg_dp));
            }
            fl &= kPublicFlags;
            if (fl) {
                uint32_t *fv = views[vid].flags;
                if (fv) atomicOr(fv + segs[sid].pixel, fl);
            }
        }
        }
        __syncthreads();   // every wave is done with this block's LDS copy
    }
    if (fp.collect) {
        flush_counter(ctr, C_RK_STEPS, c_steps);
        flush_counter(ctr, C_RK_REJECTED, c_rej);
        flush_counter(ctr, C_SAMPLES, c_samp);
        flush_counter(ctr, C_W_EVALS, c_w);
        flush_counter(ctr, C_FP64_SOLVES, c_fp64);
        flush_counter(ctr, C_SUBSAMPLES, c_sub);
        if constexpr (DIAG) {
            flush_counter(ctr, C_DP_OVER, c_dpo);
            flush_counter(ctr, C_ORDER_BAD, c_ord);
        }
    }
}

// LDS budget of the staged block per integrator workgroup.
constexpr size_t kLdsBlockBytes = 48 * 1024;

template <int P, bool RAT, typename R, bool LDS, int METHOD, int FIELD = 0, bool DIAG = false>
static hipError_t launch_integrate_t(const Model &m, const ViewRec *views, int n_views, const void *segs,
                                     const IntegrateArgs &a, unsigned long long *ctr,
                                     int n_cu, const LaunchCfg &lc, hipStream_t st) {
    const size_t lds = sizeof(ViewLds) * (size_t)n_views +
                       (LDS ? (size_t)a.max_cp * sizeof(float4) +
                                  (RAT ? (size_t)(a.max_cp + 3) / 4 * 4 * sizeof(float) : 0) +
                                  (size_t)a.max_tab * sizeof(float)
                            : 0);
    const int block = lc.int_block;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_integrate<P, RAT, R, LDS, METHOD, FIELD, DIAG>, block, lds) !=
            hipSuccess || nb < 1)
        nb = 1;
    if (lc.int_waves_cu > 0) nb = std::min(nb, std::max(1, lc.int_waves_cu / (block / 64)));
    hipLaunchKernelGGL((k_integrate<P, RAT, R, LDS, METHOD, FIELD, DIAG>), dim3(n_cu * nb), dim3(block), lds, st, m, views,
                       n_views, (Seg<R> *)segs, a.order, a.pperm, a.q_begin, a.q_end, a.pbase,
                       a.pcount, a.pcur, LDS ? a.max_cp : 0, ctr);
    return hipGetLastError();
}

template <int P, bool RAT, int METHOD>
static hipError_t launch_integrate_m(bool fp64, const Model &m, const ViewRec *views, int n_views,
                                     void *segs, const IntegrateArgs &a, unsigned long long *ctr, int n_cu,
                                     const LaunchCfg &lc, hipStream_t st) {
    if (fp64)
        return launch_integrate_t<P, RAT, double, false, METHOD>(m, views, n_views, segs, a, ctr, n_cu, lc, st);
    const size_t bytes = (size_t)a.max_cp * sizeof(float4) +
                         (RAT ? (size_t)(a.max_cp + 3) / 4 * 4 * sizeof(float) : 0) +
                         (size_t)a.max_tab * sizeof(float);
    if (bytes <= kLdsBlockBytes)
        return launch_integrate_t<P, RAT, float, true, METHOD>(m, views, n_views, segs, a, ctr, n_cu, lc, st);
    return launch_integrate_t<P, RAT, float, false, METHOD>(m, views, n_views, segs, a, ctr, n_cu, lc, st);
}

template <int P, bool RAT>
static hipError_t launch_integrate_pr(bool fp64, int method, const Model &m, const ViewRec *views, int n_views,
                                      void *segs, const IntegrateArgs &a, unsigned long long *ctr, int n_cu,
                                      const LaunchCfg &lc, hipStream_t st) {
    if (method == IVR_INTERIOR_RF)
        return launch_integrate_m<P, RAT, kRootFinding>(fp64, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    if (method >= IVR_INTERIOR_RK1 && method <= IVR_INTERIOR_RKF5)
        return launch_integrate_m<P, RAT, kFixedRK>(fp64, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    if (method == IVR_INTERIOR_IRK1)
        return launch_integrate_m<P, RAT, kImplicitEuler>(fp64, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    return launch_integrate_m<P, RAT, kOde>(fp64, m, views, n_views, segs, a, ctr, n_cu, lc, st);
}


}  // namespace ivr
