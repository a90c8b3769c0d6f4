// gfx950 kernels of the per-pixel hot path.
//
//   k_fragments  one wave per 8x8 pixel tile.  For every block whose box the
//                tile's rays hit: every face element box hit by the ray starts a
//                Newton solve of S_f(a,b) = o + t d from the element centre
//                (FP32, then FP64 refinement), crossings are classified
//                front/back facing, de-duplicated, sorted and paired per block
//                by Algorithm "Blockwise depth-sorting".  Segments are written
//                contiguously per pixel (sorted by entry depth) after a wave
//                prefix sum, and their indices are appended to one queue per
//                degree class.
//   k_integrate  persistent: every lane owns one segment, runs one RKF45 attempt
//                per loop iteration on p' = W(p) (Eqs. (odepar), (VgVp)), samples
//                rho at every accepted step, applies the transfer function with
//                supersampling and composites by Algorithm "Front-to-back
//                compositing"; finished lanes take the next segment from the
//                class queue (wave-aggregated atomic), so short and long
//                segments share waves without idling.
//   k_merge      per pixel: over-composites its segments front to back.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ivr.h"
#include "ivr_internal.h"
#include "ivr_mlp_dev.h"
#include "ivr_spline.h"

namespace ivr {

using u32 = uint32_t;
using u64 = unsigned long long;

constexpr int kFlat = 256;    // candidates solved per pass of the flattened solve
constexpr int kRayStart = 255;  // entry index of a segment that starts on the near plane
constexpr int kFragLds = 16;  // crossings per ray kept in LDS (the rest in scratch)
constexpr int kExtra = 64;    // second roots of one element per pass of the flattened solve

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

__device__ __forceinline__ bool slab(const float (&o)[3], const float (&inv)[3], const float *lo,
                                     const float *hi) {
    float tmin = 0.f, tmax = INFINITY;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float t0 = (lo[c] - o[c]) * inv[c], t1 = (hi[c] - o[c]) * inv[c];
        tmin = fmaxf(tmin, fminf(t0, t1));
        tmax = fminf(tmax, fmaxf(t0, t1));
    }
    return tmin <= tmax;
}

template <typename R>
struct Frag {
    // a boundary crossing: ray parameter, face parameters (a, b), and the block,
    // face and facing packed as block << 4 | face << 1 | entering (16 B in FP32)
    R t, a, b;
    uint32_t info;
};

// The parameter point of a crossing: face parameters (a, b) on the face of info.
template <typename R>
__device__ __forceinline__ void face_point(uint32_t info, R a, R b, R (&p)[3]) {
    const int face = (int)((info >> 1) & 7u), dn = face >> 1;
    const R pn = (face & 1) ? R(1) : R(0);
    // (a, b) are the two other directions in increasing order
    p[0] = dn == 0 ? pn : a;
    p[1] = dn == 0 ? a : (dn == 1 ? pn : b);
    p[2] = dn == 2 ? pn : b;
}

// A root of one candidate, handed from the lane that solved it to the lane that
// owns the ray: the crossing (t, a, b, info as in Frag; info ~0 when there is
// none) and the info of the shared face's crossing at the same root (or ~0).
template <typename R>
struct RootRec {
    R t, a, b;
    uint32_t info, tinfo;
};

// Ray (t >= 0) against an oriented box; [tmin, tmax] is the ray's interval inside.
template <typename Box3>
__device__ __forceinline__ bool obb_hit(const Box3 &E, const float (&o)[3], const float (&d)[3],
                                        float &tmin, float &tmax) {
    const float oc[3] = {o[0] - E.c[0], o[1] - E.c[1], o[2] - E.c[2]};
    tmin = 0.f;
    tmax = INFINITY;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float po = E.ax[r][0] * oc[0] + E.ax[r][1] * oc[1] + E.ax[r][2] * oc[2];
        const float pd = E.ax[r][0] * d[0] + E.ax[r][1] * d[1] + E.ax[r][2] * d[2];
        const float inv = __builtin_amdgcn_rcpf(pd);
        const float t0 = (-E.ext[r] - po) * inv, t1 = (E.ext[r] - po) * inv;
        tmin = fmaxf(tmin, fminf(t0, t1));
        tmax = fminf(tmax, fmaxf(t0, t1));
    }
    return tmin <= tmax;
}

// The test alone: per axis the slab's interval is -po/pd -+ ext/|pd| (ext >= 0),
// one product and two FMAs with the reciprocal's absolute value.  Boxes are
// padded well beyond the FP32 rounding of either form.
template <typename Box3>
__device__ __forceinline__ bool obb_hit(const Box3 &E, const float (&o)[3], const float (&d)[3]) {
    const float oc[3] = {o[0] - E.c[0], o[1] - E.c[1], o[2] - E.c[2]};
    float tmin = 0.f, tmax = INFINITY;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float po = E.ax[r][0] * oc[0] + E.ax[r][1] * oc[1] + E.ax[r][2] * oc[2];
        const float pd = E.ax[r][0] * d[0] + E.ax[r][1] * d[1] + E.ax[r][2] * d[2];
        const float inv = __builtin_amdgcn_rcpf(pd);
        const float mid = -po * inv, ai = fabsf(inv);
        tmin = fmaxf(tmin, fmaf(-E.ext[r], ai, mid));
        tmax = fminf(tmax, fmaf(E.ext[r], ai, mid));
    }
    return tmin <= tmax;
}

// Front facing: the sign of (J^-1 d) along the face's inward normal.  By
// Cramer's rule it equals the sign of d . (S_a x S_b) times the face's side,
// the orientation of (a, b, n) and the block's orientation (sign of det J).
template <typename R>
__device__ __forceinline__ int facing(int face, float orient, const R (&Sa)[3], const R (&Sb)[3],
                                      const R (&d)[3], bool &grazing) {
    R nrm[3];
    cross3(Sa, Sb, nrm);
    const R g = dot3(nrm, d);
    grazing = !(fabs(g) > R(1e-10) * sqrt(dot3(nrm, nrm)));
    const R sigma = ((face >> 1) == 1) ? R(-1) : R(1), side = (face & 1) ? R(-1) : R(1);
    return (side * sigma * g * R(orient)) > R(0);
}

// Newton on S_f(a,b) - (o + t d) = 0 (Eqs. (F), (newtonsmethod) restricted to
// the face) in precision RN from (a, b); true when it converges.
template <int P, bool RAT, typename RN>
__device__ __forceinline__ bool face_newton(const FaceView<RN> &fv, const Arrays<RN> &ar,
                                            const RN (&o)[3], const RN (&d)[3], RN tol, int max_it,
                                            RN &a, RN &b, RN &t, RN (&Sa)[3], RN (&Sb)[3], u32 &n_iter) {
    RN S[3];
    eval_face<P, RAT, RN>(fv, ar, a, b, S, Sa, Sb);
    t = (S[0] - o[0]) * d[0] + (S[1] - o[1]) * d[1] + (S[2] - o[2]) * d[2];
    for (int it = 0; it < max_it; ++it) {
        ++n_iter;
        RN F[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) F[q] = S[q] - o[q] - t * d[q];
        if (dot3(F, F) <= tol * tol) return true;
        RN nd[3] = {-d[0], -d[1], -d[2]}, rhs[3] = {-F[0], -F[1], -F[2]}, st[3];
        solve_cols(Sa, Sb, nd, rhs, st);
        a += st[0];
        b += st[1];
        t += st[2];
        if (!(a >= RN(-1) && a <= RN(2) && b >= RN(-1) && b <= RN(2))) return false;
        eval_face<P, RAT, RN>(fv, ar, a, b, S, Sa, Sb);
    }
    return false;
}

// Boundary roots of a ray in one candidate element E (Eqs. (F), (newtonsmethod)
// restricted to the face): FP32 Newton, then FP64 refinement.  First seed by
// seed_mode:
//   PLAIN  the element centre;
//   BOX    the point of the ray in the middle of its passage through E's box,
//          mapped to (a, b) through the box axes;
//   MLP    the block's learned inverse map at that same point, restricted to the
//          face's (a, b).
// If Newton does not converge from it: the element centre and its four quarter
// points.  A root on the closed face becomes the crossing in out and, across a
// shared face, the neighbouring block's crossing (out.tinfo).  A ray nearly
// tangent to the element may cross it twice: then `again` is set, and a second
// call with T1 = the first root's depth looks for another root by Newton from
// points of the ray's passage through the element's box on both sides of it.
template <int P, bool RAT, typename RN>
__device__ void face_root(const Model &m, const DevPatch &Pd, const FaceElem &E, const double (&od)[3],
                          const double (&dd)[3], const float (&of)[3], const float (&df)[3],
                          const FrameParams &fp, const float (&mseed)[3], float T1, RootRec<RN> &out,
                          bool &again, u32 &n_iter, u32 &n_polish) {
    const int face = E.face;
    const FaceView<RN> fv = face_view<RN>(Pd, face);
    const Arrays<RN> ar = arrays_of(m, RN(0));
    const RN o[3] = {RN(od[0]), RN(od[1]), RN(od[2])}, d[3] = {RN(dd[0]), RN(dd[1]), RN(dd[2])};
    const RN tol = (sizeof(RN) == 4 ? RN(2e-6) : RN(1e-12)) * RN(fp.scaled);
    const RN ac = RN(0.5) * (RN(E.a0) + RN(E.a1)), bc = RN(0.5) * (RN(E.b0) + RN(E.b1));
    const RN ha = RN(0.5) * (RN(E.a1) - RN(E.a0)), hb = RN(0.5) * (RN(E.b1) - RN(E.b0));
    int dn, da, db;
    face_dirs(face, dn, da, db);
    float t0, t1;
    obb_hit(E, of, df, t0, t1);
    t1 = fminf(t1, t0 + 4.0f * fp.scale);
    // Two crossings need the ray's slope against the element's plane below the
    // surface's largest slope there (the surface's height along the ray has a
    // stationary point between them); E.graze bounds that slope from the net.
    const bool tangent = fabsf(E.ax[2][0] * df[0] + E.ax[2][1] * df[1] + E.ax[2][2] * df[2]) < E.graze;
    const bool second = T1 >= 0.f;
    const double tsame = 2e-5 * fp.scaled;   // one crossing
    const FaceView<double> fv64 = face_view<double>(Pd, face);
    const Arrays<double> ar64 = arrays_of(m, 0.0);
    const double tol64 = 1e-12 * fp.scaled;
    const int s_begin = second ? 6 : (fp.seed_mode == IVR_SEED_PLAIN ? 1 : 0);
    const int s_end = second ? 12 : 6;
    // Seeds in turn until Newton converges; the first search ends there, with or
    // without a crossing, the second goes on past roots off the face and the
    // first root again.
    for (int seed = s_begin; seed < s_end; ++seed) {
        RN a, b, t, Sa[3], Sb[3];
        if (seed == 0 || seed >= 6) {
            // the ray's point in the middle of its interval in the box (for the
            // second root: points of that interval 1 and 3 eighths of its length
            // before and after the first root, then its ends)
            const float h = 0.125f * (t1 - t0);
            const float tm = seed == 0 ? 0.5f * (t0 + t1)
                             : seed < 10 ? fminf(fmaxf(T1 + ((seed & 1) ? h : -h) * (seed < 8 ? 1.f : 3.f), t0), t1)
                                         : (seed == 10 ? t0 : t1);
            float x[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) x[q] = of[q] + tm * df[q];
            if (seed == 0 && fp.seed_mode == IVR_SEED_MLP && isfinite(mseed[0])) {
                a = RN(clamp01(da == 0 ? mseed[0] : mseed[1]));
                b = RN(clamp01(db == 1 ? mseed[1] : mseed[2]));
            } else {
#pragma unroll
                for (int q = 0; q < 3; ++q) x[q] -= E.c[q];
                const float xu = (E.ax[0][0] * x[0] + E.ax[0][1] * x[1] + E.ax[0][2] * x[2]) / E.ext[0];
                const float xv = (E.ax[1][0] * x[0] + E.ax[1][1] * x[1] + E.ax[1][2] * x[2]) / E.ext[1];
                a = ac + ha * RN(fminf(fmaxf(xu, -1.f), 1.f));
                b = bc + hb * RN(fminf(fmaxf(xv, -1.f), 1.f));
            }
        } else if (seed == 1) {
            a = ac;
            b = bc;
        } else {
            a = ac + ha * RN((seed & 1) ? -0.5 : 0.5);
            b = bc + hb * RN((seed & 2) ? -0.5 : 0.5);
        }
        if (!face_newton<P, RAT, RN>(fv, ar, o, d, tol, fp.max_newton, a, b, t, Sa, Sb, n_iter)) continue;
        const RN mg = RN(1e-4);
        if (!(a >= -mg && a <= RN(1) + mg && b >= -mg && b <= RN(1) + mg && t > RN(0))) {
            if (second) continue;
            return;
        }
        // FP64 refinement of the boundary root by mixed-precision iterative
        // refinement: the residual S(a, b) - o - t d in FP64 from the FP64 control
        // points, the correction from FP32 tangents.  It contracts by the FP32
        // tangents' relative error (~1e-7) times the system's condition per step,
        // so from the FP32 stopping residual (<= 2e-6 scale) one step reaches
        // ~1e-12 scale.  A ray nearly tangent to the face has a large condition and
        // an FP32 root far off along the tangent: after a step above 1e-4 in
        // (a, b) the FP32 tangents are taken again at the new point.  A step of at
        // most 1e-5 in (a, b) and 1e-5 scale in t leaves a residual below the 1e-9
        // scale acceptance bound and is taken without evaluating it again.
        double A = a, B = b, T = t, S2[3], F2[3], Sa2[3], Sb2[3];
        bool ok = false;
        for (int k = 0; k < 4; ++k) {
            eval_face<P, RAT, double, false>(fv64, ar64, A, B, S2, Sa2, Sb2);
#pragma unroll
            for (int q = 0; q < 3; ++q) F2[q] = S2[q] - od[q] - T * dd[q];
            const double r2 = dot3(F2, F2);
            if (r2 <= tol64 * tol64) {
                ok = true;
                break;
            }
            if (k == 3) {
                ok = r2 <= 1e-18 * fp.scaled * fp.scaled;
                break;
            }
            ++n_polish;
            RN nd[3] = {-d[0], -d[1], -d[2]}, rhs[3] = {RN(-F2[0]), RN(-F2[1]), RN(-F2[2])}, st[3];
            solve_cols(Sa, Sb, nd, rhs, st);
            A += double(st[0]);
            B += double(st[1]);
            T += double(st[2]);
            const double sab = fmax(fabs(double(st[0])), fabs(double(st[1])));
            if (sab <= 1e-5 && fabs(double(st[2])) <= 1e-5 * fp.scaled) {
                ok = true;
                break;
            }
            if (sab > 1e-4) {
                RN S[3];
                eval_face<P, RAT, RN>(fv, ar, RN(A), RN(B), S, Sa, Sb);
            }
        }
        // A crossing is a root on the closed face up to 1e-9 in (a, b): the refined
        // root is accurate to ~1e-11, so a crossing exactly at an edge is kept, while
        // a ray passing just outside the edge yields no crossing of this face (its
        // crossing of the block, if any, is a root on the neighbouring face).
        const double mg64 = 1e-9;
        if (!ok || !(A >= -mg64 && A <= 1.0 + mg64 && B >= -mg64 && B <= 1.0 + mg64 && T > 0.0)) {
            if (second) continue;
            return;
        }
        if (second && fabs(T - double(T1)) <= tsame) continue;   // the first root again
#pragma unroll
        for (int q = 0; q < 3; ++q) {   // facing from the FP32 tangents at the root
            Sa2[q] = double(Sa[q]);
            Sb2[q] = double(Sb[q]);
        }
        bool grazing;
        const int ent = facing(face, Pd.orient, Sa2, Sb2, dd, grazing);
        if (grazing) return;
        // the same root is the crossing of the block on the other side of a shared face
        const int tw = Pd.twin[face];
        int tent = 0;
        if (tw >= 0) tent = facing(tw & 7, m.patches[tw >> 3].orient, Sa2, Sb2, dd, grazing);
        out.t = RN(T);
        out.a = RN(clamp01(A));
        out.b = RN(clamp01(B));
        out.info = ((uint32_t)E.patch << 4) | ((uint32_t)face << 1) | (uint32_t)(ent & 1);
        out.tinfo = tw >= 0 ? (((uint32_t)(tw >> 3) << 4) | ((uint32_t)(tw & 7) << 1) | (uint32_t)(tent & 1))
                            : 0xFFFFFFFFu;
        again = tangent && !second;
        return;
    }
}

// The root of one candidate in out (info stays ~0 when there is none); T1 < 0
// for the first search, else the depth of the first root (see face_root).
template <typename R>
__device__ __forceinline__ void face_root_any(const Model &m, const DevPatch &Pd, const FaceElem &E,
                                              const double (&od)[3], const double (&dd)[3],
                                              const float (&of)[3], const float (&df)[3],
                                              const FrameParams &fp, const float (&ms)[3], float T1,
                                              RootRec<R> &out, bool &again, u32 &ni, u32 &np) {
    out.info = out.tinfo = 0xFFFFFFFFu;
    again = false;
    switch (Pd.deg * 2 + Pd.rational) {
    case 2: face_root<1, false, R>(m, Pd, E, od, dd, of, df, fp, ms, T1, out, again, ni, np); break;
    case 3: face_root<1, true, R>(m, Pd, E, od, dd, of, df, fp, ms, T1, out, again, ni, np); break;
    case 4: face_root<2, false, R>(m, Pd, E, od, dd, of, df, fp, ms, T1, out, again, ni, np); break;
    case 5: face_root<2, true, R>(m, Pd, E, od, dd, of, df, fp, ms, T1, out, again, ni, np); break;
    case 6: face_root<3, false, R>(m, Pd, E, od, dd, of, df, fp, ms, T1, out, again, ni, np); break;
    default: face_root<3, true, R>(m, Pd, E, od, dd, of, df, fp, ms, T1, out, again, ni, np); break;
    }
}

// rho and d rho/ds at a parameter point; returns det J_phi there.
template <typename R>
__device__ __forceinline__ R rho_ds_any(const Model &m, const DevPatch &Pd, const R (&p)[3],
                                        const R (&d)[3], R &rho, R &drho) {
    const PatchView<R> pv = view_of<R>(Pd);
    const Arrays<R> ar = arrays_of(m, R(0));
    switch (Pd.deg * 2 + Pd.rational) {
    case 2: return eval_rho_ds<1, false>(pv, ar, p, d, rho, drho);
    case 3: return eval_rho_ds<1, true>(pv, ar, p, d, rho, drho);
    case 4: return eval_rho_ds<2, false>(pv, ar, p, d, rho, drho);
    case 5: return eval_rho_ds<2, true>(pv, ar, p, d, rho, drho);
    case 6: return eval_rho_ds<3, false>(pv, ar, p, d, rho, drho);
    default: return eval_rho_ds<3, true>(pv, ar, p, d, rho, drho);
    }
}

__device__ __forceinline__ u32 wave_incl_scan(u32 v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const u32 x = __shfl_up(v, off);
        if (lane >= off) v += x;
    }
    return v;
}

// The view that owns batch tile g (views sorted by tile_begin; uniform per wave).
__device__ __forceinline__ int view_of_tile(const ViewRec *views, int n_views, u32 g) {
    int lo = 0, hi = n_views;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (__builtin_amdgcn_readfirstlane(views[mid].tile_begin) <= g) lo = mid;
        else hi = mid;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// The fragment pass in two launches.  MODE 1 traverses the block, face, tile
// and element boxes and records each wave's candidates (elements whose box the
// ray hits), with MLP seeds one network query each (evaluated by k_mlp_seeds in
// between).  MODE 2 solves the candidates, pairs the
// roots into segments and writes them.
template <typename R, int MODE>
__global__ __launch_bounds__(64) void k_fragments(Model m, const ViewRec *views, int n_views,
                                                  u32 n_tiles, LaunchCfg lc, Seg<R> *segs, u32 seg_cap,
                                                  uint2 *seg_kr, u32 *pcount, QueueState *qs,
                                                  uint2 *pixseg, CandLists mq, u64 *ctr) {
    const int lane = threadIdx.x;
    // Consecutive blocks are dealt round-robin to the 8 XCDs.  With xcd_chunk = C
    // > 0, XCD x's j-th block takes tile j mod C of chunk (j / C) * 8 + x: runs of C
    // neighbouring tiles (which test the same blocks and elements) share one XCD's
    // L2, while the chunks still interleave over the image across XCDs (balance).
    // Tiles past the last whole round of 8 C keep the plain order.
    u32 g = blockIdx.x;
    if (lc.xcd_chunk > 0) {
        const u32 C = (u32)lc.xcd_chunk, full = (n_tiles / (8u * C)) * (8u * C);
        if (g < full) {
            const u32 x = g & 7u, j = g >> 3;
            g = ((j / C) * 8u + x) * C + (j % C);
        }
    }
    // the view is uniform over the wave: its record is read once through the
    // scalar cache into a private copy (no reloads after the kernel's stores)
    const int v = view_of_tile(views, n_views, g);
    const ViewRec vr = views[v];
    const FrameParams &fp = vr.fp;
    const u32 tl = g - vr.tile_begin;
    const int th = 64 / lc.tile_w;
    const int px = (int)(tl % vr.tiles_x) * lc.tile_w + (lane % lc.tile_w);
    const int py = (int)(tl / vr.tiles_x) * th + (lane / lc.tile_w);
    const bool valid = px < fp.width && py < fp.height;
    const u32 pixel = valid ? (u32)(py * fp.width + px) : 0u;

    double dd[3];
    ray_dir(fp, valid ? px : 0, valid ? py : 0, dd);
    const double od[3] = {fp.eye[0], fp.eye[1], fp.eye[2]};
    float of[3], df[3], inv[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        of[q] = float(od[q]);
        df[q] = float(dd[q]);
        inv[q] = 1.0f / df[q];
    }
    u32 c_anom = 0, c_fovf = 0, c_sovf = 0, c_box = 0, c_newton = 0, c_iter = 0, c_pol = 0, c_mlp = 0;

    // 1. face elements whose oriented box the ray hits (block and face boxes
    //    first) become Newton seeds; 2. the seeds are solved (a wave's 64 at a
    //    time whatever their rays, in the second launch).
    u32 cand[kCandCap];
    u32 cpos[MODE == 1 ? kCandCap : 1];   // position in the wave's block-major list
    int ncand = 0;
    // The ray's boundary crossings, unsorted in the order they were found: depth
    // and info (Frag) of the first kFragLds in LDS (slot-major, so a wave's
    // accesses to one slot are consecutive), of the rest in the lane's scratch
    // array, which also keeps every crossing's face parameters (a, b).
    __shared__ R s_ft[MODE == 2 ? kFragLds * 64 : 1];
    __shared__ u32 s_fi[MODE == 2 ? kFragLds * 64 : 1];
    Frag<R> fr[MODE == 1 ? 1 : kFragCap];
    int nfr = 0;
    auto ft = [&](int q) __attribute__((always_inline)) -> R {
        return q < kFragLds ? s_ft[q * 64 + lane] : fr[q].t;
    };
    auto fi = [&](int q) __attribute__((always_inline)) -> u32 {
        return q < kFragLds ? s_fi[q * 64 + lane] : fr[q].info;
    };
    // a crossing of the same block and facing within tol of depth t is there already
    auto known = [&](u32 info, R t, R tol) __attribute__((always_inline)) -> bool {
        bool dup = false;
        for (int q = 0; q < nfr; ++q) dup |= ((fi(q) ^ info) & ~0xEu) == 0u && fabs(ft(q) - t) <= tol;
        return dup;
    };
    auto push = [&](u32 info, R t, R a, R b) __attribute__((always_inline)) {
        if (nfr >= fp.max_frag) {
            ++c_fovf;
            return;
        }
        const int q = nfr++;
        fr[q].a = a;
        fr[q].b = b;
        if (q < kFragLds) {
            s_ft[q * 64 + lane] = t;
            s_fi[q * 64 + lane] = info;
        } else {
            fr[q].t = t;
            fr[q].info = info;
        }
    };
    // A root of one of the ray's candidates: the block's crossing and the
    // neighbour's across a shared face, each dropped on its own when the list
    // has it already (the same crossing through an edge or corner shared by
    // elements or faces).  A ray through an edge of four blocks crosses two of
    // them at one point: their entry and exit come from different faces'
    // roots, whose other crossings are duplicates.
    auto add_root = [&](const RootRec<R> &rr) __attribute__((always_inline)) {
        if (rr.info == 0xFFFFFFFFu) return;
        const R tol = R(2e-5 * fp.scaled);
        if (!known(rr.info, rr.t, tol)) push(rr.info, rr.t, rr.a, rr.b);
        if (rr.tinfo != 0xFFFFFFFFu && !known(rr.tinfo, rr.t, tol)) push(rr.tinfo, rr.t, rr.a, rr.b);
    };
    // The lane's listed candidates, all lanes in step (only for rays whose
    // candidates the first launch could not record).  Always inlined: a call
    // would see the kernel's pointers as generic and load through flat.
    auto solve_candidates = [&]() __attribute__((always_inline)) {
        for (int k = 0; __ballot(k < ncand) != 0; ++k) {
            if (k < ncand) {
                const FaceElem E = m.elems[cand[k]];
                const float ms[3] = {NAN, NAN, NAN};
                float T1 = -1.f;
                ++c_newton;
                for (int s = 0; s < 2; ++s) {   // a second search where the ray is nearly tangent
                    RootRec<R> rr;
                    bool again;
                    face_root_any<R>(m, m.patches[E.patch], E, od, dd, of, df, fp, ms, T1, rr, again, c_iter,
                                     c_pol);
                    add_root(rr);
                    if (!again) break;
                    T1 = float(rr.t);
                }
            }
        }
        ncand = 0;
    };
    // The traversal: on_hit(e, he) for every face element e of a tile the wave
    // tests (he: the lane's ray hits its box), after_block(pi, nc0) after each
    // block the wave's rays may hit, with nc0 the lane's candidate count before it.
    auto traverse = [&](bool act, auto &&on_hit, auto &&after_block) __attribute__((always_inline)) {
        for (int pi = vr.patch_begin; pi < vr.patch_end; ++pi) {
            const DevPatch &Pd = m.patches[pi];
            ++c_box;
            const bool hp = act && slab(of, inv, Pd.box, Pd.box + 3);
            if (__ballot(hp) == 0) continue;
            const int nc0 = ncand;
            for (int f = 0; f < 6; ++f) {
                if ((Pd.face_skip >> f) & 1) continue;   // tested from the neighbouring block
                c_box += hp;
                const bool hf = hp && slab(of, inv, Pd.fbox[f], Pd.fbox[f] + 3);
                if (__ballot(hf) == 0) continue;
                for (int ti = Pd.tile_off[f]; ti < Pd.tile_off[f + 1]; ++ti) {
                    const FaceTile &T = m.tiles[ti];
                    c_box += hf;
                    const bool ht = hf && obb_hit(T, of, df);
                    if (__ballot(ht) == 0) continue;
                    const bool split = T.sub_end > T.sub_begin;
                    for (int si = split ? T.sub_begin : ti; si < (split ? T.sub_end : ti + 1); ++si) {
                        const FaceTile &S = m.tiles[si];
                        bool hs = ht;
                        if (split) {
                            c_box += ht;
                            hs = ht && obb_hit(S, of, df);
                            if (__ballot(hs) == 0) continue;
                        }
                        for (int e = S.elem_begin; e < S.elem_end; ++e) {
                            c_box += hs;
                            on_hit((u32)e, hs && obb_hit(m.elems[e], of, df));
                        }
                    }
                }
            }
            after_block(pi, nc0);
        }
    };
    auto no_block = [&](int, int) __attribute__((always_inline)) {};
    bool c_more = false;   // the lane found more candidates than its list holds
    if constexpr (MODE == 1) {
        auto hit = [&](u32 e, bool he) __attribute__((always_inline)) {
            if (he) {
                if (ncand < kCandCap) cand[ncand++] = e;
                else c_more = true;
            }
        };
        // The wave's list holds the candidates block after block (lane after lane
        // within a block): a solve round then meets one or two blocks, of one
        // degree, instead of the blocks of a few rays.
        // With MLP seeds every candidate has one network query (the ray's
        // midpoint in the element's box, and the element's block), stored at its
        // position in the list, where the seed kernel leaves its seed.
        const bool mlp = fp.seed_mode == IVR_SEED_MLP;
        u32 wrun = 0;
        auto block = [&](int pi, int nc0) __attribute__((always_inline)) {
            const u32 nb = (u32)(ncand - nc0);
            if (__ballot(nb > 0) == 0) return;
            const u32 incl = wave_incl_scan(nb, lane);
            const u32 total = __shfl(incl, 63);
            for (int k = nc0; k < ncand; ++k) cpos[k] = wrun + incl - nb + (u32)(k - nc0);
            wrun += total;
        };
        traverse(valid, hit, block);
        // the candidates for the solve pass
        u32 base = 0;
        if (lane == 0 && wrun) base = atomicAdd(&qs->n_cands, wrun);
        base = __shfl(base, 0);
        if (base + wrun > mq.c_cap) {   // the list is full: the solve pass traverses again
            c_more = ncand > 0 || c_more;
            ncand = 0;
        }
        const u32 excl = wave_incl_scan((u32)ncand, lane) - (u32)ncand;
        for (int k = 0; k < ncand; ++k) {
            const u32 pos = cpos[k];
            if (mlp) {
                const FaceElem &E = m.elems[cand[k]];
                float t0, t1;
                obb_hit(E, of, df, t0, t1);
                const float tm = 0.5f * (t0 + fminf(t1, t0 + 4.0f * fp.scale));
                mq.query[base + pos] = make_float4(of[0] + tm * df[0], of[1] + tm * df[1], of[2] + tm * df[2],
                                                   __int_as_float(E.patch));
                ++c_mlp;
            }
            mq.clist[base + pos] = make_uint2(cand[k] | ((u32)lane << kCandLaneShift), mlp ? base + pos : 0xFFFFFFFFu);
            mq.plist[base + excl + (u32)k] = pos;
        }
        // the wave's base and the lane's count; the top bit asks the solve pass for the rest
        mq.crange[g * 64u + (u32)lane] = make_uint2(base, (u32)ncand | (c_more ? 0x80000000u : 0u));
        if (fp.collect) {
            flush_counter(ctr, C_BOX_TESTS, c_box);
            flush_counter(ctr, C_MLP_QUERIES, c_mlp);
        }
        return;
    }
    if constexpr (MODE == 2) {
        // The wave's candidates (block after block from the first pass) are solved
        // 64 at a time whatever lane owns them; the roots go through LDS back to
        // the owning lanes, which find them by their positions in the list and
        // keep their fragment lists.
        __shared__ double s_dd[64 * 3];
        __shared__ RootRec<R> s_res[kFlat];
        __shared__ RootRec<R> s_x[kExtra];   // second roots of a pass and their owning lanes
        __shared__ u32 s_xo[kExtra];
        __shared__ u32 s_nx;
        const uint2 cr = mq.crange[g * 64u + (u32)lane];
        const u32 nrec = cr.y & 0x7FFFFFFFu;
        const u32 incl = wave_incl_scan(nrec, lane);
        const u32 total = __shfl(incl, 63);
        const u32 wbase = __builtin_amdgcn_readfirstlane(cr.x);
        const u32 *own = mq.plist + wbase + (incl - nrec);
#pragma unroll
        for (int q = 0; q < 3; ++q) s_dd[lane * 3 + q] = dd[q];
        __syncthreads();
        u32 kk = 0, mypos = nrec ? own[0] : 0xFFFFFFFFu;
        for (u32 b0 = 0; b0 < total; b0 += kFlat) {
            const u32 nb = min((u32)kFlat, total - b0);
            if (lane == 0) s_nx = 0;
            __syncthreads();
            for (u32 r = 0; r < nb; r += 64) {
                const u32 j = r + (u32)lane;
                if (j < nb) {
                    const uint2 c = mq.clist[wbase + b0 + j];
                    const u32 ol = c.x >> kCandLaneShift;
                    const double odd[3] = {s_dd[ol * 3], s_dd[ol * 3 + 1], s_dd[ol * 3 + 2]};
                    const float odf[3] = {float(odd[0]), float(odd[1]), float(odd[2])};
                    const FaceElem E = m.elems[c.x & kCandElemMask];
                    float ms[3] = {NAN, NAN, NAN};
                    if (c.y != 0xFFFFFFFFu) {
                        const float4 s = mq.seed[c.y];
                        ms[0] = s.x; ms[1] = s.y; ms[2] = s.z;
                    }
                    float T1 = -1.f;
                    ++c_newton;
                    for (int s = 0; s < 2; ++s) {   // a second search where the ray is nearly tangent
                        RootRec<R> out;
                        bool again;
                        face_root_any<R>(m, m.patches[E.patch], E, od, odd, of, odf, fp, ms, T1, out, again,
                                         c_iter, c_pol);
                        if (s == 0) {
                            s_res[j] = out;
                        } else if (out.info != 0xFFFFFFFFu) {   // to the pass's short list of second roots
                            const u32 x = atomicAdd(&s_nx, 1u);
                            if (x < (u32)kExtra) {
                                s_x[x] = out;
                                s_xo[x] = ol;
                            } else {
                                ++c_fovf;
                            }
                        }
                        if (!again) break;
                        T1 = float(out.t);
                    }
                }
            }
            __syncthreads();
            // the lane's own roots of this pass, in the order of its candidates
            while (mypos < b0 + nb) {
                add_root(s_res[mypos - b0]);
                mypos = ++kk < nrec ? own[kk] : 0xFFFFFFFFu;
            }
            const u32 nx = min(s_nx, (u32)kExtra);
            for (u32 i = 0; i < nx; ++i)
                if (s_xo[i] == (u32)lane) add_root(s_x[i]);
            __syncthreads();
        }
        // Rays with more candidates than were recorded traverse again and solve
        // the rest (box or element-centre seeds) with all lanes in step,
        // whenever a lane's list is full and at the end.
        const bool more = (cr.y >> 31) != 0;
        if (__ballot(more) != 0) {
            u32 seen = 0;
            auto hit_rest = [&](u32 e, bool he) __attribute__((always_inline)) {
                if (he && seen++ >= nrec) cand[ncand++] = e;
                if (__ballot(ncand == kCandCap) != 0) solve_candidates();
            };
            traverse(valid && more, hit_rest, no_block);
            solve_candidates();
        }
    }
    // 3. Algorithm "Blockwise depth-sorting": the nearest unused exit, then the
    //    nearest unused entry of the same block in front of it.  Depth order is
    //    (depth, order found); an entry counts as in front of an exit up to the
    //    depth tolerance of one crossing (an entry and exit at one point, as
    //    where a ray passes through an edge of the block, come from roots of
    //    different faces and may round to neighbouring FP32 depths).
    //    Sec. "Cutting and Near Clip Planes": segments are clipped to the kept
    //    interval [klo, khi] of the ray (beyond the near plane, on the kept side of
    //    the cutting plane); with a near plane an exit without an entry in front
    //    starts where the ray starts (entry index kRayStart), the near plane
    //    lying inside that block.  An end moved to a plane has no parameter point.
    R klo = -INFINITY, khi = INFINITY;
    if (fp.near_clip > 0.0)
        klo = R(fp.near_clip / (dd[0] * fp.fwd[0] + dd[1] * fp.fwd[1] + dd[2] * fp.fwd[2]));
    if (fp.cut) {
        const double sd = fp.cut_n[0] * dd[0] + fp.cut_n[1] * dd[1] + fp.cut_n[2] * dd[2];
        if (sd > 0.0) klo = fmax(klo, R(-fp.cut_s0 / sd));
        else if (sd < 0.0) khi = R(-fp.cut_s0 / sd);
        else if (fp.cut_s0 < 0.0) khi = -INFINITY;
    }
    auto t_in_of = [&](int q) __attribute__((always_inline)) -> R {
        return q == kRayStart ? klo : fmax(ft(q), klo);
    };
    unsigned char pin[kSegCap], pout[kSegCap];
    int npair = 0;
    u64 used = 0;
    const R teq = R(1e-6 * fp.scaled);
    for (;;) {
        int ib = -1;
        R tb = R(0);
        for (int q = 0; q < nfr; ++q) {
            const R tq = ft(q);
            if (!((used >> q) & 1ull) && !(fi(q) & 1u) && (ib < 0 || tq < tb)) {
                ib = q;
                tb = tq;
            }
        }
        if (ib < 0) break;
        used |= 1ull << ib;
        const u32 pb = fi(ib) >> 4;
        int ifr = -1;
        R tf = R(0);
        for (int q = 0; q < nfr; ++q) {
            const u32 iq = fi(q);
            const R tq = ft(q);
            if (!((used >> q) & 1ull) && (iq & 1u) && (iq >> 4) == pb && tq <= tb + teq && (ifr < 0 || tq < tf)) {
                ifr = q;
                tf = tq;
            }
        }
        if (ifr < 0) {
            if (!(fp.near_clip > 0.0)) {
                ++c_anom;
                continue;
            }
            ifr = kRayStart;
        } else {
            used |= 1ull << ifr;
        }
        const R t_in = t_in_of(ifr);
        if (!(fmin(tb, khi) > t_in)) continue;   // nothing of it is kept
        if (npair >= kSegCap) { ++c_sovf; continue; }
        // keep the pairs ordered by (kept) entry depth
        int q = npair++;
        while (q > 0 && t_in_of(pin[q - 1]) > t_in) {
            pin[q] = pin[q - 1];
            pout[q] = pout[q - 1];
            --q;
        }
        pin[q] = (unsigned char)ifr;
        pout[q] = (unsigned char)ib;
    }
    for (int q = 0; q < nfr; ++q) c_anom += !((used >> q) & 1ull);

    // 4. contiguous per-pixel ranges: wave prefix sum, one atomic per wave
    int nseg = npair;
    const u32 incl = wave_incl_scan((u32)nseg, lane);
    const u32 total = __shfl(incl, 63);
    u32 base = 0;
    if (lane == 63 && total) base = atomicAdd(&qs->seg_total, total);
    base = __shfl(base, 63);
    u32 first = base + incl - (u32)nseg;
    if (base + total > seg_cap) {  // capacity exhausted: drop this wave's segments
        // (their slots below the capacity are marked empty for the block sort)
        for (int k = 0; k < nseg; ++k)
            if (first + k < seg_cap) seg_kr[first + k] = make_uint2(0xFFFFFFFFu, 0u);
        c_sovf += nseg;
        nseg = 0;
        first = 0;
    }
    const R dr[3] = {R(dd[0]), R(dd[1]), R(dd[2])};
    for (int k = 0; k < nseg; ++k) {
        const int qi = pin[k], qo = pout[k];
        const u32 info_o = fi(qo);
        Seg<R> s;
        s.t_in = t_in_of(qi);
        s.t_out = fmin(ft(qo), khi);
        R pi_[3], po_[3];
        if (qi != kRayStart && ft(qi) >= klo) {
            face_point(fi(qi), fr[qi].a, fr[qi].b, pi_);
        } else {
            pi_[0] = pi_[1] = pi_[2] = R(NAN);   // entry on a plane: found by the integrator
        }
        face_point(info_o, fr[qo].a, fr[qo].b, po_);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            s.p_in[q] = pi_[q];
            s.p_out[q] = po_[q];
        }
        if (ft(qo) <= khi) {
            const R det_out = rho_ds_any<R>(m, m.patches[info_o >> 4], po_, dr, s.rho_out, s.drho_out);
            // singular J at the exit (a degenerate boundary): no slope; the
            // integrator then stops short of the exit, Eq. (degeneracyfix)
            if (!(fabs(det_out) >= (sizeof(R) == 4 ? R(fp.det_sing) : R(fp.det_singd))))
                s.drho_out = R(NAN);
        } else {
            // exit on the cutting plane: no parameter point, the integrator samples it
            s.p_out[0] = R(NAN);
            s.rho_out = R(0);
            s.drho_out = R(0);
        }
        s.pixel = pixel;
        s.patch = (info_o >> 4) | ((u32)v << kViewShift);
        segs[first + k] = s;
    }
    // 5. the rank of every segment among the segments of its block (one atomic per
    //    block and wave): the integrator takes the segments block by block
    {
        u32 ranked = 0;   // bit k: segment k has its rank
        for (;;) {
            int kk = -1;
            for (int k = 0; k < nseg; ++k)
                if (!((ranked >> k) & 1u)) { kk = k; break; }
            const int myp = kk >= 0 ? (int)(fi(pout[kk]) >> 4) : -1;
            const u64 any = __ballot(myp >= 0);
            if (any == 0) break;
            const int leader = __ffsll((long long)any) - 1;
            const int p = __shfl(myp, leader);
            u32 cnt = 0;
            for (int k = 0; k < nseg; ++k) cnt += (!((ranked >> k) & 1u) && (int)(fi(pout[k]) >> 4) == p) ? 1u : 0u;
            const u32 ci = wave_incl_scan(cnt, lane);
            const u32 ctot = __shfl(ci, 63);
            u32 b = 0;
            if (lane == leader) b = atomicAdd(&pcount[p], ctot);
            b = __shfl(b, leader);
            u32 r = b + ci - cnt;
            for (int k = 0; k < nseg; ++k)
                if (!((ranked >> k) & 1u) && (int)(fi(pout[k]) >> 4) == p) {
                    seg_kr[first + k] = make_uint2((u32)p, r++);
                    ranked |= 1u << k;
                }
        }
    }
    if (valid) {
        pixseg[vr.pix_begin + pixel] = make_uint2(first, (u32)nseg);
        if (vr.depth) vr.depth[pixel] = nseg ? float(t_in_of(pin[0])) : INFINITY;
        // the pixel's flags start here; the integrator ORs in its segments' flags
        if (vr.flags)
            vr.flags[pixel] = (c_anom ? (u32)IVR_FLAG_ANOMALY : 0u) | (c_fovf ? (u32)IVR_FLAG_FRAGMENT_OVERFLOW : 0u) |
                              (c_sovf ? (u32)IVR_FLAG_SEGMENT_OVERFLOW : 0u);
    }
    if (fp.collect) {
        flush_counter(ctr, C_RAYS, valid ? 1 : 0);
        flush_counter(ctr, C_SEGMENTS, nseg);
        flush_counter(ctr, C_FRAGMENTS, nfr);
        flush_counter(ctr, C_ANOMALIES, c_anom);
        flush_counter(ctr, C_FRAG_OVF, c_fovf);
        flush_counter(ctr, C_SEG_OVF, c_sovf);
        flush_counter(ctr, C_BOX_TESTS, c_box);
        flush_counter(ctr, C_FACE_NEWTON, c_newton);
        flush_counter(ctr, C_FACE_NEWTON_ITER, c_iter);
        flush_counter(ctr, C_FP64_POLISH, c_pol);
        flush_counter(ctr, C_MLP_QUERIES, c_mlp);
    }
}

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
__constant__ RkTableau kRkFamily[6] = {
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

// Network seeds of a frame's candidates: the recorded queries, 64 rows per wave
// and call in list order (rows of different blocks share a call), the seed
// written where the query is.  Rows of waves whose lists did not fit carry no
// query; a block index outside the model marks them.
__global__ __launch_bounds__(64) void k_mlp_seeds(const uint16_t *wb, const float *norm, int npatch,
                                                  const QueueState *qs, CandLists mq) {
    __shared__ uint16_t sA[64 * 72];
    __shared__ float sZ[64 * 65];
    __shared__ int sQ[64];
    const int lane = threadIdx.x;
    const u32 nq = min(qs->n_cands, mq.c_cap);
    for (u32 r0 = blockIdx.x * 64u; r0 < nq; r0 += gridDim.x * 64u) {
        const u32 row = r0 + (u32)lane;
        float x[3] = {0.f, 0.f, 0.f}, p[3];
        int q = 0;
        if (row < nq) {
            const float4 v = mq.query[row];
            x[0] = v.x; x[1] = v.y; x[2] = v.z;
            q = __float_as_int(v.w);
        }
        const bool ok = row < nq && q >= 0 && q < npatch && isfinite(x[0] + x[1] + x[2]);
        mlp_infer_rows(wb, norm, q, ok, x, p, sA, sZ, sQ);
        if (ok) mq.seed[row] = make_float4(p[0], p[1], p[2], 0.f);
    }
}

// Segments are taken block by block.  The fragment kernel gave every segment its
// rank among the segments of its block; one workgroup scans the block counts in
// class order (bases, cursors), and the scatter writes the block-sorted order.
__global__ __launch_bounds__(1024) void k_block_scan(const u32 *pperm, int nperm, const u32 *pcount,
                                                     u32 *pbase, u32 *pcur) {
    __shared__ u32 part[1024];
    __shared__ u32 run;
    const int t = threadIdx.x;
    if (t == 0) run = 0;
    __syncthreads();
    for (int q0 = 0; q0 < nperm; q0 += 1024) {
        const int q = q0 + t;
        const u32 v = q < nperm ? pcount[pperm[q]] : 0u;
        part[t] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan (Hillis-Steele)
            const u32 x = t >= off ? part[t - off] : 0u;
            __syncthreads();
            part[t] += x;
            __syncthreads();
        }
        const u32 base = run + part[t] - v;
        if (q < nperm) {
            pbase[pperm[q]] = base;
            pcur[pperm[q]] = base;
        }
        __syncthreads();
        if (t == 1023) run += part[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_block_scatter(const QueueState *qs, u32 seg_cap, const uint2 *seg_kr,
                                                       const u32 *pbase, u32 *order) {
    const u32 n = min(qs->seg_total, seg_cap);
    for (u32 i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        const uint2 kr = seg_kr[i];
        if (kr.x != 0xFFFFFFFFu) order[pbase[kr.x] + kr.y] = i;
    }
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
// METHOD kOde: the ray preimage ODE by adaptive RKF45 (Sec. "ODE Based
// Algorithm"); kRootFinding: every sample's preimage by Newton (Sec. "Root
// Finding Based Algorithm"), seeded from the previous sample along J^-1 d.
// kFixedRK: a fixed-step explicit method of the family above; kImplicitEuler:
// implicit Euler with the exact Jacobian of its Newton (Eq. (JacG)).
constexpr int kOde = 0, kRootFinding = 1, kFixedRK = 2, kImplicitEuler = 3;

template <int P, bool RAT, typename R, bool LDS, int METHOD>
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
                    s = R(0);
                    h = L < hmax ? L : hmax;
                    rho_out = sg.rho_out;
                    m_out = sg.drho_out;
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
        const R det1 = eval_W<P, RAT, 2, R, LDS, METHOD == kRootFinding>(pv, ar, p, gin, d, cperp, dthr, k1,
                                                                         rho_cur, grho, c_fp64, shrinking, res2,
                                                                         xw, wt);
        ++c_w;
        const R m_cur = dot3(grho, k1);
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
                if (res2 <= tolx * tolx || newton_it >= 12 || !isfinite(k1[0] + k1[1] + k1[2])) {
                    // the sample: rho and d rho/ds = grad rho . J^-1 d at the preimage
                    // (where Newton stopped if it did not converge: counted, flagged)
                    if (!(res2 <= tolx * tolx)) {
                        fl |= IVR_FLAG_RESTART_FAIL;
                        count_rare(C_RESTART_FAIL);
                    }
                    shrink = 0;
                    const R m_t = dot3(grho, wt);
                    composite(fp, views[vid].fp, vls[vid], rho_prev, m_prev, rho_cur, m_t, h_prev, C, A, c_sub);
                    ++c_samp;
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
    }
}

// The view that owns batch pixel g (views sorted by pix_begin).
__device__ __forceinline__ int view_of_pixel(const ViewRec *views, int n_views, u32 g) {
    int lo = 0, hi = n_views;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (views[mid].pix_begin <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_merge(const ViewRec *views, int n_views, u32 n_pixels,
                                               const uint2 *pixseg, const unsigned char *segs, u32 seg_bytes,
                                               const QueueState *qs, u32 *totals) {
    const u32 g = blockIdx.x * 256u + threadIdx.x;
    // the frame's totals (segments requested, candidates recorded, pixels) to
    // host memory: they size the next frame's buffers without a readback call
    if (g == 0 && totals) {
        totals[0] = qs->seg_total;
        totals[1] = qs->n_cands;
        totals[2] = n_pixels;
    }
    if (g >= n_pixels) return;
    const ViewRec &vr = views[view_of_pixel(views, n_views, g)];
    const float early = views[0].fp.early_term;
    const uint2 ps = pixseg[g];
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, A = 0.f;
    for (u32 k = 0; k < ps.y; ++k) {
        if (A >= 1.0f - early) break;
        const float4 r = *reinterpret_cast<const float4 *>(segs + (size_t)(ps.x + k) * seg_bytes);
        const float w = 1.0f - A;
        C0 += w * r.x;
        C1 += w * r.y;
        C2 += w * r.z;
        A += w * r.w;
    }
    reinterpret_cast<float4 *>(vr.rgba)[g - vr.pix_begin] = make_float4(C0, C1, C2, A);
}

// Clears the queue bookkeeping and (collect) the counters: a kernel rather than a
// memset so that the whole render can be captured in a graph.
__global__ void k_clear(QueueState *qs, u64 *ctr, int collect, u32 *pcount, int npatch) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t *q = reinterpret_cast<uint32_t *>(qs);
    if (t < (int)(sizeof(QueueState) / 4)) q[t] = 0u;
    if (collect && t < C_COUNT) ctr[t] = 0ull;
    for (int i = t; i < npatch; i += gridDim.x * blockDim.x) pcount[i] = 0u;
}

// ------------------------------------------------------------------ launchers

template <typename R>
static hipError_t launch_fragments_t(const Model &m, const ViewRec *views, int n_views, uint32_t n_tiles,
                                     const LaunchCfg &lc, bool mlp, void *segs, uint32_t seg_cap,
                                     uint2 *seg_kr, uint32_t *pcount, QueueState *qs, uint2 *pixseg,
                                     const CandLists &mq, unsigned long long *ctr, int n_cu,
                                     hipStream_t st) {
    hipLaunchKernelGGL((k_fragments<R, 1>), dim3(n_tiles), dim3(64), 0, st, m, views, n_views, n_tiles, lc,
                       (Seg<R> *)segs, seg_cap, seg_kr, pcount, qs, pixseg, mq, ctr);
    if (mlp) hipLaunchKernelGGL(k_mlp_seeds, dim3(n_cu * 8), dim3(64), 0, st, m.mlp_wb, m.mlp_norm, m.npatch, qs, mq);
    hipLaunchKernelGGL((k_fragments<R, 2>), dim3(n_tiles), dim3(64), 0, st, m, views, n_views, n_tiles, lc,
                       (Seg<R> *)segs, seg_cap, seg_kr, pcount, qs, pixseg, mq, ctr);
    return hipGetLastError();
}

hipError_t launch_fragments(bool fp64, bool mlp, const Model &m, const ViewRec *views, int n_views,
                            uint32_t n_tiles, const LaunchCfg &lc, void *segs, uint32_t seg_cap,
                            uint2 *seg_kr, uint32_t *pcount, QueueState *qs, uint2 *pixseg,
                            const CandLists &mq, unsigned long long *ctr, int n_cu, hipStream_t st) {
    return fp64 ? launch_fragments_t<double>(m, views, n_views, n_tiles, lc, mlp, segs, seg_cap, seg_kr,
                                             pcount, qs, pixseg, mq, ctr, n_cu, st)
                : launch_fragments_t<float>(m, views, n_views, n_tiles, lc, mlp, segs, seg_cap, seg_kr,
                                            pcount, qs, pixseg, mq, ctr, n_cu, st);
}

hipError_t launch_block_sort(const QueueState *qs, uint32_t seg_cap, const uint2 *seg_kr,
                             const uint32_t *pperm, int nperm, const uint32_t *pcount, uint32_t *pbase,
                             uint32_t *pcur, uint32_t *order, int n_cu, hipStream_t st) {
    hipLaunchKernelGGL(k_block_scan, dim3(1), dim3(1024), 0, st, pperm, nperm, pcount, pbase, pcur);
    hipLaunchKernelGGL(k_block_scatter, dim3(n_cu * 4), dim3(256), 0, st, qs, seg_cap, seg_kr, pbase, order);
    return hipGetLastError();
}

// LDS budget of the staged block per integrator workgroup.
constexpr size_t kLdsBlockBytes = 48 * 1024;

template <int P, bool RAT, typename R, bool LDS, int METHOD>
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
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_integrate<P, RAT, R, LDS, METHOD>, block, lds) !=
            hipSuccess || nb < 1)
        nb = 1;
    if (lc.int_waves_cu > 0) nb = std::min(nb, std::max(1, lc.int_waves_cu / (block / 64)));
    hipLaunchKernelGGL((k_integrate<P, RAT, R, LDS, METHOD>), dim3(n_cu * nb), dim3(block), lds, st, m, views,
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

hipError_t launch_integrate(bool fp64, int method, int klass, const Model &m, const ViewRec *views, int n_views,
                            void *segs, const IntegrateArgs &a,
                            unsigned long long *ctr, int n_cu, const LaunchCfg &lc, hipStream_t st) {
    switch (klass) {
    case 0: return launch_integrate_pr<1, false>(fp64, method, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    case 1: return launch_integrate_pr<1, true>(fp64, method, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    case 2: return launch_integrate_pr<2, false>(fp64, method, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    case 3: return launch_integrate_pr<2, true>(fp64, method, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    case 4: return launch_integrate_pr<3, false>(fp64, method, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    case 5: return launch_integrate_pr<3, true>(fp64, method, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_merge(const ViewRec *views, int n_views, uint32_t n_pixels, const uint2 *pixseg,
                        const void *segs, bool fp64, const QueueState *qs, uint32_t *totals, hipStream_t st) {
    hipLaunchKernelGGL(k_merge, dim3((n_pixels + 255) / 256), dim3(256), 0, st, views, n_views, n_pixels,
                       pixseg, (const unsigned char *)segs, (u32)(fp64 ? sizeof(Seg<double>) : sizeof(Seg<float>)), qs,
                       totals);
    return hipGetLastError();
}

hipError_t launch_clear(QueueState *qs, unsigned long long *ctr, bool collect, uint32_t *pcount, int npatch,
                        hipStream_t st) {
    const int blocks = std::max(1, std::min(64, (npatch + 255) / 256));
    hipLaunchKernelGGL(k_clear, dim3(blocks), dim3(256), 0, st, qs, ctr, collect ? 1 : 0, pcount, npatch);
    return hipGetLastError();
}

}  // namespace ivr
