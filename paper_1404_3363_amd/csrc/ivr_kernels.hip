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
#include "ivr_device.h"
#include "ivr_integrate.h"
#include "ivr_mlp_dev.h"
#include "ivr_spline.h"

namespace ivr {

using u32 = uint32_t;
using u64 = unsigned long long;

constexpr int kFlat = 256;    // candidates solved per pass of the flattened solve
constexpr int kRayStart = 255;  // entry index of a segment that starts on the near plane
constexpr int kFragLds = 16;  // crossings per ray kept in LDS (the rest in scratch)
constexpr int kExtra = 64;    // second roots of one element per pass of the flattened solve

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

// A direction component as a divisor: zero (and anything below 1e-30 in size)
// becomes +-1e-30, so that a ray parallel to a slab gets a finite, enormous
// interval (no hit from outside the slab, no limit inside it) rather than a NaN
// that the min/max would skip.
__device__ __forceinline__ float safe_divisor(float x) { return copysignf(fmaxf(fabsf(x), 1e-30f), x); }

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
        const float inv = __builtin_amdgcn_rcpf(safe_divisor(pd));
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
        const float inv = __builtin_amdgcn_rcpf(safe_divisor(pd));
        const float mid = -po * inv, ai = fabsf(inv);
        tmin = fmaxf(tmin, fmaf(-E.ext[r], ai, mid));
        tmax = fminf(tmax, fmaf(E.ext[r], ai, mid));
    }
    return tmin <= tmax;
}

// The view frustum of a pixel tile: the four planes through the eye that
// contain the rays of its corner pixels, normals pointing inwards.  Every ray of
// the tile lies inside (the rays' directions are affine in the pixel
// coordinates), so a box wholly outside one plane is missed by all of them.
struct TileFrustum {
    float n[4][3];
    float e[3];
};

// The plane through the eye that holds directions u and v, its normal turned so
// that its product with the camera axis a has the sign sg.
__device__ __forceinline__ void frustum_plane(const double (&u)[3], const double (&v)[3], double a0, double a1,
                                              double a2, double sg, float (&n)[3]) {
    const double x = u[1] * v[2] - u[2] * v[1], y = u[2] * v[0] - u[0] * v[2], z = u[0] * v[1] - u[1] * v[0];
    const double s = (x * a0 + y * a1 + z * a2) * sg < 0.0 ? -1.0 : 1.0;
    n[0] = float(s * x);
    n[1] = float(s * y);
    n[2] = float(s * z);
}

// Planes left, right, top, bottom: the pixel column grows along the camera's
// right axis, the row index against its up axis.  A tile one pixel wide (or
// high) has no top and bottom (left and right) planes: their two rays are one,
// and the rounding of their cross product (contracted to FMAs) would leave a
// normal of random direction; those normals are zero, which culls nothing.
__device__ __forceinline__ TileFrustum tile_frustum(const FrameParams &fp, int x0, int y0, int x1, int y1) {
    double c00[3], c10[3], c01[3], c11[3];
    ray_dir(fp, x0, y0, c00);
    ray_dir(fp, x1, y0, c10);
    ray_dir(fp, x0, y1, c01);
    ray_dir(fp, x1, y1, c11);
    const double r0 = fp.right[0], r1 = fp.right[1], r2 = fp.right[2];
    const double u0 = fp.up[0], u1 = fp.up[1], u2 = fp.up[2];
    TileFrustum F;
    frustum_plane(c00, c01, r0, r1, r2, 1.0, F.n[0]);
    frustum_plane(c10, c11, r0, r1, r2, -1.0, F.n[1]);
    frustum_plane(c00, c10, u0, u1, u2, -1.0, F.n[2]);
    frustum_plane(c01, c11, u0, u1, u2, 1.0, F.n[3]);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (y0 == y1) F.n[0][q] = F.n[1][q] = 0.f;
        if (x0 == x1) F.n[2][q] = F.n[3][q] = 0.f;
    }
    F.e[0] = float(fp.eye[0]);
    F.e[1] = float(fp.eye[1]);
    F.e[2] = float(fp.eye[2]);
    return F;
}

// True when the axis-aligned box [lo, hi] lies wholly outside a plane of F, by
// more than 1e-5 of the size of the terms (FP32 rounding stays far below).
__device__ __forceinline__ bool frustum_misses_box(const TileFrustum &F, const float *lo, const float *hi) {
    bool out = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float mx = 0.f, sz = 0.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float a = lo[q] - F.e[q], b = hi[q] - F.e[q];
            mx += fmaxf(F.n[i][q] * a, F.n[i][q] * b);
            sz += fabsf(F.n[i][q]) * fmaxf(fabsf(a), fabsf(b));
        }
        out |= mx < -1e-5f * sz;
    }
    return out;
}

// The same for an oriented box (centre c, unit axes ax, half extents ext).
template <typename Box3>
__device__ __forceinline__ bool frustum_misses_obb(const TileFrustum &F, const Box3 &B) {
    bool out = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float mx = 0.f, sz = 0.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float a = B.c[q] - F.e[q];
            mx += F.n[i][q] * a;
            sz += fabsf(F.n[i][q] * a);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float r = B.ext[k] * fabsf(F.n[i][0] * B.ax[k][0] + F.n[i][1] * B.ax[k][1] + F.n[i][2] * B.ax[k][2]);
            mx += r;
            sz += r;
        }
        out |= mx < -1e-5f * sz;
    }
    return out;
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
        //   An FP64 Newton root stopped at the refinement's own tolerance already.
        double A = a, B = b, T = t, S2[3], F2[3], Sa2[3], Sb2[3];
        bool ok = sizeof(RN) == 8;
        for (int k = 0; k < 4 && !ok; ++k) {
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
        inv[q] = 1.0f / safe_divisor(df[q]);
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
    // f(q, t, info) for every crossing in the order found: the LDS part and the
    // scratch part in loops of their own, so that every load names its memory
    // (one loop over both would load through flat addresses)
    auto each_frag = [&](auto &&f) __attribute__((always_inline)) {
        const int nl = min(nfr, kFragLds);
        for (int q = 0; q < nl; ++q) f(q, s_ft[q * 64 + lane], s_fi[q * 64 + lane]);
        for (int q = kFragLds; q < nfr; ++q) f(q, fr[q].t, fr[q].info);
    };
    // a crossing of the same block and facing within tol of depth t is there already
    auto known = [&](u32 info, R t, R tol) __attribute__((always_inline)) -> bool {
        bool dup = false;
        each_frag([&](int, R tq, u32 iq) __attribute__((always_inline)) {
            dup |= ((iq ^ info) & ~0xEu) == 0u && fabs(tq - t) <= tol;
        });
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
    // The blocks, face tiles and elements that no ray of the pixel tile can hit
    // are culled first, 64 at a time (a lane a box) against the tile's frustum:
    // what remains is tested ray by ray in the same order, so the candidates and
    // their order are those of testing every box.
    auto traverse = [&](bool act, auto &&on_hit, auto &&after_block) __attribute__((always_inline)) {
        const TileFrustum fru = tile_frustum(fp, (int)(tl % vr.tiles_x) * lc.tile_w, (int)(tl / vr.tiles_x) * th,
                                             min((int)(tl % vr.tiles_x + 1) * lc.tile_w, fp.width) - 1,
                                             min((int)(tl / vr.tiles_x + 1) * th, fp.height) - 1);
        for (int pb0 = vr.patch_begin; pb0 < vr.patch_end; pb0 += 64) {
            const int pj = pb0 + lane;
            const bool pnear = pj < vr.patch_end && !frustum_misses_box(fru, m.patches[pj].box, m.patches[pj].box + 3);
            for (u64 bm = __ballot(pnear); bm != 0ull; bm &= bm - 1ull) {
                const int pi = pb0 + __ffsll((long long)bm) - 1;
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
                    for (int t0 = Pd.tile_off[f]; t0 < Pd.tile_off[f + 1]; t0 += 64) {
                        const int tj = t0 + lane;
                        const bool tnear = tj < Pd.tile_off[f + 1] && !frustum_misses_obb(fru, m.tiles[tj]);
                        for (u64 tm = __ballot(tnear); tm != 0ull; tm &= tm - 1ull) {
                            const int ti = t0 + __ffsll((long long)tm) - 1;
                            const FaceTile &T = m.tiles[ti];
                            c_box += hf;
                            const bool ht = hf && obb_hit(T, of, df);
                            if (__ballot(ht) == 0) continue;
                            // the tile's elements (at most kTile^2) against the frustum, one a lane
                            const int e0 = T.elem_begin;
                            const u64 emask =
                                __ballot(lane < T.elem_end - e0 && !frustum_misses_obb(fru, m.elems[e0 + lane]));
                            if (emask == 0ull) continue;
                            const bool split = T.sub_end > T.sub_begin;
                            for (int si = split ? T.sub_begin : ti; si < (split ? T.sub_end : ti + 1); ++si) {
                                const FaceTile &S = m.tiles[si];
                                const u64 smask = (emask >> (S.elem_begin - e0)) &
                                                  ((1ull << (S.elem_end - S.elem_begin)) - 1ull);
                                if (smask == 0ull) continue;
                                bool hs = ht;
                                if (split) {
                                    c_box += ht;
                                    hs = ht && obb_hit(S, of, df);
                                    if (__ballot(hs) == 0) continue;
                                }
                                for (u64 em = smask; em != 0ull; em &= em - 1ull) {
                                    const int e = S.elem_begin + __ffsll((long long)em) - 1;
                                    c_box += hs;
                                    on_hit((u32)e, hs && obb_hit(m.elems[e], of, df));
                                }
                            }
                        }
                    }
                }
                after_block(pi, nc0);
            }
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
            // the wave's rows that still fall inside the list carry no query: a
            // block index outside the model tells the seed kernel to skip them
            if (mlp) {
                const u32 end = min(base + wrun, mq.c_cap);
                for (u32 r = base + (u32)lane; r < end; r += 64u)
                    mq.query[r] = make_float4(0.f, 0.f, 0.f, __int_as_float(m.npatch));
            }
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
    unsigned char pin[kSegCap], pout[kSegCap];
    R ptin[kSegCap];   // the pairs' kept entry depths
    u32 pblk[kSegCap]; // and blocks
    int npair = 0;
    u64 used = 0;
    const R teq = R(1e-6 * fp.scaled);
    for (;;) {
        int ib = -1;
        R tb = R(0);
        u32 pb = 0;
        each_frag([&](int q, R tq, u32 iq) __attribute__((always_inline)) {
            if (!((used >> q) & 1ull) && !(iq & 1u) && (ib < 0 || tq < tb)) {
                ib = q;
                tb = tq;
                pb = iq >> 4;
            }
        });
        if (ib < 0) break;
        used |= 1ull << ib;
        int ifr = -1;
        R tf = R(0);
        each_frag([&](int q, R tq, u32 iq) __attribute__((always_inline)) {
            if (!((used >> q) & 1ull) && (iq & 1u) && (iq >> 4) == pb && tq <= tb + teq && (ifr < 0 || tq < tf)) {
                ifr = q;
                tf = tq;
            }
        });
        R t_in = klo;
        if (ifr < 0) {
            if (!(fp.near_clip > 0.0)) {
                ++c_anom;
                continue;
            }
            ifr = kRayStart;
        } else {
            used |= 1ull << ifr;
            t_in = fmax(tf, klo);
        }
        if (!(fmin(tb, khi) > t_in)) continue;   // nothing of it is kept
        if (npair >= kSegCap) { ++c_sovf; continue; }
        // keep the pairs ordered by (kept) entry depth
        int q = npair++;
        while (q > 0 && ptin[q - 1] > t_in) {
            pin[q] = pin[q - 1];
            pout[q] = pout[q - 1];
            ptin[q] = ptin[q - 1];
            pblk[q] = pblk[q - 1];
            --q;
        }
        pin[q] = (unsigned char)ifr;
        pout[q] = (unsigned char)ib;
        ptin[q] = t_in;
        pblk[q] = pb;
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
        s.t_in = ptin[k];
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
            const int myp = kk >= 0 ? (int)pblk[kk] : -1;
            const u64 any = __ballot(myp >= 0);
            if (any == 0) break;
            const int leader = __ffsll((long long)any) - 1;
            const int p = __shfl(myp, leader);
            u32 cnt = 0;
            for (int k = 0; k < nseg; ++k) cnt += (!((ranked >> k) & 1u) && (int)pblk[k] == p) ? 1u : 0u;
            const u32 ci = wave_incl_scan(cnt, lane);
            const u32 ctot = __shfl(ci, 63);
            u32 b = 0;
            if (lane == leader) b = atomicAdd(&pcount[p], ctot);
            b = __shfl(b, leader);
            u32 r = b + ci - cnt;
            for (int k = 0; k < nseg; ++k)
                if (!((ranked >> k) & 1u) && (int)pblk[k] == p) {
                    seg_kr[first + k] = make_uint2((u32)p, r++);
                    ranked |= 1u << k;
                }
        }
    }
    if (valid) {
        pixseg[vr.pix_begin + pixel] = make_uint2(first, (u32)nseg);
        if (vr.depth) vr.depth[pixel] = nseg ? float(ptin[0]) : INFINITY;
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

hipError_t launch_integrate(bool fp64, int method, int field, bool diag, int klass, const Model &m,
                            const ViewRec *views, int n_views, void *segs, const IntegrateArgs &a,
                            unsigned long long *ctr, int n_cu, const LaunchCfg &lc, hipStream_t st) {
    if (field != IVR_FIELD_SCALAR || diag)
        return launch_integrate_field(fp64, method, field, diag, klass, m, views, n_views, segs, a, ctr, n_cu, lc,
                                      st);
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

// ---------------------------------------------------------------- image comparison
// CIEDE2000 colour difference (CIE 142-2001) of two premultiplied RGBA images
// composited over a background, read as sRGB (IEC 61966-2-1), in FP64: the
// measure the paper compares renders with (1 just noticeable, 5 accepted).
__device__ __forceinline__ void srgb_lab(const float4 px, const double (&bg)[3], double (&lab)[3]) {
    const double c[3] = {px.x + (1.0 - px.w) * bg[0], px.y + (1.0 - px.w) * bg[1], px.z + (1.0 - px.w) * bg[2]};
    double lin[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = fmin(1.0, fmax(0.0, c[k]));
        lin[k] = v <= 0.04045 ? v / 12.92 : pow((v + 0.055) / 1.055, 2.4);
    }
    // linear sRGB -> XYZ (D65), relative to the white the same matrix gives (1, 1, 1)
    const double X = (0.4124 * lin[0] + 0.3576 * lin[1] + 0.1805 * lin[2]) / (0.4124 + 0.3576 + 0.1805);
    const double Y = (0.2126 * lin[0] + 0.7152 * lin[1] + 0.0722 * lin[2]);
    const double Z = (0.0193 * lin[0] + 0.1192 * lin[1] + 0.9505 * lin[2]) / (0.0193 + 0.1192 + 0.9505);
    const double e = 216.0 / 24389.0, kf = 24389.0 / 27.0;   // (6/29)^3, (29/3)^3
    auto f = [&](double t) { return t > e ? cbrt(t) : (kf * t + 16.0) / 116.0; };
    const double fx = f(X), fy = f(Y), fz = f(Z);
    lab[0] = 116.0 * fy - 16.0;
    lab[1] = 500.0 * (fx - fy);
    lab[2] = 200.0 * (fy - fz);
}

__device__ double ciede2000(const double (&p)[3], const double (&q)[3]) {
    constexpr double kDeg = 3.14159265358979323846 / 180.0;
    const double c25 = 6103515625.0;   // 25^7
    const double cm = 0.5 * (hypot(p[1], p[2]) + hypot(q[1], q[2]));
    const double cm7 = pow(cm, 7.0);
    const double g = 0.5 * (1.0 - sqrt(cm7 / (cm7 + c25)));
    const double ap = (1.0 + g) * p[1], aq = (1.0 + g) * q[1];
    const double cp = hypot(ap, p[2]), cq = hypot(aq, q[2]);
    double hp = (ap == 0.0 && p[2] == 0.0) ? 0.0 : atan2(p[2], ap) / kDeg;
    double hq = (aq == 0.0 && q[2] == 0.0) ? 0.0 : atan2(q[2], aq) / kDeg;
    if (hp < 0.0) hp += 360.0;
    if (hq < 0.0) hq += 360.0;
    const bool achrom = cp * cq == 0.0;
    double dh = hq - hp;
    if (dh > 180.0) dh -= 360.0;
    else if (dh < -180.0) dh += 360.0;
    if (achrom) dh = 0.0;
    const double dL = q[0] - p[0], dC = cq - cp;
    const double dH = 2.0 * sqrt(cp * cq) * sin(0.5 * dh * kDeg);
    const double lm = 0.5 * (p[0] + q[0]), cpm = 0.5 * (cp + cq);
    double hm = hp + hq;
    if (!achrom) {
        if (fabs(hp - hq) <= 180.0) hm *= 0.5;
        else hm = hm < 360.0 ? 0.5 * (hm + 360.0) : 0.5 * (hm - 360.0);
    }
    const double t = 1.0 - 0.17 * cos((hm - 30.0) * kDeg) + 0.24 * cos(2.0 * hm * kDeg) +
                     0.32 * cos((3.0 * hm + 6.0) * kDeg) - 0.20 * cos((4.0 * hm - 63.0) * kDeg);
    const double dth = 30.0 * exp(-((hm - 275.0) / 25.0) * ((hm - 275.0) / 25.0));
    const double cpm7 = pow(cpm, 7.0);
    const double rc = 2.0 * sqrt(cpm7 / (cpm7 + c25));
    const double l50 = (lm - 50.0) * (lm - 50.0);
    const double sl = 1.0 + 0.015 * l50 / sqrt(20.0 + l50), sc = 1.0 + 0.045 * cpm, sh = 1.0 + 0.015 * cpm * t;
    const double rt = -sin(2.0 * dth * kDeg) * rc;
    const double a = dL / sl, b = dC / sc, c = dH / sh;
    return sqrt(a * a + b * b + c * c + rt * b * c);
}

// Per pixel difference (optional) and the summary: largest (as float bits),
// sum, and the count above `threshold`.
__global__ __launch_bounds__(256) void k_delta_e(const float4 *a, const float4 *b, u64 n, double bg0, double bg1,
                                                 double bg2, double threshold, float *out, DeltaESum *sum) {
    __shared__ double s_sum[256];
    __shared__ unsigned s_max[256];
    __shared__ unsigned long long s_cnt[256];
    const double bg[3] = {bg0, bg1, bg2};
    double acc = 0.0;
    unsigned mx = 0;
    unsigned long long cnt = 0;
    for (u64 i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (u64)gridDim.x * 256ull) {
        double la[3], lb[3];
        srgb_lab(a[i], bg, la);
        srgb_lab(b[i], bg, lb);
        const double de = ciede2000(la, lb);
        if (out) out[i] = (float)de;
        acc += de;
        mx = max(mx, __float_as_uint((float)de));
        cnt += de > threshold ? 1ull : 0ull;
    }
    s_sum[threadIdx.x] = acc;
    s_max[threadIdx.x] = mx;
    s_cnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s_sum[threadIdx.x] += s_sum[threadIdx.x + off];
            s_max[threadIdx.x] = max(s_max[threadIdx.x], s_max[threadIdx.x + off]);
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && sum) {
        atomicAdd(&sum->sum, s_sum[0]);
        atomicMax(&sum->max_bits, s_max[0]);
        atomicAdd(&sum->over, s_cnt[0]);
    }
}

hipError_t launch_delta_e(const float *a, const float *b, uint64_t n, const double (&bg)[3], double threshold,
                          float *out, DeltaESum *sum, int n_cu, hipStream_t st) {
    const uint64_t want = (n + 255) / 256;
    const unsigned blocks = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)n_cu * 8));
    hipLaunchKernelGGL(k_delta_e, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const float4 *>(a),
                       reinterpret_cast<const float4 *>(b), (u64)n, bg[0], bg[1], bg[2], threshold, out, sum);
    return hipGetLastError();
}

// The views' pixel-accuracy records start at zero (no samples: Delta P 0).
__global__ __launch_bounds__(256) void k_dp_clear(const ViewRec *views, int n_views, u32 n_pixels) {
    const u32 g = blockIdx.x * 256u + threadIdx.x;
    if (g >= n_pixels) return;
    const int v = view_of_pixel(views, n_views, g);
    float *dp = views[v].dp;
    if (dp) dp[g - views[v].pix_begin] = 0.f;
}

hipError_t launch_dp_clear(const ViewRec *views, int n_views, uint32_t n_pixels, hipStream_t st) {
    hipLaunchKernelGGL(k_dp_clear, dim3((n_pixels + 255) / 256), dim3(256), 0, st, views, n_views, n_pixels);
    return hipGetLastError();
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
