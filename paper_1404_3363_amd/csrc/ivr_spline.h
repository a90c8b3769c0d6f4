// Device spline library for gfx950: span search, B-spline basis with first
// derivatives, sum-factorised tensor-product contraction (volume and face),
// the pulled-back ray field W and the transfer function.
//
// Eq. (Bspline): S(u,v,w) = sum_i sum_j sum_k K_i(u) L_j(v) M_k(w) C_ijk.  Only the
// (p+1)^3 basis functions that are non-zero on the knot span of the point are
// evaluated (triangular scheme over the 2p knots around the span), and the
// contraction runs along u, then v, then w, producing phi and its three partial
// derivatives together (Sec. "Root Finding Based Algorithm": the Jacobian reuses
// the evaluation of phi).  NURBS run the same contraction on homogeneous points
// and finish with the quotient rule.
#pragma once
#include <hip/hip_runtime.h>

#include "ivr_types.h"

namespace ivr {

template <typename R> struct CpType;
template <> struct CpType<float> { using T = float4; };
template <> struct CpType<double> { using T = double4; };

template <typename R>
struct Arrays {
    const typename CpType<R>::T *cp;
    const R *rho;
    const R *knots;
    const float *tab;   // the block's basis tables (evaluators with TAB only)
};

__device__ __forceinline__ Arrays<float> arrays_of(const Model &m, float) {
    return {m.cp32, m.rho32, m.knots32, nullptr};
}
__device__ __forceinline__ Arrays<double> arrays_of(const Model &m, double) {
    return {m.cp64, m.rho64, m.knots64, nullptr};
}

// Per-block quantities the evaluators need.
template <typename R>
struct PatchView {
    int n[3];
    int nspan[3];
    R inv_nspan[3];
    int uniform;
    int cp_off;
    int knot_off[3];
};

template <typename R>
__device__ __forceinline__ PatchView<R> view_of(const DevPatch &P) {
    PatchView<R> v;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        v.n[d] = P.n[d];
        v.nspan[d] = P.nspan[d];
        v.inv_nspan[d] = R(1) / R(P.nspan[d]);
        v.knot_off[d] = P.knot_off[d];
    }
    v.uniform = P.uniform;
    v.cp_off = P.cp_off;
    return v;
}

// 1 / w of a rational point: in FP32 the hardware reciprocal (1 ulp), in FP64
// the correctly rounded quotient.
__device__ __forceinline__ float inv_weight(float w) { return __builtin_amdgcn_rcpf(w); }
__device__ __forceinline__ double inv_weight(double w) { return 1.0 / w; }

// a / b from the hardware reciprocal.  FP32: the reciprocal (1 ulp) times a.
__device__ __forceinline__ float div_fast(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// FP64: hardware reciprocal refined by one Newton step (relative error ~1e-16).
__device__ __forceinline__ double div_fast(double a, double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    return a * r;
}

template <typename R> __device__ __forceinline__ R clamp01(R v) {
    return v < R(0) ? R(0) : (v > R(1) ? R(1) : v);
}

// Knot span s (t_s <= u < t_{s+1}, s in [P, n-1]) and the 2P knots
// t_{s-P+1} .. t_{s+P} around it.  Open-uniform directions compute the knots;
// others binary-search the stored knot vector.
template <int P, typename R>
__device__ __forceinline__ int span_knots(R u_in, int n, int nspan, R inv_nspan, bool uniform,
                                          const R *__restrict__ kn, R (&t)[2 * P]) {
    const R u = clamp01(u_in);   // outside [0,1] the boundary span's polynomial continues
    int s;
    if (uniform) {
        int e = (int)(u * R(nspan));
        e = e > nspan - 1 ? nspan - 1 : e;
        s = P + e;
#pragma unroll
        for (int m = 0; m < 2 * P; ++m) t[m] = clamp01(R(e + 1 + m - P) * inv_nspan);
    } else {
        int lo = P, hi = n;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (kn[mid] <= u) lo = mid;
            else hi = mid;
        }
        s = lo;
#pragma unroll
        for (int m = 0; m < 2 * P; ++m) t[m] = kn[s - P + 1 + m];
    }
    return s;
}

// The P+1 non-zero basis functions on the span and their first derivatives
// (triangular evaluation of the recurrence; derivative from the degree P-1 row).
template <int P, typename R, bool FAST = false>
__device__ __forceinline__ void basis_d1(R u, const R (&t)[2 * P], R (&N)[P + 1],
                                         R (&dN)[P + 1]) {
    R left[P + 1], right[P + 1], M[P + 1];
    N[0] = R(1);
#pragma unroll
    for (int j = 1; j <= P; ++j) {
        left[j] = u - t[P - j];
        right[j] = t[P - 1 + j] - u;
        if (j == P) {
#pragma unroll
            for (int r = 0; r < P; ++r) M[r] = N[r];
        }
        R saved = R(0);
#pragma unroll
        for (int r = 0; r < j; ++r) {
            R temp = FAST ? div_fast(N[r], right[r + 1] + left[j - r]) : N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * temp;
            saved = left[j - r] * temp;
        }
        N[j] = saved;
    }
#pragma unroll
    for (int r = 0; r <= P; ++r) {
        R v = R(0);
        if (r > 0) v += FAST ? div_fast(M[r - 1], t[P - 1 + r] - t[r - 1]) : M[r - 1] / (t[P - 1 + r] - t[r - 1]);
        if (r < P) v -= FAST ? div_fast(M[r], t[P + r] - t[r]) : M[r] / (t[P + r] - t[r]);
        dN[r] = R(P) * v;
    }
}

// The P+1 non-zero basis functions of direction d at u and their derivatives,
// from the block's per-span polynomial tables (Horner in the local coordinate
// x = (u - t_e) / (t_{e+1} - t_e)).  Returns the span index s (t_s <= u < t_{s+1}).
template <int P, typename R>
__device__ __forceinline__ int basis_tab(const float *tab_d, R u_in, int n, int nspan, bool uniform,
                                         const R *__restrict__ kn, R (&N)[P + 1], R (&dN)[P + 1]) {
    const R u = clamp01(u_in);
    int e;
    R x, dxdu;
    if (uniform) {
        const R un = u * R(nspan);
        e = (int)un;
        e = e > nspan - 1 ? nspan - 1 : e;
        x = un - R(e);
        dxdu = R(nspan);
    } else {
        int lo = P, hi = n;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (kn[mid] <= u) lo = mid;
            else hi = mid;
        }
        e = lo - P;
        const R t0 = kn[lo], dt = kn[lo + 1] - t0;
        dxdu = div_fast(R(1), dt);
        x = (u - t0) * dxdu;
    }
    const float *c = tab_d + e * (P + 1) * (P + 1);
#pragma unroll
    for (int i = 0; i <= P; ++i) {
        R v = R(c[i * (P + 1) + P]), dv = R(P) * R(c[i * (P + 1) + P]);
#pragma unroll
        for (int k = P - 1; k >= 0; --k) {
            v = v * x + R(c[i * (P + 1) + k]);
            if (k > 0) dv = dv * x + R(k) * R(c[i * (P + 1) + k]);
        }
        N[i] = v;
        dN[i] = dv * dxdu;
    }
    return e + P;
}

// Element i of an array under 4 GiB, addressed by a 32-bit byte offset from the
// array's base: one offset computation per load instead of a 64-bit one.
template <typename T>
__device__ __forceinline__ const T &at_off32(const T *base, uint32_t i) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + i * (uint32_t)sizeof(T));
}

template <typename R>
__device__ __forceinline__ void load_cp(const typename CpType<R>::T &c, R (&v)[4]) {
    v[0] = c.x; v[1] = c.y; v[2] = c.z; v[3] = c.w;
}

// phi(p), J[r][c] = d phi_r / d p_c and rho(p): RHO = 0 no rho, 1 value,
// 2 value and parameter gradient g[c] = d rho / d p_c.
// With TAB the basis comes from the block's polynomial tables (ar.tab).
template <int P, bool RAT, int RHO, typename R, bool TAB = false>
__device__ __forceinline__ void eval_volume(const PatchView<R> &pv, const Arrays<R> &ar,
                                            const R (&p)[3], R (&x)[3], R (&J)[3][3], R &rho,
                                            R (&g)[3]) {
    const R pc[3] = {clamp01(p[0]), clamp01(p[1]), clamp01(p[2])};
    R Nu[P + 1], dNu[P + 1], Nv[P + 1], dNv[P + 1], Nw[P + 1], dNw[P + 1];
    int su, sv, sw;
    if constexpr (TAB) {
        constexpr int Q2 = (P + 1) * (P + 1);
        su = basis_tab<P>(ar.tab, pc[0], pv.n[0], pv.nspan[0], pv.uniform & 1, ar.knots + pv.knot_off[0],
                          Nu, dNu);
        sv = basis_tab<P>(ar.tab + pv.nspan[0] * Q2, pc[1], pv.n[1], pv.nspan[1], pv.uniform & 2,
                          ar.knots + pv.knot_off[1], Nv, dNv);
        sw = basis_tab<P>(ar.tab + (pv.nspan[0] + pv.nspan[1]) * Q2, pc[2], pv.n[2], pv.nspan[2],
                          pv.uniform & 4, ar.knots + pv.knot_off[2], Nw, dNw);
    } else {
        R tu[2 * P], tv[2 * P], tw[2 * P];
        su = span_knots<P>(pc[0], pv.n[0], pv.nspan[0], pv.inv_nspan[0], pv.uniform & 1,
                           ar.knots + pv.knot_off[0], tu);
        sv = span_knots<P>(pc[1], pv.n[1], pv.nspan[1], pv.inv_nspan[1], pv.uniform & 2,
                           ar.knots + pv.knot_off[1], tv);
        sw = span_knots<P>(pc[2], pv.n[2], pv.nspan[2], pv.inv_nspan[2], pv.uniform & 4,
                           ar.knots + pv.knot_off[2], tw);
        basis_d1<P, R, true>(pc[0], tu, Nu, dNu);
        basis_d1<P, R, true>(pc[1], tv, Nv, dNv);
        basis_d1<P, R, true>(pc[2], tw, Nw, dNw);
    }
    constexpr int NC = RAT ? 4 : 3;
    const int n0 = pv.n[0], n01 = pv.n[0] * pv.n[1];
    const int base = pv.cp_off + (su - P) + n0 * (sv - P) + n01 * (sw - P);
    R X[NC], Xu[NC], Xv[NC], Xw[NC], rX = R(0), rXu = R(0), rXv = R(0), rXw = R(0);
#pragma unroll
    for (int c = 0; c < NC; ++c) X[c] = Xu[c] = Xv[c] = Xw[c] = R(0);
#pragma unroll 1
    for (int k = 0; k <= P; ++k) {
        R B0[NC], B1[NC], Bu[NC], rB = R(0), rB1 = R(0), rBu = R(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) B0[c] = B1[c] = Bu[c] = R(0);
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            const int row = base + n0 * j + n01 * k;
            R A0[NC], A1[NC], rA = R(0), rA1 = R(0);
#pragma unroll
            for (int c = 0; c < NC; ++c) A0[c] = A1[c] = R(0);
#pragma unroll
            for (int i = 0; i <= P; ++i) {
                R v[4];
                load_cp<R>(ar.cp[row + i], v);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    A0[c] += Nu[i] * v[c];
                    A1[c] += dNu[i] * v[c];
                }
                if (RHO >= 1) {
                    // B-spline blocks carry rho in the fourth lane of the point
                    const R r = RAT ? ar.rho[row + i] : v[3];
                    rA += Nu[i] * r;
                    if (RHO == 2) rA1 += dNu[i] * r;
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                B0[c] += Nv[j] * A0[c];
                B1[c] += dNv[j] * A0[c];
                Bu[c] += Nv[j] * A1[c];
            }
            if (RHO >= 1) rB += Nv[j] * rA;
            if (RHO == 2) {
                rB1 += dNv[j] * rA;
                rBu += Nv[j] * rA1;
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            X[c] += Nw[k] * B0[c];
            Xw[c] += dNw[k] * B0[c];
            Xv[c] += Nw[k] * B1[c];
            Xu[c] += Nw[k] * Bu[c];
        }
        if (RHO >= 1) rX += Nw[k] * rB;
        if (RHO == 2) {
            rXw += dNw[k] * rB;
            rXv += Nw[k] * rB1;
            rXu += Nw[k] * rBu;
        }
    }
    if (RAT) {
        const R iw = inv_weight(X[NC - 1]);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            x[r] = X[r] * iw;
            J[r][0] = (Xu[r] - x[r] * Xu[NC - 1]) * iw;
            J[r][1] = (Xv[r] - x[r] * Xv[NC - 1]) * iw;
            J[r][2] = (Xw[r] - x[r] * Xw[NC - 1]) * iw;
        }
        if (RHO >= 1) rho = rX * iw;
        if (RHO == 2) {
            g[0] = (rXu - rho * Xu[NC - 1]) * iw;
            g[1] = (rXv - rho * Xv[NC - 1]) * iw;
            g[2] = (rXw - rho * Xw[NC - 1]) * iw;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            x[r] = X[r];
            J[r][0] = Xu[r];
            J[r][1] = Xv[r];
            J[r][2] = Xw[r];
        }
        if (RHO >= 1) rho = rX;
        if (RHO == 2) {
            g[0] = rXu;
            g[1] = rXv;
            g[2] = rXw;
        }
    }
}


// Second derivatives (the implicit Euler step's Hessian, Sec. "ODE Based
// Algorithm").  The P+1 non-zero basis functions on the span with their first
// and second derivatives: the rows of degree P-2, P-1 and P of the triangular
// recurrence, then the derivative rule
//   N'_{i,q} = q (N_{i,q-1} / (t_{i+q} - t_i) - N_{i+1,q-1} / (t_{i+q+1} - t_{i+1}))
// applied to row P (from row P-1), to row P-1 (from row P-2), and once more to
// the first derivatives of row P-1 for row P's second derivatives.  On a
// non-empty span every denominator is positive.
template <int P, typename R>
__device__ __forceinline__ void basis_d2(R u, const R (&t)[2 * P], R (&N)[P + 1], R (&dN)[P + 1],
                                         R (&d2N)[P + 1]) {
    R T[P + 1][P + 1], left[P + 1], right[P + 1];
    T[0][0] = R(1);
#pragma unroll
    for (int j = 1; j <= P; ++j) {
        left[j] = u - t[P - j];
        right[j] = t[P - 1 + j] - u;
        R saved = R(0);
#pragma unroll
        for (int r = 0; r < j; ++r) {
            const R temp = T[j - 1][r] / (right[r + 1] + left[j - r]);
            T[j][r] = saved + right[r + 1] * temp;
            saved = left[j - r] * temp;
        }
        T[j][j] = saved;
    }
    // derivatives of row P-1 (zero for P = 1)
    R dM[P + 1];
#pragma unroll
    for (int r = 0; r < P; ++r) {
        R v = R(0);
        if (P >= 2) {
            if (r > 0) v += T[P - 2 > 0 ? P - 2 : 0][r - 1] / (t[P - 1 + r] - t[r]);
            if (r < P - 1) v -= T[P - 2 > 0 ? P - 2 : 0][r] / (t[P + r] - t[r + 1]);
        }
        dM[r] = R(P - 1) * v;
    }
#pragma unroll
    for (int r = 0; r <= P; ++r) {
        R v = R(0), w = R(0);
        if (r > 0) {
            const R den = t[P - 1 + r] - t[r - 1];
            v += T[P - 1][r - 1] / den;
            w += dM[r - 1] / den;
        }
        if (r < P) {
            const R den = t[P + r] - t[r];
            v -= T[P - 1][r] / den;
            w -= dM[r] / den;
        }
        N[r] = T[P][r];
        dN[r] = R(P) * v;
        d2N[r] = R(P) * w;
    }
}

// As basis_tab, with second derivatives (Horner on the span's polynomials).
template <int P, typename R>
__device__ __forceinline__ int basis_tab2(const float *tab_d, R u_in, int n, int nspan, bool uniform,
                                          const R *__restrict__ kn, R (&N)[P + 1], R (&dN)[P + 1],
                                          R (&d2N)[P + 1]) {
    const R u = clamp01(u_in);
    int e;
    R x, dxdu;
    if (uniform) {
        const R un = u * R(nspan);
        e = (int)un;
        e = e > nspan - 1 ? nspan - 1 : e;
        x = un - R(e);
        dxdu = R(nspan);
    } else {
        int lo = P, hi = n;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (kn[mid] <= u) lo = mid;
            else hi = mid;
        }
        e = lo - P;
        const R t0 = kn[lo], dt = kn[lo + 1] - t0;
        dxdu = R(1) / dt;
        x = (u - t0) * dxdu;
    }
    const float *c = tab_d + e * (P + 1) * (P + 1);
#pragma unroll
    for (int i = 0; i <= P; ++i) {
        R v = R(0), dv = R(0), d2v = R(0);
#pragma unroll
        for (int k = P; k >= 0; --k) {
            const R ck = R(c[i * (P + 1) + k]);
            v = v * x + ck;
            if (k >= 1) dv = dv * x + R(k) * ck;
            if (k >= 2) d2v = d2v * x + R(k * (k - 1)) * ck;
        }
        N[i] = v;
        dN[i] = dv * dxdu;
        d2N[i] = d2v * dxdu * dxdu;
    }
    return e + P;
}

// phi(p), J[r][a] = d phi_r / d p_a and the Hessian in packed symmetric form,
// H[r][k] = d^2 phi_r / dp_a dp_b for (a, b) = (0,0), (1,1), (2,2), (0,1),
// (0,2), (1,2) in k = 0..5.  Sum-factorised like eval_volume, carrying the
// second derivatives along; NURBS by the quotient rule applied twice,
//   phi_ab = (X_ab - phi_a w_b - phi_b w_a - phi w_ab) / w.
template <int P, bool RAT, typename R, bool TAB = false>
__device__ __forceinline__ void eval_volume_h(const PatchView<R> &pv, const Arrays<R> &ar, const R (&p)[3],
                                              R (&x)[3], R (&J)[3][3], R (&H)[3][6]) {
    const R pc[3] = {clamp01(p[0]), clamp01(p[1]), clamp01(p[2])};
    R Nu[P + 1], dNu[P + 1], ddNu[P + 1], Nv[P + 1], dNv[P + 1], ddNv[P + 1], Nw[P + 1], dNw[P + 1],
        ddNw[P + 1];
    int su, sv, sw;
    if constexpr (TAB) {
        constexpr int Q2 = (P + 1) * (P + 1);
        su = basis_tab2<P>(ar.tab, pc[0], pv.n[0], pv.nspan[0], pv.uniform & 1, ar.knots + pv.knot_off[0], Nu,
                           dNu, ddNu);
        sv = basis_tab2<P>(ar.tab + pv.nspan[0] * Q2, pc[1], pv.n[1], pv.nspan[1], pv.uniform & 2,
                           ar.knots + pv.knot_off[1], Nv, dNv, ddNv);
        sw = basis_tab2<P>(ar.tab + (pv.nspan[0] + pv.nspan[1]) * Q2, pc[2], pv.n[2], pv.nspan[2],
                           pv.uniform & 4, ar.knots + pv.knot_off[2], Nw, dNw, ddNw);
    } else {
        R tu[2 * P], tv[2 * P], tw[2 * P];
        su = span_knots<P>(pc[0], pv.n[0], pv.nspan[0], pv.inv_nspan[0], pv.uniform & 1,
                           ar.knots + pv.knot_off[0], tu);
        sv = span_knots<P>(pc[1], pv.n[1], pv.nspan[1], pv.inv_nspan[1], pv.uniform & 2,
                           ar.knots + pv.knot_off[1], tv);
        sw = span_knots<P>(pc[2], pv.n[2], pv.nspan[2], pv.inv_nspan[2], pv.uniform & 4,
                           ar.knots + pv.knot_off[2], tw);
        basis_d2<P, R>(pc[0], tu, Nu, dNu, ddNu);
        basis_d2<P, R>(pc[1], tv, Nv, dNv, ddNv);
        basis_d2<P, R>(pc[2], tw, Nw, dNw, ddNw);
    }
    constexpr int NC = RAT ? 4 : 3;
    const int n0 = pv.n[0], n01 = pv.n[0] * pv.n[1];
    const int base = pv.cp_off + (su - P) + n0 * (sv - P) + n01 * (sw - P);
    // X: value; X1[a]: d/dp_a; X2[k]: the packed second derivatives
    R X[NC], X1[3][NC], X2[6][NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        X[c] = R(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) X1[a][c] = R(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) X2[k][c] = R(0);
    }
#pragma unroll 1
    for (int k = 0; k <= P; ++k) {
        // B[.]: sums over u and v with the v-derivatives of orders 0..2 and the
        // u-derivatives of orders 0..2 (combined order at most 2)
        R B00[NC], B01[NC], B02[NC], B10[NC], B11[NC], B20[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) B00[c] = B01[c] = B02[c] = B10[c] = B11[c] = B20[c] = R(0);
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            const int row = base + n0 * j + n01 * k;
            R A0[NC], A1[NC], A2[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) A0[c] = A1[c] = A2[c] = R(0);
#pragma unroll
            for (int i = 0; i <= P; ++i) {
                R v[4];
                load_cp<R>(ar.cp[row + i], v);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    A0[c] += Nu[i] * v[c];
                    A1[c] += dNu[i] * v[c];
                    A2[c] += ddNu[i] * v[c];
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                B00[c] += Nv[j] * A0[c];
                B01[c] += dNv[j] * A0[c];
                B02[c] += ddNv[j] * A0[c];
                B10[c] += Nv[j] * A1[c];
                B11[c] += dNv[j] * A1[c];
                B20[c] += Nv[j] * A2[c];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            X[c] += Nw[k] * B00[c];
            X1[0][c] += Nw[k] * B10[c];
            X1[1][c] += Nw[k] * B01[c];
            X1[2][c] += dNw[k] * B00[c];
            X2[0][c] += Nw[k] * B20[c];     // uu
            X2[1][c] += Nw[k] * B02[c];     // vv
            X2[2][c] += ddNw[k] * B00[c];   // ww
            X2[3][c] += Nw[k] * B11[c];     // uv
            X2[4][c] += dNw[k] * B10[c];    // uw
            X2[5][c] += dNw[k] * B01[c];    // vw
        }
    }
    if constexpr (RAT) {
        const R iw = R(1) / X[3];
        constexpr int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            x[r] = X[r] * iw;
#pragma unroll
            for (int a = 0; a < 3; ++a) J[r][a] = (X1[a][r] - x[r] * X1[a][3]) * iw;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                H[r][k] = (X2[k][r] - J[r][pa[k]] * X1[pb[k]][3] - J[r][pb[k]] * X1[pa[k]][3] - x[r] * X2[k][3]) * iw;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            x[r] = X[r];
#pragma unroll
            for (int a = 0; a < 3; ++a) J[r][a] = X1[a][r];
#pragma unroll
            for (int k = 0; k < 6; ++k) H[r][k] = X2[k][r];
        }
    }
}

// Boundary face f (0..5 = u0,u1,v0,v1,w0,w1): in-face directions (a, b) are the two
// remaining parameter directions in increasing order.
__device__ __forceinline__ void face_dirs(int face, int &dn, int &da, int &db) {
    dn = face >> 1;
    da = dn == 0 ? 1 : 0;
    db = dn == 2 ? 1 : 2;
}

// Face f of a block as the face evaluator needs it: along the in-face directions
// (a, b) the control-point counts, spans, open-uniform flags, knot offsets and
// control-point strides, and the index of the face layer's first control point.
// Taken once per face from the block record in global memory: a private copy of
// the block's per-direction arrays, indexed by the face's runtime directions,
// would live in scratch memory.
template <typename R>
struct FaceView {
    int na, nb, nsa, nsb;
    bool ua, ub;
    R inva, invb;
    int koa, kob;
    int stra, strb;
    int base;
};

template <typename R>
__device__ __forceinline__ FaceView<R> face_view(const DevPatch &P, int face) {
    int dn, da, db;
    face_dirs(face, dn, da, db);
    FaceView<R> f;
    f.na = P.n[da];
    f.nb = P.n[db];
    f.nsa = P.nspan[da];
    f.nsb = P.nspan[db];
    f.ua = (P.uniform >> da) & 1;
    f.ub = (P.uniform >> db) & 1;
    if constexpr (sizeof(R) == 4) {   // the block record holds 1 / spans in FP32
        f.inva = P.inv_nspan[da];
        f.invb = P.inv_nspan[db];
    } else {
        f.inva = R(1) / R(f.nsa);
        f.invb = R(1) / R(f.nsb);
    }
    f.koa = P.knot_off[da];
    f.kob = P.knot_off[db];
    const int n0 = P.n[0], n01 = P.n[0] * P.n[1];
    f.stra = da == 0 ? 1 : n0;     // da is 0 or 1
    f.strb = db == 1 ? n0 : n01;   // db is 1 or 2
    const int strn = dn == 0 ? 1 : (dn == 1 ? n0 : n01);
    f.base = P.cp_off + ((face & 1) ? (P.n[dn] - 1) * strn : 0);
    return f;
}

// S(a,b), dS/da, dS/db on face f: the bivariate spline of the boundary layer.
// Outside [0,1]^2 the polynomial of the nearest boundary span is continued, so
// Newton iterates may leave the face and come back.
// With DERIV false only S is computed (Sa, Sb are left untouched).
template <int P, bool RAT, typename R, bool DERIV = true>
__device__ __forceinline__ void eval_face(const FaceView<R> &fv, const Arrays<R> &ar, R a, R b,
                                          R (&S)[3], R (&Sa)[3], R (&Sb)[3]) {
    R ta[2 * P], tb[2 * P];
    const int sa = span_knots<P>(a, fv.na, fv.nsa, fv.inva, fv.ua, ar.knots + fv.koa, ta);
    const int sb = span_knots<P>(b, fv.nb, fv.nsb, fv.invb, fv.ub, ar.knots + fv.kob, tb);
    R Na[P + 1], dNa[P + 1], Nb[P + 1], dNb[P + 1];
    basis_d1<P, R, true>(a, ta, Na, dNa);
    basis_d1<P, R, true>(b, tb, Nb, dNb);
    const int base = fv.base + (sa - P) * fv.stra + (sb - P) * fv.strb;
    constexpr int NC = RAT ? 4 : 3;
    R H[NC], Ha[NC], Hb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) H[c] = Ha[c] = Hb[c] = R(0);
#pragma unroll 1
    for (int jb = 0; jb <= P; ++jb) {
        R A0[NC], A1[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) A0[c] = A1[c] = R(0);
#pragma unroll
        for (int ia = 0; ia <= P; ++ia) {
            R v[4];
            load_cp<R>(at_off32(ar.cp, (uint32_t)(base + ia * fv.stra + jb * fv.strb)), v);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                A0[c] += Na[ia] * v[c];
                if (DERIV) A1[c] += dNa[ia] * v[c];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            H[c] += Nb[jb] * A0[c];
            if (DERIV) {
                Hb[c] += dNb[jb] * A0[c];
                Ha[c] += Nb[jb] * A1[c];
            }
        }
    }
    if (RAT) {
        const R iw = inv_weight(H[NC - 1]);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            S[r] = H[r] * iw;
            if (DERIV) {
                Sa[r] = (Ha[r] - S[r] * Ha[NC - 1]) * iw;
                Sb[r] = (Hb[r] - S[r] * Hb[NC - 1]) * iw;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            S[r] = H[r];
            if (DERIV) {
                Sa[r] = Ha[r];
                Sb[r] = Hb[r];
            }
        }
    }
}

template <typename R> __device__ __forceinline__ R dot3(const R (&a)[3], const R (&b)[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
template <typename R>
__device__ __forceinline__ void cross3(const R (&a)[3], const R (&b)[3], R (&c)[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Solve [c0 c1 c2] x = r by Cramer's rule (the determinant is returned).
template <typename R>
__device__ __forceinline__ R solve_cols(const R (&c0)[3], const R (&c1)[3], const R (&c2)[3],
                                        const R (&r)[3], R (&x)[3]) {
    R k12[3], k20[3], k01[3];
    cross3(c1, c2, k12);
    cross3(c2, c0, k20);
    cross3(c0, c1, k01);
    const R det = dot3(c0, k12);
    const R inv = div_fast(R(1), det);
    x[0] = dot3(r, k12) * inv;
    x[1] = dot3(r, k20) * inv;
    x[2] = dot3(r, k01) * inv;
    return det;
}

// rho at p and its derivative along the ray, d rho/ds = grad rho . W with
// J W = d (W on the ray itself, where V_perp vanishes).
// Returns det J_phi(p).
template <int P, bool RAT, typename R>
__device__ __forceinline__ R eval_rho_ds(const PatchView<R> &pv, const Arrays<R> &ar,
                                         const R (&p)[3], const R (&d)[3], R &rho, R &drho) {
    R x[3], J[3][3], g[3];
    eval_volume<P, RAT, 2>(pv, ar, p, x, J, rho, g);
    R ju[3] = {J[0][0], J[1][0], J[2][0]}, jv[3] = {J[0][1], J[1][1], J[2][1]},
      jw[3] = {J[0][2], J[1][2], J[2][2]}, W[3];
    const R det = solve_cols(ju, jv, jw, d, W);
    drho = (det != R(0) && isfinite(det)) ? dot3(g, W) : R(0);
    return det;
}

// Pulled-back ray field, Eq. (VgVp): J_phi(p) W = V(phi(p)) with
// V(g) = V_par + c V_perp(g), V_perp(g) = (g_in - g) - <g_in - g, V_par> V_par (Eq. (vec2)).
// The view ray itself gives V_par = d and g_in.  Returns the determinant of J;
// near-singular systems are solved again in FP64.
// With newton set, the right-hand side is r = gin - phi(p) instead, so W is the
// Newton step of phi(p) = gin (Eq. (newtonsmethod)); res2 = |r|^2.
// x: phi(p).  With TAN, Wt = J^-1 d as well (the ray's tangent in P, from the
// same factors).
template <int P, bool RAT, int RHO, typename R, bool TAB = false, bool TAN = false>
__device__ __forceinline__ R eval_W(const PatchView<R> &pv, const Arrays<R> &ar, const R (&p)[3],
                                    const R (&gin)[3], const R (&d)[3], R c, R det_thr, R (&W)[3],
                                    R &rho, R (&grho)[3], uint32_t &n_fp64, bool newton, R &res2,
                                    R (&x)[3], R (&Wt)[3]) {
    R J[3][3];
    eval_volume<P, RAT, RHO, R, TAB>(pv, ar, p, x, J, rho, grho);
    R r[3] = {gin[0] - x[0], gin[1] - x[1], gin[2] - x[2]};
    const R rd = dot3(r, d);
    res2 = dot3(r, r);
    R V[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) V[q] = newton ? r[q] : d[q] + c * (r[q] - rd * d[q]);
    R ju[3] = {J[0][0], J[1][0], J[2][0]}, jv[3] = {J[0][1], J[1][1], J[2][1]},
      jw[3] = {J[0][2], J[1][2], J[2][2]};
    R det;
    if constexpr (TAN) {
        R k12[3], k20[3], k01[3];
        cross3(jv, jw, k12);
        cross3(jw, ju, k20);
        cross3(ju, jv, k01);
        det = dot3(ju, k12);
        const R inv = div_fast(R(1), det);
        W[0] = dot3(V, k12) * inv;
        W[1] = dot3(V, k20) * inv;
        W[2] = dot3(V, k01) * inv;
        Wt[0] = dot3(d, k12) * inv;
        Wt[1] = dot3(d, k20) * inv;
        Wt[2] = dot3(d, k01) * inv;
    } else {
        det = solve_cols(ju, jv, jw, V, W);
    }
    if (!(fabs(det) >= det_thr)) {
        double du[3] = {ju[0], ju[1], ju[2]}, dv[3] = {jv[0], jv[1], jv[2]},
               dw[3] = {jw[0], jw[1], jw[2]}, dV[3] = {V[0], V[1], V[2]}, dW[3];
        solve_cols(du, dv, dw, dV, dW);
        W[0] = R(dW[0]); W[1] = R(dW[1]); W[2] = R(dW[2]);
        if constexpr (TAN) {
            double dd[3] = {d[0], d[1], d[2]};
            solve_cols(du, dv, dw, dd, dW);
            Wt[0] = R(dW[0]); Wt[1] = R(dW[1]); Wt[2] = R(dW[2]);
        }
        ++n_fp64;
    }
    return det;
}

// Transfer function: value on the interval that contains n (exact piecewise
// linear).  out = (R, G, B, kappa).
__device__ __forceinline__ void tf_eval(const FrameParams &fp, float rho, float (&out)[4]) {
    float n = clamp01((rho - fp.tf_lo) * fp.tf_inv_range);
    float x0 = fp.tf_x[0];
    float v[4] = {fp.tf_v[0][0], fp.tf_v[0][1], fp.tf_v[0][2], fp.tf_v[0][3]};
    float s[4] = {fp.tf_s[0][0], fp.tf_s[0][1], fp.tf_s[0][2], fp.tf_s[0][3]};
#pragma unroll
    for (int k = 1; k < kMaxTfKnots - 1; ++k) {
        if (k < fp.tf_n - 1) {
            const bool in = n >= fp.tf_x[k];
            x0 = in ? fp.tf_x[k] : x0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                v[c] = in ? fp.tf_v[k][c] : v[c];
                s[c] = in ? fp.tf_s[k][c] : s[c];
            }
        }
    }
    const float dn = n - x0;
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c] = v[c] + s[c] * dn;
}

__device__ __forceinline__ void tf_eval(const FrameParams &fp, double rho, double (&out)[4]) {
    double n = clamp01((rho - fp.tf_lod) * fp.tf_inv_ranged);
    double x0 = fp.tf_xd[0];
    double v[4] = {fp.tf_vd[0][0], fp.tf_vd[0][1], fp.tf_vd[0][2], fp.tf_vd[0][3]};
    double s[4] = {fp.tf_sd[0][0], fp.tf_sd[0][1], fp.tf_sd[0][2], fp.tf_sd[0][3]};
#pragma unroll
    for (int k = 1; k < kMaxTfKnots - 1; ++k) {
        if (k < fp.tf_n - 1) {
            const bool in = n >= fp.tf_xd[k];
            x0 = in ? fp.tf_xd[k] : x0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                v[c] = in ? fp.tf_vd[k][c] : v[c];
                s[c] = in ? fp.tf_sd[k][c] : s[c];
            }
        }
    }
    const double dn = n - x0;
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c] = v[c] + s[c] * dn;
}

// The integrator stages every view's transfer function and step bounds in LDS
// (ViewLds); one thread per view fills a record.
__device__ __forceinline__ void view_stage(const ViewRec *views, int n_views, ViewLds *vls) {
    for (int v = threadIdx.x; v < n_views; v += blockDim.x) {
        const FrameParams &f = views[v].fp;
        ViewLds &w = vls[v];
#pragma unroll
        for (int k = 0; k < kMaxTfKnots; ++k) {
            const float x = f.tf_x[k];
            w.b[k] = make_float4(f.tf_s[k][0], f.tf_s[k][1], f.tf_s[k][2], f.tf_s[k][3]);
            w.a[k] = make_float4(f.tf_v[k][0] - f.tf_s[k][0] * x, f.tf_v[k][1] - f.tf_s[k][1] * x,
                                 f.tf_v[k][2] - f.tf_s[k][2] * x, f.tf_v[k][3] - f.tf_s[k][3] * x);
            w.x[k] = (k >= 1 && k < f.tf_n - 1) ? x : INFINITY;
            w.smax[k] = f.tf_smax[k];
        }
        w.lo = f.tf_lo;
        w.inv_range = f.tf_inv_range;
        w.dn = f.tf_dn;
        w.h_max = f.h_max;
        w.h_min = f.h_min;
        w.scale = f.scale;
        w.inv_ranged = f.tf_inv_ranged;
    }
    __syncthreads();
}

// Interval of n: the number of interior knots at or below it, from the sign
// bits of n - x (n - x >= +0 exactly when n >= x; a +inf slot gives -inf), with
// no compares.  nint (uniform): the most interior knots of any view of the
// batch; the slots past a view's own knots hold +inf.
__device__ __forceinline__ int tf_interval(const ViewLds &w, float n, int nint) {
    static_assert(kMaxTfKnots == 16, "interior knot slots 1..14");
    auto below = [&](int m) __attribute__((always_inline)) -> uint32_t {
        return __float_as_uint(n - w.x[m]) >> 31;
    };
    uint32_t lt = below(1) + below(2) + below(3) + below(4) + below(5) + below(6);
    int slots = 6;
    if (nint > 6) {
        lt += below(7) + below(8) + below(9) + below(10) + below(11) + below(12) + below(13) + below(14);
        slots = 14;
    }
    return slots - (int)lt;
}

__device__ __forceinline__ void tf_eval(const ViewLds &w, float rho, float (&out)[4], int nint) {
    const float n = clamp01((rho - w.lo) * w.inv_range);
    const int k = tf_interval(w, n, nint);
    const float4 a = w.a[k], b = w.b[k];
    out[0] = a.x + b.x * n;
    out[1] = a.y + b.y * n;
    out[2] = a.z + b.z * n;
    out[3] = a.w + b.w * n;
}

__device__ __forceinline__ float fast_exp(float x) { return __expf(x); }
__device__ __forceinline__ double fast_exp(double x) { return exp(x); }

// Supersampling (Sec. "Quadrature of volume render integral"): between two
// samples rho is interpolated without further spline evaluations, either
// linearly (the paper's assumption) or as the cubic Hermite interpolant of the
// two values and their derivatives along the ray (ma, mb = d rho / ds).  The
// interval is split into n_super equal sub-intervals, each evaluated at its
// midpoint and composited by Algorithm "Front-to-back compositing" with
// (1 - alpha_src)^(ds/xi) = exp(-kappa ds).
// The number of sub-steps is at least n_super and grows with the change of the
// normalised value n over the step and with the transfer function's slope over
// that range of n (the transfer function's frequencies set the sampling rate,
// not the spline): the transfer function changes by at most tf_step per
// sub-step, and n by at most dn; up to 128.
// fb: the batch's options (n_super, hermite, tf_step); fv / w: the view's
// transfer function (FP64 from fv, FP32 from its LDS copy w).
template <typename R>
__device__ __forceinline__ void composite(const FrameParams &fb, const FrameParams &fv, const ViewLds &w,
                                          R ra, R ma, R rb, R mb, R len, R (&C)[3], R &A,
                                          uint32_t &n_sub) {
    const FrameParams &fp = fb;
    const R sa = fp.hermite ? ma * len : (rb - ra), sb = fp.hermite ? mb * len : (rb - ra);
    const R inv_range = sizeof(R) == 4 ? R(w.inv_range) : R(fv.tf_inv_ranged);
    const R tdn = sizeof(R) == 4 ? R(w.dn) : R(fv.tf_dn);
    const R span = fmax(fabs(rb - ra), R(0.5) * (fabs(sa) + fabs(sb))) * inv_range;
    // the largest slope of the transfer function over the interval's range of n
    // (the Hermite interpolant stays within a quarter of its end slopes' sum)
    const R lo_r = sizeof(R) == 4 ? R(w.lo) : R(fv.tf_lod);
    const R na = (ra - lo_r) * inv_range, nb = (rb - lo_r) * inv_range;
    const R over = R(0.25) * (fabs(sa) + fabs(sb)) * inv_range;
    const float n_lo = float(fmin(na, nb) - over), n_hi = float(fmax(na, nb) + over);
    float sm = 0.f;
#pragma unroll
    for (int m = 0; m < kMaxTfKnots - 1; ++m) {   // interval m: [x[m], x[m+1]), x[0] = -inf
        const bool exists = sizeof(R) == 4 || m < fv.tf_n - 1;
        const float xm = sizeof(R) == 4 ? w.x[m] : fv.tf_x[m];
        const float xm1 = sizeof(R) == 4 ? w.x[m + 1] : (m + 1 < fv.tf_n - 1 ? fv.tf_x[m + 1] : INFINITY);
        const float smm = sizeof(R) == 4 ? w.smax[m] : fv.tf_smax[m];
        if (exists && (m == 0 || xm <= n_hi) && xm1 > n_lo) sm = fmaxf(sm, smm);
    }
    int ns = (int)ceil(fmax(span / tdn, span * R(sm) / R(fp.tf_step)));
    ns = ns < fp.n_super ? fp.n_super : (ns > 128 ? 128 : ns);
    n_sub += (uint32_t)ns;
    const R inv = R(1) / R(ns);
    const R dl = len * inv;
    for (int j = 0; j < ns; ++j) {
        const R tau = (R(j) + R(0.5)) * inv, t2 = tau * tau, t3 = t2 * tau;
        // Hermite basis; with sa = sb = rb - ra it reduces to linear interpolation
        const R rho = (R(2) * t3 - R(3) * t2 + R(1)) * ra + (t3 - R(2) * t2 + tau) * sa +
                      (R(3) * t2 - R(2) * t3) * rb + (t3 - t2) * sb;
        R e[4];
        if constexpr (sizeof(R) == 4) tf_eval(w, rho, e, fb.tf_nint_max);
        else tf_eval(fv, rho, e);
        const R T = fast_exp(-e[3] * dl);
        const R w = (R(1) - T) * (R(1) - A);
        C[0] += w * e[0];
        C[1] += w * e[1];
        C[2] += w * e[2];
        A += w;
    }
}

}  // namespace ivr
