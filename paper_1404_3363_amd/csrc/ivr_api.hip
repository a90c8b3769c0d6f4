// Host side of the C ABI declared in include/ivr.h: argument validation, model
// packing (FP32 + FP64 control nets, knot vectors, block / face / face-element
// bounding boxes), frame-buffer management and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "ivr.h"
#include "ivr_internal.h"
#include "ivr_types.h"

using namespace ivr;

struct ivr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 0;
    std::string err;
    bool has_model = false;
    // model
    DevPatch *d_patches = nullptr;
    float4 *d_cp32 = nullptr;
    float *d_rho32 = nullptr;
    double4 *d_cp64 = nullptr;
    double *d_rho64 = nullptr;
    DeltaESum *d_desum = nullptr;         // image-comparison summary (ivr_delta_e2000)
    float4 *d_disp32 = nullptr;           // displacement (w u, w) per control point, or null
    double4 *d_disp64 = nullptr;
    bool all_disp = false;                // every block carries a displacement spline
    float *d_knots32 = nullptr;
    double *d_knots64 = nullptr;
    FaceElem *d_elems = nullptr;
    float *d_btab = nullptr;
    FaceTile *d_tiles = nullptr;
    int npatch = 0, nelem = 0;
    double scale = 1.0;
    uint32_t class_mask = 0;
    struct ModelRange {
        int begin, end;          // patches [begin, end)
        double scale;            // bounding-box diagonal of its control points
        uint32_t class_mask;     // degree classes present
    };
    std::vector<ModelRange> models;
    // batch view table: device copy and pinned host staging (grow-only)
    ViewRec *d_views = nullptr;
    ViewRec *h_views = nullptr;
    int view_cap = 0;
    hipEvent_t views_copied = nullptr;   // the staging buffer may be rewritten after it
    hipStream_t capture = nullptr;       // private stream the batch graphs are captured on
    // launch shapes (autotuned) and captured batch graphs keyed by their shape
    LaunchCfg lc = {8, 0, 256, 0};
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
    unsigned long long generation = 0;   // bumps when buffers move (graphs hold pointers)
    // frame buffers, sized from counts: segment slots and candidate entries per
    // pixel, the largest ratio the renders so far needed (read back without
    // blocking after every render of the context's own buffers)
    size_t pix_cap = 0, seg_cap = 0, seg_bytes_cap = 0;
    double seg_ratio = 0.0, cand_ratio = 0.0;
    size_t model_bytes = 0;
    // pinned host memory the merge kernel writes each frame's (segments requested,
    // candidates recorded, pixels) to, and its device address
    uint32_t *h_totals = nullptr, *d_totals = nullptr;

    void *d_segs = nullptr;
    uint2 *d_pixseg = nullptr;
    uint2 *d_seg_kr = nullptr;           // (block, rank among the block's segments)
    uint32_t *d_order = nullptr;         // segment indices sorted by block
    QueueState *d_qs = nullptr;
    // two-pass fragment kernel with MLP seeds (grow-only)
    CandLists mq = {nullptr, nullptr, nullptr, nullptr, nullptr, 0};
    size_t mq_tiles = 0;
    // blocks grouped by degree class (the integrators take their segments block by block)
    uint32_t *d_pperm = nullptr, *d_pcount = nullptr, *d_pbase = nullptr, *d_pcur = nullptr;
    int cls_q[kClasses + 1] = {0};       // class k's blocks are pperm[cls_q[k] .. cls_q[k+1])
    int cls_max_cp[kClasses] = {0};      // largest control net of the class
    int cls_max_tab[kClasses] = {0};     // largest basis tables of the class (floats)
    unsigned long long *d_ctr = nullptr;
    unsigned long long *h_ctr = nullptr;  // pinned staging of the counters (stats)
    unsigned char *scratch = nullptr;     // this device's scratch array (ivr_render_noalloc)
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // phase events of renders recorded with opts.timing (4 per render)
    std::vector<hipEvent_t> tev;
    int n_timed = 0;
    // learned initialiser
    std::vector<DevPatch> hpatch;
    MlpState mlp = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool mlp_trained = false;
};

// Scratch memory of ivr_render_noalloc: one fixed array per GPU, held until the
// process ends.  In host code the array's name is not a device address; the
// address comes from hipGetSymbolAddress on each device (at ivr_create, with the
// device current) and is kept per device.
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr uint32_t kNoAllocMaxPixels = 1u << 20;
constexpr int kNoAllocMaxBlocks = 1 << 16;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxDevices];

namespace {

ivr_status fail(ivr_ctx *c, ivr_status code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define IVR_HIP(ctx, call)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, IVR_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

float round_down(double v) {
    float f = (float)v;
    return (double)f > v ? std::nextafter(f, -INFINITY) : f;
}
float round_up(double v) {
    float f = (float)v;
    return (double)f < v ? std::nextafter(f, INFINITY) : f;
}

struct Box {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void add(const double *p) {
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], p[c]);
            hi[c] = std::max(hi[c], p[c]);
        }
    }
    void store(float *dst, double pad) const {
        for (int c = 0; c < 3; ++c) {
            dst[c] = round_down(lo[c] - pad);
            dst[3 + c] = round_up(hi[c] + pad);
        }
    }
};

std::string validate_patch(const ivr_patch_desc &P, int idx) {
    char buf[256];
    for (int d = 0; d < 3; ++d) {
        const int p = P.degree[d];
        if (p < 1 || p > kMaxDegree) {
            snprintf(buf, sizeof buf, "patch %d: degree %d outside 1..3", idx, P.degree[d]);
            return buf;
        }
        if (P.ncp[d] < p + 1 || P.ncp[d] > 4096) {
            snprintf(buf, sizeof buf, "patch %d: ncp[%d]=%d outside degree+1..4096", idx, d, P.ncp[d]);
            return buf;
        }
        if (!P.knots[d]) {
            snprintf(buf, sizeof buf, "patch %d: knots[%d] is NULL", idx, d);
            return buf;
        }
        const int nk = P.ncp[d] + p + 1, n = P.ncp[d];
        const double *t = P.knots[d];
        for (int i = 0; i < nk; ++i)
            if (!std::isfinite(t[i]) || (i > 0 && t[i] < t[i - 1])) {
                snprintf(buf, sizeof buf, "patch %d: knots[%d] not finite and non-decreasing", idx, d);
                return buf;
            }
        for (int i = 1; i <= p; ++i)
            if (t[i] != t[0] || t[n + i] != t[n]) {
                snprintf(buf, sizeof buf, "patch %d: knots[%d] not clamped", idx, d);
                return buf;
            }
        if (!(t[p] < t[n])) {
            snprintf(buf, sizeof buf, "patch %d: knots[%d] span is empty", idx, d);
            return buf;
        }
        for (int i = p + 1; i < n; ++i) {
            int mult = 1;
            while (i + mult < n && t[i + mult] == t[i]) ++mult;
            if (mult > p || t[i] == t[p] || t[i] == t[n]) {
                snprintf(buf, sizeof buf, "patch %d: knots[%d] interior multiplicity > degree", idx, d);
                return buf;
            }
        }
    }
    if (!P.cp || !P.scalar) {
        snprintf(buf, sizeof buf, "patch %d: cp or scalar is NULL", idx);
        return buf;
    }
    const size_t N = (size_t)P.ncp[0] * P.ncp[1] * P.ncp[2];
    for (size_t i = 0; i < N; ++i) {
        const double *c = P.cp + 4 * i;
        if (!finite3(c) || !std::isfinite(P.scalar[i]) ||
            (P.rational && !(std::isfinite(c[3]) && c[3] > 0.0))) {
            snprintf(buf, sizeof buf, "patch %d: control point %zu not finite or weight <= 0", idx, i);
            return buf;
        }
        if (P.displacement && !finite3(P.displacement + 3 * i)) {
            snprintf(buf, sizeof buf, "patch %d: displacement %zu not finite", idx, i);
            return buf;
        }
    }
    return "";
}

// sign of det J from the control net at the 8 corners (derivatives at a clamped
// corner are positive multiples of the first edges of the net)
float orientation(const ivr_patch_desc &P) {
    const int n0 = P.ncp[0], n1 = P.ncp[1], n2 = P.ncp[2];
    auto pt = [&](int i, int j, int k, double *o) {
        const double *c = P.cp + 4 * ((size_t)i + (size_t)n0 * (j + (size_t)n1 * k));
        for (int q = 0; q < 3; ++q) o[q] = c[q];
    };
    int pos = 0, neg = 0;
    for (int ci = 0; ci < 8; ++ci) {
        const int i = (ci & 1) ? n0 - 2 : 0, j = (ci & 2) ? n1 - 2 : 0, k = (ci & 4) ? n2 - 2 : 0;
        const int i0 = (ci & 1) ? n0 - 1 : 0, j0 = (ci & 2) ? n1 - 1 : 0, k0 = (ci & 4) ? n2 - 1 : 0;
        double c0[3], cu[3], cv[3], cw[3];
        pt(i0, j0, k0, c0);
        // forward differences in +u, +v, +w between the corner layer and the next layer
        double a[3], b[3], c[3], t0[3], t1[3];
        pt(i, j0, k0, t0); pt(i + 1, j0, k0, t1);
        for (int q = 0; q < 3; ++q) a[q] = t1[q] - t0[q];
        pt(i0, j, k0, t0); pt(i0, j + 1, k0, t1);
        for (int q = 0; q < 3; ++q) b[q] = t1[q] - t0[q];
        pt(i0, j0, k, t0); pt(i0, j0, k + 1, t1);
        for (int q = 0; q < 3; ++q) c[q] = t1[q] - t0[q];
        (void)cu; (void)cv; (void)cw;
        const double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                           a[2] * (b[0] * c[1] - b[1] * c[0]);
        if (det > 0) ++pos;
        else if (det < 0) ++neg;
    }
    return neg > pos ? -1.0f : 1.0f;
}

// Blossom of a degree-p B-spline segment on knot span s: de Boor's algorithm with
// argument args[r-1] at level r.  Q holds the p+1 homogeneous control points
// s-p..s.  The Bezier points of the span [t_s, t_{s+1}] are the blossoms at
// (t_s^(p-j), t_{s+1}^j), j = 0..p.
// Host evaluation of a block's face surface (projected), for matching shared
// faces at upload.  Basis on the normalised knots by the triangular recurrence.
static void host_basis(const double *t, int n, int p, double u, int &span, double *N) {
    const double t0 = t[p], t1 = t[n];
    auto tn = [&](int i) { return (t[i] - t0) / (t1 - t0); };
    int s = p;
    while (s < n - 1 && tn(s + 1) <= u) ++s;
    span = s;
    double left[4], right[4];
    N[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = u - tn(s + 1 - j);
        right[j] = tn(s + j) - u;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            const double tmp = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
    }
}

static void face_surface(const ivr_patch_desc &P, int face, double a, double b, double x[3]) {
    const int dn = face >> 1, da = dn == 0 ? 1 : 0, db = dn == 2 ? 1 : 2, p = P.degree[0];
    const int fix = (face & 1) ? P.ncp[dn] - 1 : 0;
    int sa, sb;
    double Na[4], Nb[4];
    host_basis(P.knots[da], P.ncp[da], p, a, sa, Na);
    host_basis(P.knots[db], P.ncp[db], p, b, sb, Nb);
    double h[4] = {0, 0, 0, 0};
    for (int jb = 0; jb <= p; ++jb)
        for (int ia = 0; ia <= p; ++ia) {
            int ijk[3];
            ijk[dn] = fix; ijk[da] = sa - p + ia; ijk[db] = sb - p + jb;
            const double *cc = P.cp + 4 * ((size_t)ijk[0] + (size_t)P.ncp[0] * (ijk[1] + (size_t)P.ncp[1] * ijk[2]));
            const double w = P.rational ? cc[3] : 1.0, k = Na[ia] * Nb[jb] * w;
            for (int c = 0; c < 3; ++c) h[c] += k * cc[c];
            h[3] += k;
        }
    for (int c = 0; c < 3; ++c) x[c] = h[c] / h[3];
}

// Corner (ca, cb) of a face: its corner control point (clamped knots).
static void face_point(const ivr_patch_desc &P, int face, int ca, int cb, double x[3]) {
    face_surface(P, face, (double)ca, (double)cb, x);
}

// The distinct normalised breakpoints of a knot vector.
static std::vector<double> breakpoints(const ivr_patch_desc &P, int d) {
    const int p = P.degree[0], n = P.ncp[d];
    const double *t = P.knots[d];
    std::vector<double> u;
    for (int i = p; i <= n; ++i) {
        const double v = (t[i] - t[p]) / (t[n] - t[p]);
        if (u.empty() || v > u.back()) u.push_back(v);
    }
    return u;
}

static bool same_surface(const ivr_patch_desc &P1, int f1, const ivr_patch_desc &P2, int f2, double tol) {
    const int dn1 = f1 >> 1, dn2 = f2 >> 1;
    const int da1 = dn1 == 0 ? 1 : 0, db1 = dn1 == 2 ? 1 : 2, da2 = dn2 == 0 ? 1 : 0, db2 = dn2 == 2 ? 1 : 2;
    auto grid = [](std::vector<double> u, const std::vector<double> &v) {
        u.insert(u.end(), v.begin(), v.end());
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end(), [](double x, double y) { return std::fabs(x - y) < 1e-14; }),
                u.end());
        return u;
    };
    const std::vector<double> ga = grid(breakpoints(P1, da1), breakpoints(P2, da2));
    const std::vector<double> gb = grid(breakpoints(P1, db1), breakpoints(P2, db2));
    const int m = std::max(P1.degree[0], P2.degree[0]) + 2;
    for (size_t i = 0; i + 1 < ga.size(); ++i)
        for (size_t j = 0; j + 1 < gb.size(); ++j)
            for (int s = 0; s < m; ++s)
                for (int r = 0; r < m; ++r) {
                    const double a = ga[i] + (ga[i + 1] - ga[i]) * s / (m - 1);
                    const double b = gb[j] + (gb[j + 1] - gb[j]) * r / (m - 1);
                    double x1[3], x2[3];
                    face_surface(P1, f1, a, b, x1);
                    face_surface(P2, f2, a, b, x2);
                    for (int c = 0; c < 3; ++c)
                        if (!(std::fabs(x1[c] - x2[c]) <= tol)) return false;
                }
    return true;
}

// Basis tables: on knot span e of direction d, the p+1 non-zero basis functions
// as polynomials in x = (u - t_e) / (t_{e+1} - t_e); coefficients from their
// values at p+1 points of the span (Vandermonde solve in FP64).
static void basis_tables(const ivr_patch_desc &P, int d, std::vector<float> &out) {
    const int p = P.degree[0], n = P.ncp[d];
    const double *t = P.knots[d];
    const double t0 = t[p], t1 = t[n];
    for (int e = p; e < n; ++e) {
        const double a = (t[e] - t0) / (t1 - t0), b = (t[e + 1] - t0) / (t1 - t0);
        double V[4][4], rhs[4][4];
        for (int j = 0; j <= p; ++j) {
            const double x = p ? (double)j / p : 0.0;
            double pw = 1.0;
            for (int k = 0; k <= p; ++k, pw *= x) V[j][k] = pw;
            // evaluate inside the span (the right end belongs to it here)
            const double u = std::min(a + x * (b - a), b - 1e-13 * (b - a));
            int span;
            double N[4];
            host_basis(P.knots[d], n, p, std::max(u, a), span, N);
            // host_basis may land on an earlier span only for empty spans
            for (int i = 0; i <= p; ++i) rhs[j][i] = (span == e) ? N[i] : 0.0;
        }
        // solve V c_i = rhs[:, i] for every function i (Gaussian elimination)
        for (int i = 0; i <= p; ++i) {
            double M[4][5];
            for (int r = 0; r <= p; ++r) {
                for (int k = 0; k <= p; ++k) M[r][k] = V[r][k];
                M[r][p + 1] = rhs[r][i];
            }
            for (int c = 0; c <= p; ++c) {
                int piv = c;
                for (int r = c + 1; r <= p; ++r)
                    if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
                for (int k = 0; k <= p + 1; ++k) std::swap(M[c][k], M[piv][k]);
                for (int r = c + 1; r <= p; ++r) {
                    const double f = M[r][c] / M[c][c];
                    for (int k = c; k <= p + 1; ++k) M[r][k] -= f * M[c][k];
                }
            }
            double cf[4];
            for (int r = p; r >= 0; --r) {
                double s = M[r][p + 1];
                for (int k = r + 1; k <= p; ++k) s -= M[r][k] * cf[k];
                cf[r] = s / M[r][r];
            }
            for (int k = 0; k <= p; ++k) out.push_back((float)cf[k]);
        }
    }
}

static void blossom(const double *t, int s, int p, const double (*Q)[4], const double *args,
                    double out[4]) {
    double d[kMaxDegree + 1][4];
    for (int k = 0; k <= p; ++k)
        for (int c = 0; c < 4; ++c) d[k][c] = Q[k][c];
    for (int r = 1; r <= p; ++r) {
        const double u = args[r - 1];
        for (int i = s; i >= s - p + r; --i) {
            const int k = i - (s - p);
            const double alpha = (u - t[i]) / (t[i + p + 1 - r] - t[i]);
            for (int c = 0; c < 4; ++c) d[k][c] = (1.0 - alpha) * d[k - 1][c] + alpha * d[k][c];
        }
    }
    for (int c = 0; c < 4; ++c) out[c] = d[p][c];
}

// Bezier net (homogeneous, (p+1)^2, a fastest) of the face element on spans
// (sa, sb); hq(ia, jb) returns the homogeneous face control point.
template <typename HQ>
static void bezier_net(const double *ta, const double *tb, int sa, int sb, int p, HQ hq,
                       double (*net)[4]) {
    double tmp[(kMaxDegree + 1) * (kMaxDegree + 1)][4];
    double args[kMaxDegree];
    for (int jb = 0; jb <= p; ++jb) {        // along a, for each of the p+1 rows
        double row[kMaxDegree + 1][4];
        for (int ia = 0; ia <= p; ++ia) hq(sa - p + ia, sb - p + jb, row[ia]);
        for (int j = 0; j <= p; ++j) {
            for (int r = 0; r < p; ++r) args[r] = r < p - j ? ta[sa] : ta[sa + 1];
            blossom(ta, sa, p, row, args, tmp[jb * (p + 1) + j]);
        }
    }
    for (int ia = 0; ia <= p; ++ia) {        // then along b
        double col[kMaxDegree + 1][4];
        for (int jb = 0; jb <= p; ++jb)
            for (int c = 0; c < 4; ++c) col[jb][c] = tmp[jb * (p + 1) + ia][c];
        for (int j = 0; j <= p; ++j) {
            for (int r = 0; r < p; ++r) args[r] = r < p - j ? tb[sb] : tb[sb + 1];
            blossom(tb, sb, p, col, args, net[j * (p + 1) + ia]);
        }
    }
}

// Oriented box around the projected Bezier points of a face element (the
// element lies in their convex hull; positive weights keep this for NURBS).
// Axes: the averaged edge directions of the net in a and b, orthonormalised,
// and their normal; extents from projecting every point, padded.  Falls back
// to the coordinate axes if an edge direction degenerates.
// Box axes come from the four corner points (c00, c10 along a, c01 along b, c11).
template <typename Box3>
static void build_obb(Box3 &E, const std::vector<std::array<double, 3>> &pts, const double *c00,
                      const double *c10, const double *c01, const double *c11, double pad) {
    double u[3] = {0, 0, 0}, v[3] = {0, 0, 0};
    for (int q = 0; q < 3; ++q) {
        u[q] = 0.5 * (c10[q] - c00[q] + c11[q] - c01[q]);
        v[q] = 0.5 * (c01[q] - c00[q] + c11[q] - c10[q]);
    }
    auto norm = [](double *w) {
        double n = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        if (!(n > 0)) return false;
        for (int q = 0; q < 3; ++q) w[q] /= n;
        return true;
    };
    double ax[3][3];
    bool ok = norm(u);
    if (ok) {
        const double dv = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
        for (int q = 0; q < 3; ++q) v[q] -= dv * u[q];
        ok = norm(v);
    }
    if (ok) {
        for (int q = 0; q < 3; ++q) { ax[0][q] = u[q]; ax[1][q] = v[q]; }
        ax[2][0] = u[1] * v[2] - u[2] * v[1];
        ax[2][1] = u[2] * v[0] - u[0] * v[2];
        ax[2][2] = u[0] * v[1] - u[1] * v[0];
    } else {
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) ax[r][q] = r == q ? 1.0 : 0.0;
    }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (const auto &P : pts)
        for (int r = 0; r < 3; ++r) {
            const double pr = ax[r][0] * P[0] + ax[r][1] * P[1] + ax[r][2] * P[2];
            lo[r] = std::min(lo[r], pr);
            hi[r] = std::max(hi[r], pr);
        }
    for (int q = 0; q < 3; ++q) {
        double cq = 0;
        for (int r = 0; r < 3; ++r) cq += ax[r][q] * 0.5 * (lo[r] + hi[r]);
        E.c[q] = (float)cq;
    }
    for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) E.ax[r][q] = (float)ax[r][q];
        // pad also covers the FP32 rounding of the centre and the axes
        E.ext[r] = round_up(0.5 * (hi[r] - lo[r]) + pad);
    }
}

// A bound on the slope of an element's surface against its box plane: the
// largest ratio of normal to in-plane component over the edges of its Bezier
// net, times 3 (the surface tangents are positive combinations of the net's
// edges, and the two parameter directions need not be orthogonal), at most 1;
// 1 for a net with an edge that has no in-plane extent.
static float element_graze(const FaceElem &E, const std::vector<std::array<double, 3>> &pts, int p) {
    double g = 0.0;
    auto edge = [&](const std::array<double, 3> &P0, const std::array<double, 3> &P1) {
        double c[3];
        for (int r = 0; r < 3; ++r)
            c[r] = E.ax[r][0] * (P1[0] - P0[0]) + E.ax[r][1] * (P1[1] - P0[1]) + E.ax[r][2] * (P1[2] - P0[2]);
        const double inpl = std::sqrt(c[0] * c[0] + c[1] * c[1]);
        const double len = std::sqrt(inpl * inpl + c[2] * c[2]);
        if (len == 0.0) return;                       // coincident points: no direction
        g = std::max(g, inpl > 1e-9 * len ? std::fabs(c[2]) / inpl : 1e30);
    };
    for (int j = 0; j <= p; ++j)
        for (int i = 0; i < p; ++i) {
            edge(pts[j * (p + 1) + i], pts[j * (p + 1) + i + 1]);
            edge(pts[i * (p + 1) + j], pts[(i + 1) * (p + 1) + j]);
        }
    return (float)std::min(1.0, 3.0 * g);
}

// Degree elevation, exact: direction d of degree p < P is rewritten in degree P.
// Every distinct knot's multiplicity grows by P - p (the ends stay clamped), so
// the degree-P space on the new knots contains every old basis function; the
// new coefficients come from collocation at the new basis's Greville points
// (distinct, so the collocation matrix is regular; it is totally positive and
// banded, so it is solved by banded elimination without pivoting) and reproduce
// the old spline up to rounding.  H holds nch channels per control point,
// i fastest; n[] is updated.
static void elevate_direction(std::vector<double> &H, int nch, int n[3], int d, const double *t_old, int p,
                              int P, std::vector<double> &t_new) {
    const int n_old = n[d], nk_old = n_old + p + 1;
    t_new.clear();
    for (int i = 0; i < nk_old;) {
        int j = i;
        while (j < nk_old && t_old[j] == t_old[i]) ++j;
        for (int r = 0; r < (j - i) + (P - p); ++r) t_new.push_back(t_old[i]);
        i = j;
    }
    const int n_new = (int)t_new.size() - P - 1;
    const double t0 = t_new[P], t1 = t_new[n_new];
    // lines along d: stride and count of the other two directions
    const int stride = d == 0 ? 1 : (d == 1 ? n[0] : n[0] * n[1]);
    const int lines = n[0] * n[1] * n[2] / n_old;
    const int K = lines * nch;   // right-hand sides
    auto line_base = [&](int l) {   // first point of line l (old layout)
        const int inner = stride, outer = l / inner;
        return (l % inner) + outer * inner * n_old;
    };
    // band of the collocation matrix (row i: columns i-P .. i+P) and the
    // right-hand sides R[i][k] = sum_j N_j(xi_i) C_j[k]
    const int W = P;
    std::vector<double> A((size_t)n_new * (2 * W + 1), 0.0), R((size_t)n_new * K, 0.0);
    for (int i = 0; i < n_new; ++i) {
        double xi = 0.0;
        for (int r = 1; r <= P; ++r) xi += t_new[i + r];
        xi = (xi / P - t0) / (t1 - t0);
        int s_new, s_old;
        double M[kMaxDegree + 1], N[kMaxDegree + 1];
        host_basis(t_new.data(), n_new, P, xi, s_new, M);
        host_basis(t_old, n_old, p, xi, s_old, N);
        for (int r = 0; r <= P; ++r) {
            const int col = s_new - P + r;
            if (col - i >= -W && col - i <= W) A[(size_t)i * (2 * W + 1) + (col - i + W)] = M[r];
        }
        for (int r = 0; r <= p; ++r) {
            const int j = s_old - p + r;
            for (int l = 0; l < lines; ++l) {
                const double *src = &H[(size_t)(line_base(l) + j * stride) * nch];
                for (int c = 0; c < nch; ++c) R[(size_t)i * K + l * nch + c] += N[r] * src[c];
            }
        }
    }
    // banded elimination without pivoting, then back substitution
    auto a = [&](int r, int c) -> double & { return A[(size_t)r * (2 * W + 1) + (c - r + W)]; };
    for (int c = 0; c < n_new; ++c) {
        for (int r = c + 1; r <= std::min(n_new - 1, c + W); ++r) {
            const double f = a(r, c) / a(c, c);
            if (f == 0.0) continue;
            for (int k = c; k <= std::min(n_new - 1, c + W); ++k) a(r, k) -= f * a(c, k);
            for (int k = 0; k < K; ++k) R[(size_t)r * K + k] -= f * R[(size_t)c * K + k];
        }
    }
    for (int r = n_new - 1; r >= 0; --r) {
        for (int k = r + 1; k <= std::min(n_new - 1, r + W); ++k) {
            const double f = a(r, k);
            if (f == 0.0) continue;
            for (int q = 0; q < K; ++q) R[(size_t)r * K + q] -= f * R[(size_t)k * K + q];
        }
        const double inv = 1.0 / a(r, r);
        for (int q = 0; q < K; ++q) R[(size_t)r * K + q] *= inv;
    }
    // scatter back in the new layout
    int nn[3] = {n[0], n[1], n[2]};
    nn[d] = n_new;
    const int stride_new = d == 0 ? 1 : (d == 1 ? nn[0] : nn[0] * nn[1]);
    std::vector<double> Hn((size_t)nn[0] * nn[1] * nn[2] * nch);
    for (int l = 0; l < lines; ++l) {
        const int inner = stride_new, outer = l / inner;
        const int base = (l % inner) + outer * inner * n_new;
        for (int i = 0; i < n_new; ++i)
            for (int c = 0; c < nch; ++c) Hn[(size_t)(base + i * stride_new) * nch + c] = R[(size_t)i * K + l * nch + c];
    }
    H.swap(Hn);
    n[0] = nn[0]; n[1] = nn[1]; n[2] = nn[2];
}

// A block with the same spline in one degree (the largest of its directions) in
// all three directions; owns its arrays.
struct IsoPatch {
    std::vector<double> knots[3], cp, scalar, disp;
    ivr_patch_desc desc;
};

static void make_isotropic(const ivr_patch_desc &P, IsoPatch &out) {
    const int Pm = std::max(P.degree[0], std::max(P.degree[1], P.degree[2]));
    int n[3] = {P.ncp[0], P.ncp[1], P.ncp[2]};
    const size_t N = (size_t)n[0] * n[1] * n[2];
    // homogeneous channels (w x, w y, w z, w, w rho[, w u_x, w u_y, w u_z])
    const int NCH = P.displacement ? 8 : 5;
    std::vector<double> H(N * NCH);
    for (size_t q = 0; q < N; ++q) {
        const double w = P.rational ? P.cp[4 * q + 3] : 1.0;
        for (int c = 0; c < 3; ++c) H[NCH * q + c] = w * P.cp[4 * q + c];
        H[NCH * q + 3] = w;
        H[NCH * q + 4] = w * P.scalar[q];
        if (P.displacement)
            for (int c = 0; c < 3; ++c) H[NCH * q + 5 + c] = w * P.displacement[3 * q + c];
    }
    for (int d = 0; d < 3; ++d) {
        if (P.degree[d] == Pm) {
            out.knots[d].assign(P.knots[d], P.knots[d] + P.ncp[d] + P.degree[d] + 1);
        } else {
            elevate_direction(H, NCH, n, d, P.knots[d], P.degree[d], Pm, out.knots[d]);
        }
    }
    const size_t M = (size_t)n[0] * n[1] * n[2];
    out.cp.resize(4 * M);
    out.scalar.resize(M);
    if (P.displacement) out.disp.resize(3 * M);
    for (size_t q = 0; q < M; ++q) {
        const double w = H[NCH * q + 3];
        for (int c = 0; c < 3; ++c) out.cp[4 * q + c] = H[NCH * q + c] / w;
        out.cp[4 * q + 3] = P.rational ? w : 1.0;
        out.scalar[q] = H[NCH * q + 4] / w;
        if (P.displacement)
            for (int c = 0; c < 3; ++c) out.disp[3 * q + c] = H[NCH * q + 5 + c] / w;
    }
    out.desc = P;
    for (int d = 0; d < 3; ++d) {
        out.desc.degree[d] = Pm;
        out.desc.ncp[d] = n[d];
        out.desc.knots[d] = out.knots[d].data();
    }
    out.desc.cp = out.cp.data();
    out.desc.scalar = out.scalar.data();
    out.desc.displacement = P.displacement ? out.disp.data() : nullptr;
}

// Splits a block (one degree P in every direction) at every interior knot of
// multiplicity P, where the spline is only C0: the pieces share the control
// layer that the spline passes through there, so together they are the block.
// Pieces without such knots are appended to out (their arrays in store).
static void split_at_c0(const ivr_patch_desc &P, std::deque<IsoPatch> &store, std::vector<ivr_patch_desc> &out) {
    const int p = P.degree[0];
    for (int d = 0; d < 3; ++d) {
        const int n = P.ncp[d];
        const double *t = P.knots[d];
        for (int i = p + 1; i < n; ++i) {
            int mult = 1;
            while (i + mult < n && t[i + mult] == t[i]) ++mult;
            if (mult < p) {
                i += mult - 1;
                continue;
            }
            // knots t[i .. i+p-1] = u; the spline passes through control layer i-1
            const int n0 = P.ncp[0], n1 = P.ncp[1];
            int nl[3] = {P.ncp[0], P.ncp[1], P.ncp[2]}, nr[3] = {P.ncp[0], P.ncp[1], P.ncp[2]};
            nl[d] = i;
            nr[d] = n - i + 1;
            IsoPatch *piece[2];
            for (int side = 0; side < 2; ++side) {
                store.emplace_back();
                IsoPatch &Q = store.back();
                const int *nn = side ? nr : nl;
                const int off = side ? i - 1 : 0;
                for (int e = 0; e < 3; ++e) {
                    if (e != d) {
                        Q.knots[e].assign(P.knots[e], P.knots[e] + P.ncp[e] + p + 1);
                    } else if (side == 0) {
                        Q.knots[e].assign(t, t + i);
                        Q.knots[e].insert(Q.knots[e].end(), p + 1, t[i]);
                    } else {
                        Q.knots[e].assign(p + 1, t[i]);
                        Q.knots[e].insert(Q.knots[e].end(), t + i + p, t + n + p + 1);
                    }
                }
                const size_t N = (size_t)nn[0] * nn[1] * nn[2];
                Q.cp.resize(4 * N);
                Q.scalar.resize(N);
                if (P.displacement) Q.disp.resize(3 * N);
                for (int k = 0; k < nn[2]; ++k)
                    for (int j = 0; j < nn[1]; ++j)
                        for (int a = 0; a < nn[0]; ++a) {
                            int src[3] = {a, j, k};
                            src[d] += off;
                            const size_t si = (size_t)src[0] + (size_t)n0 * (src[1] + (size_t)n1 * src[2]);
                            const size_t di = (size_t)a + (size_t)nn[0] * (j + (size_t)nn[1] * k);
                            for (int c = 0; c < 4; ++c) Q.cp[4 * di + c] = P.cp[4 * si + c];
                            Q.scalar[di] = P.scalar[si];
                            if (P.displacement)
                                for (int c = 0; c < 3; ++c) Q.disp[3 * di + c] = P.displacement[3 * si + c];
                        }
                Q.desc = P;
                for (int e = 0; e < 3; ++e) {
                    Q.desc.ncp[e] = nn[e];
                    Q.desc.knots[e] = Q.knots[e].data();
                }
                Q.desc.cp = Q.cp.data();
                Q.desc.scalar = Q.scalar.data();
                Q.desc.displacement = P.displacement ? Q.disp.data() : nullptr;
                piece[side] = &Q;
            }
            split_at_c0(piece[0]->desc, store, out);
            split_at_c0(piece[1]->desc, store, out);
            return;
        }
    }
    out.push_back(P);
}

}  // namespace

extern "C" {

void ivr_default_opts(ivr_render_opts *o) {
    if (!o) return;
    o->precision = IVR_PRECISION_FP32;
    o->rk_tol = 1e-5;
    o->h_max = 0.0;
    o->c_perp = 1.0;
    o->n_super = 4;
    o->det_fp64_threshold = 1e-6;
    o->max_fragments = kFragCap;
    o->seed_mode = IVR_SEED_BOX;
    o->early_term = 1e-4;
    o->max_newton_iter = 16;
    o->rho_interp = IVR_RHO_HERMITE;
    o->timing = 0;
    o->tf_step = 0.025;
    o->rho_step = 0.1;
    o->cand_per_pixel = 8;
    o->det_singular = 1e-6;
    o->drift_tol = 1e-4;
    o->interior = IVR_INTERIOR_ODE;
    o->field = IVR_FIELD_SCALAR;
    o->newton_stop = IVR_NEWTON_STOP_TOL;
    o->cut = 0;
    for (int q = 0; q < 3; ++q) o->cut_point[q] = o->cut_normal[q] = 0.0;
    o->near_clip = 0.0;
}

static ivr_status ensure_views(ivr_ctx *c, int n);

ivr_status ivr_create(ivr_ctx **out, int32_t device, void *hip_stream) {
    if (!out) return IVR_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return IVR_EDEVICE;
    if (device < 0 || device >= ndev) return IVR_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return IVR_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return IVR_EDEVICE;
    ivr_ctx *c = new (std::nothrow) ivr_ctx();
    if (!c) return IVR_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->n_cu = prop.multiProcessorCount;
    if (hipSetDevice(device) != hipSuccess ||
        hipMalloc((void **)&c->d_qs, sizeof(QueueState)) != hipSuccess ||
        hipMalloc((void **)&c->d_ctr, sizeof(unsigned long long) * C_COUNT) != hipSuccess) {
        ivr_destroy(c);
        return IVR_ENOMEM;
    }
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            ivr_destroy(c);
            return IVR_EDEVICE;
        }
    if (hipEventCreateWithFlags(&c->views_copied, hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) {
        ivr_destroy(c);
        return IVR_EDEVICE;
    }
    // the view table and the pinned counter staging exist from the start, so that
    // ivr_render_noalloc allocates nothing
    if (hipHostMalloc((void **)&c->h_ctr, sizeof(unsigned long long) * C_COUNT) != hipSuccess ||
        hipHostMalloc((void **)&c->h_totals, 4 * sizeof(uint32_t), hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->d_totals, c->h_totals, 0) != hipSuccess || ensure_views(c, 8) != IVR_OK) {
        ivr_destroy(c);
        return IVR_ENOMEM;
    }
    if (device < kMaxDevices) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
                ivr_destroy(c);
                return IVR_EDEVICE;
            }
            g_scratch_ptr[device] = static_cast<unsigned char *>(p);
        }
        c->scratch = g_scratch_ptr[device];
    }
    *out = c;
    return IVR_OK;
}

const char *ivr_last_error(const ivr_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

static void free_model(ivr_ctx *c) {
    dfree(c->d_patches); dfree(c->d_cp32); dfree(c->d_rho32); dfree(c->d_cp64); dfree(c->d_rho64);
    dfree(c->d_disp32); dfree(c->d_disp64);
    dfree(c->d_knots32); dfree(c->d_knots64); dfree(c->d_elems); dfree(c->d_tiles); dfree(c->d_btab);
    dfree(c->d_pperm); dfree(c->d_pcount); dfree(c->d_pbase); dfree(c->d_pcur);
    c->has_model = false;
}

static void free_mlp(ivr_ctx *c) {
    dfree(c->mlp.w); dfree(c->mlp.m); dfree(c->mlp.v); dfree(c->mlp.wb); dfree(c->mlp.norm);
    c->mlp_trained = false;
}

static void drop_graphs(ivr_ctx *c) {
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
    ++c->generation;
}

static void free_cand_lists(ivr_ctx *c) {
    dfree(c->mq.query); dfree(c->mq.seed); dfree(c->mq.clist); dfree(c->mq.plist); dfree(c->mq.crange);
    c->mq.c_cap = 0;
    c->mq_tiles = 0;
}

static void free_frame(ivr_ctx *c) {
    drop_graphs(c);
    free_cand_lists(c);
    dfree(c->d_segs); dfree(c->d_pixseg); dfree(c->d_seg_kr); dfree(c->d_order);
    c->pix_cap = c->seg_cap = c->seg_bytes_cap = 0;
}

void ivr_destroy(ivr_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_model(c);
    free_frame(c);
    free_mlp(c);
    dfree(c->d_qs);
    dfree(c->d_ctr);
    dfree(c->d_views);
    if (c->h_views) (void)hipHostFree(c->h_views);
    if (c->h_ctr) (void)hipHostFree(c->h_ctr);
    if (c->h_totals) (void)hipHostFree(c->h_totals);
    if (c->d_desum) (void)hipFree(c->d_desum);
    if (c->views_copied) (void)hipEventDestroy(c->views_copied);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &e : c->tev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

ivr_status ivr_upload_patches(ivr_ctx *c, const ivr_patch_desc *patches, int32_t n) {
    return ivr_upload_models(c, patches, n, &n, 1);
}

ivr_status ivr_upload_models(ivr_ctx *c, const ivr_patch_desc *patches, int32_t n,
                             const int32_t *model_sizes, int32_t n_models) {
    if (!c) return IVR_EINVAL;
    if (!patches || n < 1) return fail(c, IVR_EINVAL, "need at least one patch");
    if (n > (int32_t)kPatchMask) return fail(c, IVR_EINVAL, "more than 2^20-1 patches");
    if (!model_sizes || n_models < 1) return fail(c, IVR_EINVAL, "need at least one model");
    std::vector<ivr_ctx::ModelRange> models(n_models);
    std::vector<int> model_of(n);
    {
        long long at = 0;
        for (int mi = 0; mi < n_models; ++mi) {
            if (model_sizes[mi] < 1) return fail(c, IVR_EINVAL, "every model needs at least one patch");
            models[mi].begin = (int)at;
            at += model_sizes[mi];
            if (at > n) return fail(c, IVR_EINVAL, "model sizes exceed the number of patches");
            models[mi].end = (int)at;
            for (int i = models[mi].begin; i < models[mi].end; ++i) model_of[i] = mi;
        }
        if (at != n) return fail(c, IVR_EINVAL, "model sizes must add up to the number of patches");
    }
    for (int i = 0; i < n; ++i) {
        std::string e = validate_patch(patches[i], i);
        if (!e.empty()) return fail(c, IVR_EINVAL, e);
    }
    // Blocks whose directions differ in degree are raised to their largest degree,
    // and blocks are split at interior knots of full multiplicity (where the map
    // and rho are only C0), both exactly: the kernels see one degree per block
    // and smooth blocks, joined at the splits as at any conforming interface.
    // Block indices from here on (segments, MLPs) are those of the split model.
    std::deque<IsoPatch> iso;
    std::vector<ivr_patch_desc> descs;
    {
        std::vector<int> sizes(n_models, 0);
        for (int i = 0; i < n; ++i) {
            ivr_patch_desc P = patches[i];
            if (P.degree[0] != P.degree[1] || P.degree[0] != P.degree[2]) {
                iso.emplace_back();
                make_isotropic(P, iso.back());
                P = iso.back().desc;
            }
            const size_t before = descs.size();
            split_at_c0(P, iso, descs);
            sizes[model_of[i]] += (int)(descs.size() - before);
        }
        if (descs.size() > kPatchMask) return fail(c, IVR_EINVAL, "more than 2^20-1 blocks after splitting");
        n = (int32_t)descs.size();
        model_of.assign(n, 0);
        int at = 0;
        for (int mi = 0; mi < n_models; ++mi) {
            models[mi].begin = at;
            at += sizes[mi];
            models[mi].end = at;
            for (int i = models[mi].begin; i < models[mi].end; ++i) model_of[i] = mi;
        }
    }
    patches = descs.data();
    IVR_HIP(c, hipSetDevice(c->device));
    // scale of each model: diagonal of the box of its (projected) control points
    for (auto &M : models) {
        Box all;
        for (int i = M.begin; i < M.end; ++i) {
            const auto &P = patches[i];
            const size_t N = (size_t)P.ncp[0] * P.ncp[1] * P.ncp[2];
            for (size_t q = 0; q < N; ++q) all.add(P.cp + 4 * q);
        }
        double diag = 0;
        for (int q = 0; q < 3; ++q) diag += (all.hi[q] - all.lo[q]) * (all.hi[q] - all.lo[q]);
        M.scale = std::max(std::sqrt(diag), 1e-30);
        M.class_mask = 0;
        for (int i = M.begin; i < M.end; ++i)
            M.class_mask |= 1u << (2 * (patches[i].degree[0] - 1) + (patches[i].rational ? 1 : 0));
    }
    const double scale = models[0].scale;

    std::vector<DevPatch> hp(n);
    std::vector<float4> cp32;
    std::vector<float> rho32, knots32;
    std::vector<double4> cp64;
    std::vector<double> rho64, knots64;
    std::vector<float4> disp32;
    std::vector<double4> disp64;
    size_t n_disp = 0;   // blocks with a displacement spline
    std::vector<FaceElem> elems;
    std::vector<FaceTile> tiles, subs;
    std::vector<float> btab;
    uint32_t class_mask = 0;
    for (int pi = 0; pi < n; ++pi) {
        const auto &P = patches[pi];
        DevPatch &D = hp[pi];
        std::memset(&D, 0, sizeof D);
        const double pad = 1e-5 * models[model_of[pi]].scale;
        const int p = P.degree[0];
        D.deg = p;
        D.rational = P.rational ? 1 : 0;
        D.klass = 2 * (p - 1) + D.rational;
        class_mask |= 1u << D.klass;
        D.cp_off = (int)cp32.size();
        D.orient = orientation(P);
        std::vector<double> tn[3];
        for (int d = 0; d < 3; ++d) {
            const int nd = P.ncp[d], nk = nd + p + 1;
            D.n[d] = nd;
            D.nspan[d] = nd - p;
            D.inv_nspan[d] = 1.0f / (float)(nd - p);
            const double *t = P.knots[d];
            const double t0 = t[p], t1 = t[nd];
            tn[d].resize(nk);
            for (int i = 0; i < nk; ++i) tn[d][i] = std::min(1.0, std::max(0.0, (t[i] - t0) / (t1 - t0)));
            bool uni = true;
            for (int i = p + 1; i < nd; ++i)
                if (std::fabs(tn[d][i] - (double)(i - p) / (nd - p)) > 1e-12) uni = false;
            if (uni) D.uniform |= 1 << d;
            D.knot_off[d] = (int)knots32.size();
            for (int i = 0; i < nk; ++i) {
                knots32.push_back((float)tn[d][i]);
                knots64.push_back(tn[d][i]);
            }
        }
        D.btab_off = (int)btab.size();
        for (int d = 0; d < 3; ++d) basis_tables(P, d, btab);
        D.btab_len = (int)btab.size() - D.btab_off;
        const int n0 = P.ncp[0], n1 = P.ncp[1], n2 = P.ncp[2];
        const size_t N = (size_t)n0 * n1 * n2;
        // the face evaluator addresses the nets by 32-bit byte offsets (32 B per FP64 point)
        if (cp32.size() + N > ((size_t)1 << 27))
            return fail(c, IVR_EOVERFLOW, "more than 2^27 control points");
        Box pb;
        for (size_t q = 0; q < N; ++q) {
            const double *cc = P.cp + 4 * q;
            const double w = P.rational ? cc[3] : 1.0;
            // homogeneous (wx, wy, wz, w) for NURBS; (x, y, z, rho) for B-splines
            const double w4 = P.rational ? w : P.scalar[q];
            cp32.push_back(make_float4((float)(w * cc[0]), (float)(w * cc[1]), (float)(w * cc[2]), (float)w4));
            cp64.push_back(make_double4(w * cc[0], w * cc[1], w * cc[2], w4));
            rho32.push_back((float)(w * P.scalar[q]));
            rho64.push_back(w * P.scalar[q]);
            // displacement as (w u, w); blocks without one hold zeros
            const double *u = P.displacement ? P.displacement + 3 * q : nullptr;
            const double du[3] = {u ? w * u[0] : 0.0, u ? w * u[1] : 0.0, u ? w * u[2] : 0.0};
            disp32.push_back(make_float4((float)du[0], (float)du[1], (float)du[2], (float)w));
            disp64.push_back(make_double4(du[0], du[1], du[2], w));
            pb.add(cc);
        }
        if (P.displacement) ++n_disp;
        pb.store(D.box, pad);
        auto idx = [&](int i, int j, int k) { return (size_t)i + (size_t)n0 * (j + (size_t)n1 * k); };
        for (int f = 0; f < 6; ++f) {
            const int dn = f >> 1, da = dn == 0 ? 1 : 0, db = dn == 2 ? 1 : 2;
            const int fix = (f & 1) ? P.ncp[dn] - 1 : 0;
            Box fb;
            D.elem_off[f] = (int)elems.size();
            auto at = [&](int ia, int jb) {
                int ijk[3];
                ijk[dn] = fix;
                ijk[da] = ia;
                ijk[db] = jb;
                return P.cp + 4 * idx(ijk[0], ijk[1], ijk[2]);
            };
            for (int jb = 0; jb < P.ncp[db]; ++jb)
                for (int ia = 0; ia < P.ncp[da]; ++ia) fb.add(at(ia, jb));
            fb.store(D.fbox[f], pad);
            std::vector<int> spa, spb;   // non-empty spans in a and b
            for (int sa = p; sa < P.ncp[da]; ++sa)
                if (tn[da][sa] < tn[da][sa + 1]) spa.push_back(sa);
            for (int sb = p; sb < P.ncp[db]; ++sb)
                if (tn[db][sb] < tn[db][sb + 1]) spb.push_back(sb);
            auto hq = [&](int ia, int jb, double *o) {
                const double *cc = at(ia, jb);
                const double w = P.rational ? cc[3] : 1.0;
                o[0] = w * cc[0]; o[1] = w * cc[1]; o[2] = w * cc[2]; o[3] = w;
            };
            D.tile_off[f] = (int)tiles.size();
            for (size_t tb = 0; tb < spb.size(); tb += kTile)
                for (size_t ta = 0; ta < spa.size(); ta += kTile) {
                    FaceTile T;
                    std::memset(&T, 0, sizeof T);
                    T.elem_begin = (int)elems.size();
                    T.sub_begin = (int)subs.size();
                    std::vector<std::array<double, 3>> tpts;
                    double corner[4][3];
                    const size_t ea1 = std::min(spa.size(), ta + kTile), eb1 = std::min(spb.size(), tb + kTile);
                    for (size_t sb0 = tb; sb0 < eb1; sb0 += 2)
                    for (size_t sa0 = ta; sa0 < ea1; sa0 += 2) {
                    FaceTile S;
                    std::memset(&S, 0, sizeof S);
                    S.elem_begin = (int)elems.size();
                    std::vector<std::array<double, 3>> spts;
                    double scorner[4][3];
                    const size_t sa1 = std::min(ea1, sa0 + 2), sb1 = std::min(eb1, sb0 + 2);
                    for (size_t ib = sb0; ib < sb1; ++ib)
                        for (size_t ia = sa0; ia < sa1; ++ia) {
                            const int sa = spa[ia], sb = spb[ib];
                            double net[(kMaxDegree + 1) * (kMaxDegree + 1)][4];
                            bezier_net(tn[da].data(), tn[db].data(), sa, sb, p, hq, net);
                            std::vector<std::array<double, 3>> pts;
                            for (int k = 0; k < (p + 1) * (p + 1); ++k)
                                pts.push_back({net[k][0] / net[k][3], net[k][1] / net[k][3], net[k][2] / net[k][3]});
                            FaceElem E;
                            std::memset(&E, 0, sizeof E);
                            build_obb(E, pts, pts[0].data(), pts[p].data(), pts[p * (p + 1)].data(),
                                      pts[(p + 1) * (p + 1) - 1].data(), pad);
                            E.graze = element_graze(E, pts, p);
                            E.a0 = (float)tn[da][sa];
                            E.a1 = (float)tn[da][sa + 1];
                            E.b0 = (float)tn[db][sb];
                            E.b1 = (float)tn[db][sb + 1];
                            E.face = f;
                            E.patch = pi;
                            elems.push_back(E);
                            tpts.insert(tpts.end(), pts.begin(), pts.end());
                            spts.insert(spts.end(), pts.begin(), pts.end());
                            if (ia == ta && ib == tb) std::memcpy(corner[0], pts[0].data(), sizeof corner[0]);
                            if (ia + 1 == ea1 && ib == tb) std::memcpy(corner[1], pts[p].data(), sizeof corner[1]);
                            if (ia == ta && ib + 1 == eb1) std::memcpy(corner[2], pts[p * (p + 1)].data(), sizeof corner[2]);
                            if (ia + 1 == ea1 && ib + 1 == eb1)
                                std::memcpy(corner[3], pts[(p + 1) * (p + 1) - 1].data(), sizeof corner[3]);
                            if (ia == sa0 && ib == sb0) std::memcpy(scorner[0], pts[0].data(), sizeof scorner[0]);
                            if (ia + 1 == sa1 && ib == sb0) std::memcpy(scorner[1], pts[p].data(), sizeof scorner[1]);
                            if (ia == sa0 && ib + 1 == sb1) std::memcpy(scorner[2], pts[p * (p + 1)].data(), sizeof scorner[2]);
                            if (ia + 1 == sa1 && ib + 1 == sb1)
                                std::memcpy(scorner[3], pts[(p + 1) * (p + 1) - 1].data(), sizeof scorner[3]);
                        }
                    S.elem_end = (int)elems.size();
                    build_obb(S, spts, scorner[0], scorner[1], scorner[2], scorner[3], pad);
                    subs.push_back(S);
                    }
                    T.elem_end = (int)elems.size();
                    T.sub_end = (int)subs.size();
                    if (T.sub_end - T.sub_begin <= 1) {   // one sub-tile: the tile itself
                        subs.resize(T.sub_begin);
                        T.sub_end = T.sub_begin;
                    }
                    build_obb(T, tpts, corner[0], corner[1], corner[2], corner[3], pad);
                    tiles.push_back(T);
                }
        }
        D.elem_off[6] = (int)elems.size();
        D.tile_off[6] = (int)tiles.size();
    }
    {   // sub-tiles after all tiles
        const int off = (int)tiles.size();
        for (auto &T : tiles) {
            T.sub_begin += off;
            T.sub_end += off;
        }
        tiles.insert(tiles.end(), subs.begin(), subs.end());
    }
    if (elems.size() > kCandElemMask)
        return fail(c, IVR_EOVERFLOW, "more than 2^26 face elements");
    // Faces shared by two blocks of a model: the same parametric surface S(a, b)
    // (as at conforming interfaces, also between blocks of different degree or
    // knots): test them from the first block only and emit the second block's
    // crossing from the same root.  Candidates share their four corners; the
    // surfaces are then compared at (p+2)^2 points of every span of the union of
    // both knot grids, which decides equality of the piecewise polynomials.
    {
        for (int pi = 0; pi < n; ++pi) {
            for (int f = 0; f < 6; ++f) hp[pi].twin[f] = -1;
            hp[pi].face_skip = 0;
        }
        std::map<std::vector<long long>, std::vector<int>> by_corners;
        for (int pi = 0; pi < n; ++pi) {
            const double q = 1e-9 * models[model_of[pi]].scale;
            for (int f = 0; f < 6; ++f) {
                std::vector<long long> key = {model_of[pi]};
                for (int cb = 0; cb < 2; ++cb)
                    for (int ca = 0; ca < 2; ++ca) {
                        double x[3];
                        face_point(patches[pi], f, ca, cb, x);
                        for (int c = 0; c < 3; ++c) key.push_back(std::llround(x[c] / q));
                    }
                by_corners[key].push_back(8 * pi + f);
            }
        }
        for (auto &kv : by_corners) {
            const auto &fl = kv.second;
            for (size_t i = 0; i < fl.size(); ++i) {
                const int p1 = fl[i] >> 3, f1 = fl[i] & 7;
                if (hp[p1].twin[f1] >= 0 || ((hp[p1].face_skip >> f1) & 1)) continue;
                for (size_t j = i + 1; j < fl.size(); ++j) {
                    const int p2 = fl[j] >> 3, f2 = fl[j] & 7;
                    if (p2 == p1 || hp[p2].twin[f2] >= 0 || ((hp[p2].face_skip >> f2) & 1)) continue;
                    if (!same_surface(patches[p1], f1, patches[p2], f2, 1e-10 * models[model_of[p1]].scale))
                        continue;
                    hp[p1].twin[f1] = 8 * p2 + f2;
                    hp[p2].face_skip |= 1 << f2;
                    break;
                }
            }
        }
    }
    // blocks grouped by degree class (stable), with each class's range and largest net
    std::vector<uint32_t> pperm;
    int cls_q[kClasses + 1] = {0}, cls_max_cp[kClasses] = {0}, cls_max_tab[kClasses] = {0};
    for (int k = 0; k < kClasses; ++k) {
        cls_q[k] = (int)pperm.size();
        for (int pi = 0; pi < n; ++pi)
            if (hp[pi].klass == k) {
                pperm.push_back((uint32_t)pi);
                cls_max_cp[k] = std::max(cls_max_cp[k], hp[pi].n[0] * hp[pi].n[1] * hp[pi].n[2]);
                cls_max_tab[k] = std::max(cls_max_tab[k], hp[pi].btab_len);
            }
    }
    cls_q[kClasses] = (int)pperm.size();
    const std::vector<uint32_t> zeros(n, 0u);
    // allocate and copy, then swap in
    ivr_ctx tmp;
    size_t model_bytes = 0;
    auto up = [&](auto *&dst, const auto &vec) -> bool {
        using T = typename std::remove_reference<decltype(vec)>::type::value_type;
        model_bytes += sizeof(T) * std::max<size_t>(vec.size(), 1);
        if (hipMalloc((void **)&dst, sizeof(T) * std::max<size_t>(vec.size(), 1)) != hipSuccess) return false;
        return hipMemcpy((void *)dst, vec.data(), sizeof(T) * vec.size(), hipMemcpyHostToDevice) == hipSuccess;
    };
    if (n_disp == 0) {   // no displacement anywhere: nothing to store
        disp32.clear();
        disp64.clear();
    }
    bool ok = up(tmp.d_patches, hp) && up(tmp.d_cp32, cp32) && up(tmp.d_rho32, rho32) &&
              up(tmp.d_disp32, disp32) && up(tmp.d_disp64, disp64) &&
              up(tmp.d_cp64, cp64) && up(tmp.d_rho64, rho64) && up(tmp.d_knots32, knots32) &&
              up(tmp.d_knots64, knots64) && up(tmp.d_elems, elems) && up(tmp.d_tiles, tiles) &&
              up(tmp.d_btab, btab) &&
              up(tmp.d_pperm, pperm) && up(tmp.d_pcount, zeros) && up(tmp.d_pbase, zeros) &&
              up(tmp.d_pcur, zeros);
    if (!ok) {
        free_model(&tmp);
        return fail(c, IVR_ENOMEM, "device allocation for the model failed");
    }
    IVR_HIP(c, hipStreamSynchronize(c->stream));
    free_model(c);
    free_mlp(c);
    c->hpatch = hp;
    c->d_patches = tmp.d_patches; c->d_cp32 = tmp.d_cp32; c->d_rho32 = tmp.d_rho32;
    c->d_cp64 = tmp.d_cp64; c->d_rho64 = tmp.d_rho64; c->d_knots32 = tmp.d_knots32;
    c->d_disp32 = tmp.d_disp32; c->d_disp64 = tmp.d_disp64;
    tmp.d_disp32 = nullptr; tmp.d_disp64 = nullptr;
    c->all_disp = n_disp == (size_t)n;
    c->d_knots64 = tmp.d_knots64; c->d_elems = tmp.d_elems; c->d_tiles = tmp.d_tiles;
    c->d_btab = tmp.d_btab;
    tmp.d_btab = nullptr;
    c->d_pperm = tmp.d_pperm; c->d_pcount = tmp.d_pcount; c->d_pbase = tmp.d_pbase; c->d_pcur = tmp.d_pcur;
    tmp.d_pperm = tmp.d_pcount = tmp.d_pbase = tmp.d_pcur = nullptr;
    std::copy(cls_q, cls_q + kClasses + 1, c->cls_q);
    std::copy(cls_max_cp, cls_max_cp + kClasses, c->cls_max_cp);
    std::copy(cls_max_tab, cls_max_tab + kClasses, c->cls_max_tab);
    tmp.d_tiles = nullptr;
    tmp.d_patches = nullptr; tmp.d_cp32 = nullptr; tmp.d_rho32 = nullptr; tmp.d_cp64 = nullptr;
    tmp.d_rho64 = nullptr; tmp.d_knots32 = nullptr; tmp.d_knots64 = nullptr; tmp.d_elems = nullptr;
    drop_graphs(c);
    c->npatch = n;
    c->model_bytes = model_bytes;
    c->nelem = (int)elems.size();
    c->scale = scale;
    c->class_mask = class_mask;
    c->models = models;
    c->has_model = true;
    c->err.clear();
    return IVR_OK;
}

static ivr_status make_frame(ivr_ctx *c, const ivr_camera *cam, const ivr_transfer_fn *tf,
                             const ivr_render_opts &o, double scale, FrameParams &fp) {
    std::memset(&fp, 0, sizeof fp);
    if (!cam || !tf) return fail(c, IVR_EINVAL, "camera and transfer function are required");
    if (cam->width < 1 || cam->height < 1 || cam->width > 16384 || cam->height > 16384)
        return fail(c, IVR_EINVAL, "image size outside 1..16384");
    if (!(cam->fov_y_deg > 0.0 && cam->fov_y_deg < 179.0))
        return fail(c, IVR_EINVAL, "fov_y_deg outside (0, 179)");
    if (!finite3(cam->eye) || !finite3(cam->target) || !finite3(cam->up))
        return fail(c, IVR_EINVAL, "camera vectors must be finite");
    double f[3], r[3], u[3];
    for (int q = 0; q < 3; ++q) f[q] = cam->target[q] - cam->eye[q];
    double nf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(nf > 0)) return fail(c, IVR_EINVAL, "eye equals target");
    for (int q = 0; q < 3; ++q) f[q] /= nf;
    r[0] = f[1] * cam->up[2] - f[2] * cam->up[1];
    r[1] = f[2] * cam->up[0] - f[0] * cam->up[2];
    r[2] = f[0] * cam->up[1] - f[1] * cam->up[0];
    double nr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(nr > 1e-12)) return fail(c, IVR_EINVAL, "up is parallel to the view direction");
    for (int q = 0; q < 3; ++q) r[q] /= nr;
    u[0] = r[1] * f[2] - r[2] * f[1];
    u[1] = r[2] * f[0] - r[0] * f[2];
    u[2] = r[0] * f[1] - r[1] * f[0];
    for (int q = 0; q < 3; ++q) {
        fp.eye[q] = cam->eye[q]; fp.fwd[q] = f[q]; fp.right[q] = r[q]; fp.up[q] = u[q];
        fp.eyef[q] = (float)cam->eye[q]; fp.fwdf[q] = (float)f[q]; fp.rightf[q] = (float)r[q]; fp.upf[q] = (float)u[q];
    }
    fp.tan_half = std::tan(0.5 * cam->fov_y_deg * M_PI / 180.0);
    fp.aspect = (double)cam->width / (double)cam->height;
    fp.tan_halff = (float)fp.tan_half;
    fp.aspectf = (float)fp.aspect;
    fp.width = cam->width;
    fp.height = cam->height;
    // transfer function
    const int nk = tf->n_knots;
    if (nk < 2 || nk > kMaxTfKnots || !tf->x || !tf->rgba)
        return fail(c, IVR_EINVAL, "transfer function needs 2..16 knots");
    if (tf->x[0] != 0.0 || tf->x[nk - 1] != 1.0)
        return fail(c, IVR_EINVAL, "transfer function knots must run from 0 to 1");
    for (int k = 0; k < nk; ++k) {
        if (!std::isfinite(tf->x[k]) || (k > 0 && !(tf->x[k] > tf->x[k - 1])))
            return fail(c, IVR_EINVAL, "transfer function knots must increase strictly");
        for (int q = 0; q < 4; ++q)
            if (!std::isfinite(tf->rgba[4 * k + q]))
                return fail(c, IVR_EINVAL, "transfer function values must be finite");
    }
    if (!(std::isfinite(tf->extinction) && tf->extinction >= 0))
        return fail(c, IVR_EINVAL, "extinction must be finite and >= 0");
    if (!(std::isfinite(tf->domain[0]) && std::isfinite(tf->domain[1]) && tf->domain[1] > tf->domain[0]))
        return fail(c, IVR_EINVAL, "transfer function domain must satisfy lo < hi");
    fp.tf_n = nk;
    for (int k = 0; k < nk; ++k) {
        double v[4];
        for (int q = 0; q < 4; ++q) v[q] = tf->rgba[4 * k + q];
        v[3] *= tf->extinction;
        fp.tf_xd[k] = tf->x[k];
        fp.tf_x[k] = (float)tf->x[k];
        for (int q = 0; q < 4; ++q) {
            fp.tf_vd[k][q] = v[q];
            fp.tf_v[k][q] = (float)v[q];
        }
        if (k + 1 < nk) {
            for (int q = 0; q < 4; ++q) {
                double v1 = tf->rgba[4 * (k + 1) + q] * (q == 3 ? tf->extinction : 1.0);
                double s = (v1 - v[q]) / (tf->x[k + 1] - tf->x[k]);
                fp.tf_sd[k][q] = s;
                fp.tf_s[k][q] = (float)s;
            }
        }
    }
    {   // supersampling resolution in n: half the smallest knot gap, within [1/64, 1/16]
        double gap = 1.0;
        for (int k = 0; k + 1 < nk; ++k) gap = std::min(gap, tf->x[k + 1] - tf->x[k]);
        const double dn = std::min(1.0 / 16.0, std::max(1.0 / 64.0, 0.5 * gap));
        fp.tf_dn = (float)dn;
    }
    {   // per-interval slope bound, widened to the neighbouring intervals
        double sm[kMaxTfKnots] = {0};
        for (int k = 0; k + 1 < nk; ++k)
            for (int q = 0; q < 4; ++q) sm[k] = std::max(sm[k], std::fabs(fp.tf_sd[k][q] / (q == 3 && tf->extinction > 0 ? tf->extinction : 1.0)));
        for (int k = 0; k + 1 < nk; ++k) {
            double v = sm[k];
            if (k > 0) v = std::max(v, sm[k - 1]);
            if (k + 2 < nk) v = std::max(v, sm[k + 1]);
            fp.tf_smax[k] = (float)v;
        }
    }
    fp.tf_lod = tf->domain[0];
    fp.tf_inv_ranged = 1.0 / (tf->domain[1] - tf->domain[0]);
    fp.tf_lo = (float)fp.tf_lod;
    fp.tf_inv_range = (float)fp.tf_inv_ranged;
    // integrator options
    if (o.precision != IVR_PRECISION_FP32 && o.precision != IVR_PRECISION_FP64)
        return fail(c, IVR_EINVAL, "unknown precision");
    if (!(o.rk_tol > 0 && std::isfinite(o.rk_tol))) return fail(c, IVR_EINVAL, "rk_tol must be > 0");
    if (!std::isfinite(o.h_max)) return fail(c, IVR_EINVAL, "h_max must be finite");
    if (!(o.c_perp >= 0 && std::isfinite(o.c_perp))) return fail(c, IVR_EINVAL, "c_perp must be >= 0");
    if (o.n_super < 1 || o.n_super > 64) return fail(c, IVR_EINVAL, "n_super outside 1..64");
    if (!(o.det_fp64_threshold >= 0)) return fail(c, IVR_EINVAL, "det_fp64_threshold must be >= 0");
    if (!(o.det_singular >= 0 && std::isfinite(o.det_singular)))
        return fail(c, IVR_EINVAL, "det_singular must be finite and >= 0");
    if (!(o.drift_tol >= 0 && std::isfinite(o.drift_tol)))
        return fail(c, IVR_EINVAL, "drift_tol must be finite and >= 0");
    if (o.interior < IVR_INTERIOR_ODE || o.interior > IVR_INTERIOR_IRK1)
        return fail(c, IVR_EINVAL, "unknown interior method");
    fp.interior = o.interior;
    if (!(o.near_clip >= 0 && std::isfinite(o.near_clip))) return fail(c, IVR_EINVAL, "near_clip must be >= 0");
    fp.near_clip = o.near_clip;
    fp.cut = o.cut ? 1 : 0;
    if (o.cut) {
        if (!finite3(o.cut_point) || !finite3(o.cut_normal)) return fail(c, IVR_EINVAL, "cutting plane not finite");
        const double nn = std::sqrt(o.cut_normal[0] * o.cut_normal[0] + o.cut_normal[1] * o.cut_normal[1] +
                                    o.cut_normal[2] * o.cut_normal[2]);
        if (!(nn > 0)) return fail(c, IVR_EINVAL, "cutting plane normal is zero");
        fp.cut_s0 = 0.0;
        for (int q = 0; q < 3; ++q) {
            fp.cut_n[q] = o.cut_normal[q] / nn;
            fp.cut_s0 += fp.cut_n[q] * (cam->eye[q] - o.cut_point[q]);
        }
    }
    if (o.max_fragments < 2 || o.max_fragments > kFragCap)
        return fail(c, IVR_EINVAL, "max_fragments outside 2..64");
    if (o.rho_interp != IVR_RHO_LINEAR && o.rho_interp != IVR_RHO_HERMITE)
        return fail(c, IVR_EINVAL, "unknown rho_interp");
    if (o.seed_mode != IVR_SEED_PLAIN && o.seed_mode != IVR_SEED_MLP && o.seed_mode != IVR_SEED_BOX)
        return fail(c, IVR_EINVAL, "unknown seed_mode");
    if (o.seed_mode == IVR_SEED_MLP && !c->mlp_trained)
        return fail(c, IVR_ESTATE, "no inverse-map MLP has been trained");
    fp.seed_mode = o.seed_mode;
    if (!(o.early_term >= 0 && o.early_term < 1)) return fail(c, IVR_EINVAL, "early_term outside [0,1)");
    if (!(o.tf_step > 0 && std::isfinite(o.tf_step))) return fail(c, IVR_EINVAL, "tf_step must be > 0");
    fp.tf_step = (float)o.tf_step;
    if (!(o.rho_step > 0 && std::isfinite(o.rho_step))) return fail(c, IVR_EINVAL, "rho_step must be > 0");
    fp.rho_step = (float)o.rho_step;
    if (o.max_newton_iter < 1 || o.max_newton_iter > 100)
        return fail(c, IVR_EINVAL, "max_newton_iter outside 1..100");
    const double hmax = o.h_max > 0 ? o.h_max : scale / 32.0;
    const double hmin = std::min(hmax, 1.5625e-6 * scale);
    double tol = o.rk_tol;
    if (o.precision == IVR_PRECISION_FP32) tol = std::max(tol, 32.0 * 1.1920929e-7);
    fp.rk_told = tol; fp.rk_tol = (float)tol;
    fp.h_maxd = hmax; fp.h_max = (float)hmax;
    fp.h_mind = hmin; fp.h_min = (float)hmin;
    fp.c_perpd = o.c_perp; fp.c_perp = (float)o.c_perp;
    fp.early_termd = o.early_term; fp.early_term = (float)o.early_term;
    fp.det_thrd = o.det_fp64_threshold; fp.det_thr = (float)o.det_fp64_threshold;
    fp.det_singd = o.det_singular; fp.det_sing = (float)o.det_singular;
    fp.drift_told = o.drift_tol; fp.drift_tol = (float)o.drift_tol;   // relative to the model's scale
    fp.n_super = o.n_super;
    fp.max_frag = o.max_fragments;
    fp.hermite = o.rho_interp == IVR_RHO_HERMITE ? 1 : 0;
    if (o.field < IVR_FIELD_SCALAR || o.field > IVR_FIELD_VON_MISES) return fail(c, IVR_EINVAL, "unknown field");
    if (o.field != IVR_FIELD_SCALAR) {
        if (o.interior != IVR_INTERIOR_ODE && o.interior != IVR_INTERIOR_RF)
            return fail(c, IVR_EINVAL, "derived fields need the ODE or RF interior method");
        if (o.field == IVR_FIELD_VON_MISES && !c->all_disp)
            return fail(c, IVR_EINVAL, "von Mises needs a displacement spline on every block");
    }
    fp.field = o.field;
    if (o.newton_stop != IVR_NEWTON_STOP_TOL && o.newton_stop != IVR_NEWTON_STOP_FRUSTUM)
        return fail(c, IVR_EINVAL, "unknown newton_stop");
    fp.newton_stop = o.newton_stop;
    fp.max_newton = o.max_newton_iter;
    fp.scaled = scale;
    fp.scale = (float)scale;
    return IVR_OK;
}

static ivr_status ensure_frame(ivr_ctx *c, size_t pixels, size_t seg_cap, bool fp64) {
    const size_t seg_bytes = seg_cap * (fp64 ? sizeof(Seg<double>) : sizeof(Seg<float>));
    if (pixels <= c->pix_cap && seg_cap <= c->seg_cap && seg_bytes <= c->seg_bytes_cap) return IVR_OK;
    IVR_HIP(c, hipStreamSynchronize(c->stream));
    free_frame(c);
    if (hipMalloc(&c->d_segs, seg_bytes) != hipSuccess ||
        hipMalloc((void **)&c->d_pixseg, sizeof(uint2) * pixels) != hipSuccess ||
        hipMalloc((void **)&c->d_seg_kr, sizeof(uint2) * seg_cap) != hipSuccess ||
        hipMalloc((void **)&c->d_order, sizeof(uint32_t) * seg_cap) != hipSuccess) {
        free_frame(c);
        return fail(c, IVR_ENOMEM, "frame buffer allocation failed");
    }
    c->pix_cap = pixels;
    c->seg_cap = seg_cap;
    c->seg_bytes_cap = seg_bytes;
    return IVR_OK;
}

// Buffers of the two-pass fragment kernel: `want` candidates (a lane keeps at
// most 64), with their network queries and seeds when MLP seeds are used; at
// least 1024.  Rays whose candidates do not fit are traversed again by the solve
// pass (box seeds).
static ivr_status ensure_cand_lists(ivr_ctx *c, size_t want, size_t tiles, bool mlp) {
    const size_t cap = std::max<size_t>(want, 1024);
    if (tiles <= c->mq_tiles && cap <= c->mq.c_cap && (!mlp || c->mq.query)) return IVR_OK;
    IVR_HIP(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    free_cand_lists(c);
    if (cap > 0xFFFFFFFEull || tiles * 64 > 0xFFFFFFFFull)
        return fail(c, IVR_EOVERFLOW, "batch too large for the candidate buffers");
    if ((mlp && (hipMalloc((void **)&c->mq.query, sizeof(float4) * cap) != hipSuccess ||
                 hipMalloc((void **)&c->mq.seed, sizeof(float4) * cap) != hipSuccess)) ||
        hipMalloc((void **)&c->mq.clist, sizeof(uint2) * cap) != hipSuccess ||
        hipMalloc((void **)&c->mq.plist, sizeof(uint32_t) * cap) != hipSuccess ||
        hipMalloc((void **)&c->mq.crange, sizeof(uint2) * tiles * 64) != hipSuccess) {
        free_cand_lists(c);
        return fail(c, IVR_ENOMEM, "candidate buffer allocation failed");
    }
    c->mq.c_cap = (uint32_t)cap;
    c->mq_tiles = tiles;
    return IVR_OK;
}

static ivr_status ensure_views(ivr_ctx *c, int n) {
    if (n <= c->view_cap) return IVR_OK;
    IVR_HIP(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    dfree(c->d_views);
    if (c->h_views) (void)hipHostFree(c->h_views);
    c->h_views = nullptr;
    c->view_cap = 0;
    const int cap = std::max(n, 8);
    if (hipMalloc((void **)&c->d_views, sizeof(ViewRec) * cap) != hipSuccess ||
        hipHostMalloc((void **)&c->h_views, sizeof(ViewRec) * cap) != hipSuccess) {
        dfree(c->d_views);
        c->h_views = nullptr;
        return fail(c, IVR_ENOMEM, "view table allocation failed");
    }
    c->view_cap = cap;
    return IVR_OK;
}

// The segment and candidate totals of the last frame that the merge kernel has
// written to host memory (no waiting; a frame still in flight shows an earlier
// one): the per-pixel ratios that size the next frame's buffers.
static void poll_counts(ivr_ctx *c) {
    const volatile uint32_t *t = c->h_totals;
    const uint32_t segs = t[0], cands = t[1], pixels = t[2];
    if (pixels == 0) return;
    c->seg_ratio = std::max(c->seg_ratio, (double)segs / (double)pixels);
    c->cand_ratio = std::max(c->cand_ratio, (double)cands / (double)pixels);
}

static Model device_model(ivr_ctx *c) {
    Model m;
    m.patches = c->d_patches; m.cp32 = c->d_cp32; m.rho32 = c->d_rho32; m.cp64 = c->d_cp64;
    m.rho64 = c->d_rho64; m.knots32 = c->d_knots32; m.knots64 = c->d_knots64; m.elems = c->d_elems;
    m.disp32 = c->d_disp32; m.disp64 = c->d_disp64;
    m.tiles = c->d_tiles;
    m.btab = c->d_btab;
    m.mlp_wb = c->mlp.wb;
    m.mlp_norm = c->mlp.norm;
    m.npatch = c->npatch; m.scale = (float)c->scale; m.scaled = c->scale;
    return m;
}

namespace {
struct HostView {
    const ivr_camera *cam;
    const ivr_transfer_fn *tf;
    int model;
    float *rgba, *depth;
    uint32_t *flags;
    float *dp;
};
struct Batch {
    int n = 0;
    int method = IVR_INTERIOR_ODE;
    int field = IVR_FIELD_SCALAR;
    bool diag = false;    // some view records the pixel accuracy
    uint32_t n_tiles = 0, n_pixels = 0, class_mask = 0;
    bool fp64 = false, mlp = false, collect = false;
    uint32_t c_cap = 0;   // candidates the fragment launches may record
};
}  // namespace

// Device buffers of one frame: the context's grow-only buffers, or the carve-up of
// the scratch array used by ivr_render_noalloc.
struct FrameBufs {
    void *segs = nullptr;
    size_t seg_cap = 0;
    uint2 *pixseg = nullptr, *seg_kr = nullptr;
    uint32_t *order = nullptr;
    QueueState *qs = nullptr;
    unsigned long long *ctr = nullptr;
    uint32_t *pcount = nullptr, *pbase = nullptr, *pcur = nullptr;
    CandLists mq = {nullptr, nullptr, nullptr, nullptr, nullptr, 0};   // c_cap: what may be recorded
    ViewRec *views = nullptr;
    uint32_t *totals = nullptr;           // host-mapped frame totals, or null
};

// Validates the views and fills the pinned view table (at most view_cap views);
// sizes of the batch in b.  Allocates nothing.
static ivr_status fill_views(ivr_ctx *c, const HostView *hv, int n, const ivr_render_opts &o,
                             bool collect, const LaunchCfg &lc, Batch &b) {
    if (!c->has_model) return fail(c, IVR_ESTATE, "no model uploaded");
    if (n < 1 || n > 64) return fail(c, IVR_EINVAL, "a batch holds 1..64 views");
    if (n > c->view_cap) return fail(c, IVR_EINVAL, "more views than the view table holds");
    IVR_HIP(c, hipSetDevice(c->device));
    // the staging buffer is still being read by the previous batch's copy
    IVR_HIP(c, hipEventSynchronize(c->views_copied));
    b = Batch();
    b.n = n;
    b.fp64 = o.precision == IVR_PRECISION_FP64;
    b.mlp = o.seed_mode == IVR_SEED_MLP;
    b.method = o.interior;
    b.field = o.field;
    b.collect = collect;
    const int th = 64 / lc.tile_w;
    uint64_t tiles = 0, pixels = 0;
    for (int v = 0; v < n; ++v) {
        if (!hv[v].rgba) return fail(c, IVR_EINVAL, "a view has no rgba buffer");
        if (hv[v].model < 0 || hv[v].model >= (int)c->models.size())
            return fail(c, IVR_EINVAL, "a view names a model that was not uploaded");
        const auto &M = c->models[hv[v].model];
        ViewRec &r = c->h_views[v];
        std::memset(&r, 0, sizeof r);
        ivr_status st = make_frame(c, hv[v].cam, hv[v].tf, o, M.scale, r.fp);
        if (st != IVR_OK) return st;
        r.fp.collect = collect ? 1 : 0;
        r.patch_begin = M.begin;
        r.patch_end = M.end;
        r.tiles_x = (uint32_t)((hv[v].cam->width + lc.tile_w - 1) / lc.tile_w);
        r.tile_begin = (uint32_t)tiles;
        r.pix_begin = (uint32_t)pixels;
        r.rgba = hv[v].rgba;
        r.depth = hv[v].depth;
        r.flags = hv[v].flags;
        r.dp = hv[v].dp;
        if (hv[v].dp) b.diag = true;
        tiles += (uint64_t)r.tiles_x * ((hv[v].cam->height + th - 1) / th);
        pixels += (uint64_t)hv[v].cam->width * hv[v].cam->height;
        b.class_mask |= M.class_mask;
    }
    if (b.diag && (b.field != IVR_FIELD_SCALAR || (b.method != IVR_INTERIOR_ODE && b.method != IVR_INTERIOR_RF)))
        return fail(c, IVR_EINVAL, "the pixel-accuracy record needs the scalar field and the ODE or RF method");
    if (pixels > 0xFFFFFFFFull || tiles > 0x3FFFFFFull)
        return fail(c, IVR_EOVERFLOW, "batch too large for 32-bit pixel and lane indices");
    if (o.cand_per_pixel < 0 || o.cand_per_pixel > kCandCap)
        return fail(c, IVR_EINVAL, "cand_per_pixel outside 0..64");
    int nint = 0;
    for (int v = 0; v < n; ++v) nint = std::max(nint, c->h_views[v].fp.tf_n - 2);
    for (int v = 0; v < n; ++v) c->h_views[v].fp.tf_nint_max = nint;
    b.n_tiles = (uint32_t)tiles;
    b.n_pixels = (uint32_t)pixels;
    return IVR_OK;
}

// The context's own frame buffers for batch b (grown as needed).
static ivr_status prepare_batch(ivr_ctx *c, const HostView *hv, int n, const ivr_render_opts &o,
                                bool collect, const LaunchCfg &lc, Batch &b, FrameBufs &fb) {
    if (n < 1 || n > 64) return fail(c, IVR_EINVAL, "a batch holds 1..64 views");
    ivr_status st = ensure_views(c, n);
    if (st != IVR_OK) return st;
    st = fill_views(c, hv, n, o, collect, lc, b);
    if (st != IVR_OK) return st;
    // Segment slots: 2.5 per pixel, or 1.2 times the most per pixel a render of
    // this context needed (at most 32 per pixel, the cap per ray); candidates: 2 per
    // pixel or 1.25 times the most needed, at most cand_per_pixel.  A render whose
    // segments do not fit drops and counts them (segment_overflow, per-pixel
    // flags) and makes the next call grow the buffers.
    poll_counts(c);
    const double px = (double)b.n_pixels;
    const double seg_pp = std::min((double)kSegCap, std::max(2.5, 1.2 * c->seg_ratio));
    const double slots = std::max(std::ceil(px * seg_pp), (double)(1u << 20));
    if (slots > 4294967040.0) return fail(c, IVR_EOVERFLOW, "batch too large for 32-bit segment indices");
    st = ensure_frame(c, b.n_pixels, (size_t)slots, b.fp64);
    if (st != IVR_OK) return st;
    const size_t limit = (size_t)b.n_pixels * (size_t)o.cand_per_pixel;
    const double cand_pp = std::max(2.0, 1.25 * c->cand_ratio);
    st = ensure_cand_lists(c, std::min(limit, (size_t)std::ceil(px * cand_pp)), b.n_tiles, b.mlp);
    if (st != IVR_OK) return st;
    b.c_cap = (uint32_t)std::min<size_t>(limit, c->mq.c_cap);
    fb = FrameBufs();
    fb.segs = c->d_segs;
    fb.seg_cap = c->seg_cap;
    fb.pixseg = c->d_pixseg;
    fb.seg_kr = c->d_seg_kr;
    fb.order = c->d_order;
    fb.qs = c->d_qs;
    fb.ctr = c->d_ctr;
    fb.pcount = c->d_pcount;
    fb.pbase = c->d_pbase;
    fb.pcur = c->d_pcur;
    fb.mq = c->mq;
    fb.mq.c_cap = b.c_cap;
    fb.views = c->d_views;
    fb.totals = c->d_totals;
    return IVR_OK;
}

// The launches of one batch: clear, fragments, one integrator per degree class, merge.
static ivr_status launch_batch(ivr_ctx *c, const Batch &b, const FrameBufs &fb, const LaunchCfg &lc,
                               hipEvent_t *ev, hipStream_t s) {
    const Model m = device_model(c);
    IVR_HIP(c, launch_clear(fb.qs, fb.ctr, b.collect, fb.pcount, c->npatch, s));
    if (b.diag) IVR_HIP(c, launch_dp_clear(fb.views, b.n, b.n_pixels, s));
    if (ev) IVR_HIP(c, hipEventRecord(ev[0], s));
    IVR_HIP(c, launch_fragments(b.fp64, b.mlp, m, fb.views, b.n, b.n_tiles, lc, fb.segs, (uint32_t)fb.seg_cap,
                                fb.seg_kr, fb.pcount, fb.qs, fb.pixseg, fb.mq, fb.ctr, c->n_cu, s));
    IVR_HIP(c, launch_block_sort(fb.qs, (uint32_t)fb.seg_cap, fb.seg_kr, c->d_pperm, c->npatch, fb.pcount,
                                 fb.pbase, fb.pcur, fb.order, c->n_cu, s));
    // the fragment phase ends after the (short) block sort, so that the
    // integrator phase is the integrator launches alone
    if (ev) IVR_HIP(c, hipEventRecord(ev[1], s));
    for (int k = 0; k < kClasses; ++k) {
        if (!((b.class_mask >> k) & 1)) continue;
        IntegrateArgs ia;
        ia.order = fb.order;
        ia.pperm = c->d_pperm;
        ia.q_begin = c->cls_q[k];
        ia.q_end = c->cls_q[k + 1];
        ia.pbase = fb.pbase;
        ia.pcount = fb.pcount;
        ia.pcur = fb.pcur;
        ia.max_cp = c->cls_max_cp[k];
        ia.max_tab = c->cls_max_tab[k];
        IVR_HIP(c, launch_integrate(b.fp64, b.method, b.field, b.diag, k, m, fb.views, b.n, fb.segs, ia, fb.ctr,
                                    c->n_cu, lc, s));
    }
    if (ev) IVR_HIP(c, hipEventRecord(ev[2], s));
    IVR_HIP(c, launch_merge(fb.views, b.n, b.n_pixels, fb.pixseg, fb.segs, b.fp64, fb.qs, fb.totals, s));
    if (ev) IVR_HIP(c, hipEventRecord(ev[3], s));
    return IVR_OK;
}

static ivr_status copy_views(ivr_ctx *c, int n, ViewRec *dst) {
    IVR_HIP(c, hipMemcpyAsync(dst, c->h_views, sizeof(ViewRec) * n, hipMemcpyHostToDevice, c->stream));
    IVR_HIP(c, hipEventRecord(c->views_copied, c->stream));
    return IVR_OK;
}

// Counters of the last render (fb.ctr) into *stats through the pinned staging
// buffer, and the phase times from the stats events.  Waits for the stream.
static ivr_status read_stats(ivr_ctx *c, const unsigned long long *ctr, ivr_stats *stats) {
    IVR_HIP(c, hipMemcpyAsync(c->h_ctr, ctr, sizeof(unsigned long long) * C_COUNT, hipMemcpyDeviceToHost,
                              c->stream));
    IVR_HIP(c, hipStreamSynchronize(c->stream));
    std::memset(stats, 0, sizeof *stats);
    uint64_t *dst = &stats->rays;
    for (int k = 0; k < C_COUNT; ++k) dst[k] = c->h_ctr[k];
    float ms;
    IVR_HIP(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    stats->ms_fragments = ms;
    IVR_HIP(c, hipEventElapsedTime(&ms, c->ev[1], c->ev[2]));
    stats->ms_integrate = ms;
    IVR_HIP(c, hipEventElapsedTime(&ms, c->ev[2], c->ev[3]));
    stats->ms_merge = ms;
    return IVR_OK;
}

// Events of this render: the stats set, or the next timing slot, or none.
static ivr_status pick_events(ivr_ctx *c, bool stats, bool timing, hipEvent_t *&ev) {
    ev = nullptr;
    if (stats) {
        ev = c->ev;
    } else if (timing) {
        if (c->n_timed >= 4096) return fail(c, IVR_EOVERFLOW, "more than 4096 timed renders pending");
        while ((int)c->tev.size() < 4 * (c->n_timed + 1)) {
            hipEvent_t e;
            IVR_HIP(c, hipEventCreate(&e));
            c->tev.push_back(e);
        }
        ev = &c->tev[4 * c->n_timed];
        ++c->n_timed;
    }
    return IVR_OK;
}

// Direct launches (no graph) of a batch of host views.
// With stats the call is synchronous anyway: a render whose segments did not fit
// the buffers is run once more after they have grown.
static ivr_status render_direct(ivr_ctx *c, const HostView *hv, int n, const ivr_render_opts &o,
                                ivr_stats *stats, const LaunchCfg &lc) {
    for (int attempt = 0;; ++attempt) {
        Batch b;
        FrameBufs fb;
        ivr_status st = prepare_batch(c, hv, n, o, stats != nullptr, lc, b, fb);
        if (st != IVR_OK) return st;
        hipEvent_t *ev;
        st = pick_events(c, stats != nullptr, o.timing != 0, ev);
        if (st != IVR_OK) return st;
        st = copy_views(c, n, fb.views);
        if (st != IVR_OK) return st;
        st = launch_batch(c, b, fb, lc, ev, c->stream);
        if (st != IVR_OK) return st;
        if (!stats) return IVR_OK;
        st = read_stats(c, fb.ctr, stats);
        if (st != IVR_OK) return st;
        poll_counts(c);   // the stream has finished: the totals are here
        if (c->h_totals[0] <= fb.seg_cap || attempt > 0) return IVR_OK;
    }
}

ivr_status ivr_render(ivr_ctx *c, const ivr_camera *cam, const ivr_transfer_fn *tf,
                      const ivr_render_opts *opts, float *rgba_dev, float *depth_dev, ivr_stats *stats) {
    if (!c) return IVR_EINVAL;
    if (!rgba_dev) return fail(c, IVR_EINVAL, "rgba_dev is NULL");
    ivr_render_opts o;
    ivr_default_opts(&o);
    if (opts) o = *opts;
    const HostView hv = {cam, tf, 0, rgba_dev, depth_dev, nullptr};
    ivr_status st = render_direct(c, &hv, 1, o, stats, c->lc);
    if (st == IVR_OK) c->err.clear();
    return st;
}

// ivr_render without allocation: the frame buffers are carved out of this
// device's scratch array.  Every call on the device shares the array.
ivr_status ivr_render_noalloc(ivr_ctx *c, const ivr_camera *cam, const ivr_transfer_fn *tf,
                              const ivr_render_opts *opts, float *rgba_dev, float *depth_dev,
                              ivr_stats *stats) {
    if (!c) return IVR_EINVAL;
    if (!rgba_dev) return fail(c, IVR_EINVAL, "rgba_dev is NULL");
    if (!c->scratch) return fail(c, IVR_EDEVICE, "no scratch array on this device");
    ivr_render_opts o;
    ivr_default_opts(&o);
    if (opts) o = *opts;
    if (o.timing) return fail(c, IVR_EINVAL, "timing events are not available without allocation");
    if (cam && (uint64_t)cam->width * (uint64_t)cam->height > kNoAllocMaxPixels)
        return fail(c, IVR_EOVERFLOW, "more than 1048576 pixels for the scratch array");
    if (c->has_model && c->npatch > kNoAllocMaxBlocks)
        return fail(c, IVR_EOVERFLOW, "more than 65536 blocks for the scratch array");
    const HostView hv = {cam, tf, 0, rgba_dev, depth_dev, nullptr};
    Batch b;
    ivr_status st = fill_views(c, &hv, 1, o, stats != nullptr, c->lc, b);
    if (st != IVR_OK) return st;
    // carve the array: fixed parts first, then a quarter of the rest for the
    // candidate list and the remainder for segment slots
    unsigned char *const base = c->scratch;
    size_t off = 0;
    auto take = [&](size_t bytes) -> unsigned char * {
        off = (off + 255) & ~size_t(255);
        unsigned char *p = base + off;
        off += bytes;
        return p;
    };
    FrameBufs fb;
    fb.views = reinterpret_cast<ViewRec *>(take(sizeof(ViewRec)));
    fb.qs = reinterpret_cast<QueueState *>(take(sizeof(QueueState)));
    fb.ctr = reinterpret_cast<unsigned long long *>(take(sizeof(unsigned long long) * C_COUNT));
    fb.pcount = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * c->npatch));
    fb.pbase = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * c->npatch));
    fb.pcur = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * c->npatch));
    fb.pixseg = reinterpret_cast<uint2 *>(take(sizeof(uint2) * b.n_pixels));
    fb.mq.crange = reinterpret_cast<uint2 *>(take(sizeof(uint2) * 64 * (size_t)b.n_tiles));
    const size_t slack = 8 * 256;   // alignment of the arrays still to come
    if (off + slack >= kScratchBytes) return fail(c, IVR_EOVERFLOW, "view too large for the scratch array");
    const size_t rest = kScratchBytes - off - slack;
    const size_t cand_bytes = sizeof(uint2) + sizeof(uint32_t) + (b.mlp ? 2 * sizeof(float4) : 0);
    const size_t c_cap = std::min<size_t>((size_t)b.n_pixels * (size_t)o.cand_per_pixel, rest / 4 / cand_bytes);
    fb.mq.clist = reinterpret_cast<uint2 *>(take(sizeof(uint2) * c_cap));
    fb.mq.plist = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * c_cap));
    if (b.mlp) {
        fb.mq.query = reinterpret_cast<float4 *>(take(sizeof(float4) * c_cap));
        fb.mq.seed = reinterpret_cast<float4 *>(take(sizeof(float4) * c_cap));
    }
    fb.mq.c_cap = (uint32_t)c_cap;
    const size_t seg_bytes = b.fp64 ? sizeof(Seg<double>) : sizeof(Seg<float>);
    const size_t slot = seg_bytes + sizeof(uint2) + sizeof(uint32_t);
    const size_t left = kScratchBytes - std::min(kScratchBytes, off + slack);
    fb.seg_cap = std::min<size_t>((size_t)b.n_pixels * kSegCap, left / slot);
    fb.segs = take(seg_bytes * fb.seg_cap);
    fb.seg_kr = reinterpret_cast<uint2 *>(take(sizeof(uint2) * fb.seg_cap));
    fb.order = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * fb.seg_cap));
    if (off > kScratchBytes || fb.seg_cap == 0)
        return fail(c, IVR_EOVERFLOW, "view too large for the scratch array");
    b.c_cap = (uint32_t)c_cap;
    st = copy_views(c, 1, fb.views);
    if (st != IVR_OK) return st;
    st = launch_batch(c, b, fb, c->lc, stats ? c->ev : nullptr, c->stream);
    if (st != IVR_OK) return st;
    if (stats) {
        st = read_stats(c, fb.ctr, stats);
        if (st != IVR_OK) return st;
    }
    c->err.clear();
    return IVR_OK;
}

ivr_status ivr_render_batch(ivr_ctx *c, const ivr_view *views, int32_t n_views,
                            const ivr_transfer_fn *tf, const ivr_render_opts *opts, ivr_stats *stats) {
    if (!c) return IVR_EINVAL;
    if (!views || n_views < 1 || n_views > 64) return fail(c, IVR_EINVAL, "a batch holds 1..64 views");
    ivr_render_opts o;
    ivr_default_opts(&o);
    if (opts) o = *opts;
    std::vector<HostView> hv(n_views);
    for (int v = 0; v < n_views; ++v) {
        hv[v] = {&views[v].cam, views[v].tf ? views[v].tf : tf, views[v].model, views[v].rgba_dev,
                 views[v].depth_dev, views[v].flags_dev, views[v].dp_dev};
        if (!hv[v].tf) return fail(c, IVR_EINVAL, "a view has no transfer function");
    }
    ivr_status st;
    if (stats || o.timing) {
        // counters and phase events need the launches one by one
        st = render_direct(c, hv.data(), n_views, o, stats, c->lc);
        if (st == IVR_OK) c->err.clear();
        return st;
    }
    Batch b;
    FrameBufs fb;
    st = prepare_batch(c, hv.data(), n_views, o, false, c->lc, b, fb);
    if (st != IVR_OK) return st;
    // the graph holds every kernel argument except what the view table carries
    // (cameras, transfer functions, output pointers): key it by the rest
    std::vector<int64_t> key = {(int64_t)c->generation, b.n, b.fp64, b.mlp, b.method, b.field, b.diag,
                                (int64_t)b.class_mask,
                                c->lc.tile_w, c->lc.xcd_chunk, c->lc.int_block, c->lc.int_waves_cu,
                                (int64_t)b.c_cap};
    for (int v = 0; v < n_views; ++v) {
        key.push_back(hv[v].cam->width);
        key.push_back(hv[v].cam->height);
        key.push_back(hv[v].model);
    }
    st = copy_views(c, n_views, fb.views);
    if (st != IVR_OK) return st;
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        // captured on the context's private stream (the render stream may be the
        // null stream, which cannot capture), replayed on the render stream
        hipGraph_t g = nullptr;
        IVR_HIP(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
        st = launch_batch(c, b, fb, c->lc, nullptr, c->capture);
        hipError_t e = hipStreamEndCapture(c->capture, &g);
        if (st != IVR_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return fail(c, IVR_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t ge = nullptr;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return fail(c, IVR_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        it = c->graphs.emplace(key, ge).first;
    }
    IVR_HIP(c, hipGraphLaunch(it->second, c->stream));
    c->err.clear();
    return IVR_OK;
}

ivr_status ivr_autotune(ivr_ctx *c, const ivr_view *views, int32_t n_views, const ivr_transfer_fn *tf,
                        const ivr_render_opts *opts, ivr_tune_report *report) {
    if (!c) return IVR_EINVAL;
    if (!views || n_views < 1 || n_views > 64) return fail(c, IVR_EINVAL, "a batch holds 1..64 views");
    ivr_render_opts o;
    ivr_default_opts(&o);
    if (opts) o = *opts;
    o.timing = 0;
    std::vector<HostView> hv(n_views);
    for (int v = 0; v < n_views; ++v) {
        hv[v] = {&views[v].cam, views[v].tf ? views[v].tf : tf, views[v].model, views[v].rgba_dev,
                 views[v].depth_dev, views[v].flags_dev, views[v].dp_dev};
        if (!hv[v].tf) return fail(c, IVR_EINVAL, "a view has no transfer function");
    }
    // time a shape: best of `reps` batches, per phase, from the stats events
    auto measure = [&](const LaunchCfg &lc, double &ms_frag, double &ms_int) -> ivr_status {
        ms_frag = ms_int = INFINITY;
        for (int r = 0; r < 3; ++r) {
            ivr_stats s;
            ivr_status st = render_direct(c, hv.data(), n_views, o, &s, lc);
            if (st != IVR_OK) return st;
            ms_frag = std::min(ms_frag, s.ms_fragments);
            ms_int = std::min(ms_int, s.ms_integrate);
        }
        return IVR_OK;
    };
    ivr_tune_report rep;
    std::memset(&rep, 0, sizeof rep);
    LaunchCfg best = c->lc;
    double f0, i0;
    ivr_status st = measure(best, f0, i0);   // also warms up
    if (st != IVR_OK) return st;
    st = measure(best, f0, i0);
    if (st != IVR_OK) return st;
    rep.ms_before = f0 + i0;
    // fragment kernel: tile shape and tile order (its time does not depend on the
    // integrator's shape, nor the integrator's on these)
    double bf = f0;
    for (int tw : {8, 16, 32})
        for (int xo : {0, 4, 16}) {
            LaunchCfg lc = best;
            lc.tile_w = tw;
            lc.xcd_chunk = xo;
            double f, i;
            st = measure(lc, f, i);
            if (st != IVR_OK) return st;
            if (rep.n_tried < 32) rep.tried_ms[rep.n_tried++] = f;
            if (f < bf) {
                bf = f;
                best.tile_w = tw;
                best.xcd_chunk = xo;
            }
        }
    // integrator: workgroup size and resident waves per CU (the queue consumers)
    double bi = INFINITY;
    for (int blk : {64, 128, 256})
        for (int wpc : {0, 16, 8}) {
            LaunchCfg lc = best;
            lc.int_block = blk;
            lc.int_waves_cu = wpc;
            double f, i;
            st = measure(lc, f, i);
            if (st != IVR_OK) return st;
            if (rep.n_tried < 32) rep.tried_ms[rep.n_tried++] = i;
            if (i < bi) {
                bi = i;
                best.int_block = blk;
                best.int_waves_cu = wpc;
            }
        }
    c->lc = best;
    drop_graphs(c);
    rep.tile_w = best.tile_w;
    rep.tile_h = 64 / best.tile_w;
    rep.xcd_chunk = best.xcd_chunk;
    rep.int_block = best.int_block;
    rep.int_waves_cu = best.int_waves_cu;
    rep.ms_after = bf + bi;
    if (report) *report = rep;
    c->err.clear();
    return IVR_OK;
}

ivr_status ivr_delta_e2000(ivr_ctx *c, const float *a, const float *b, int64_t n, const double *background,
                           double threshold, float *de_dev, ivr_delta_e_summary *summary) {
    if (!c) return IVR_EINVAL;
    if (!a || !b || n < 0) return fail(c, IVR_EINVAL, "images are NULL or n_pixels < 0");
    if (summary) *summary = ivr_delta_e_summary{0.0, 0.0, 0};
    if (n == 0) return IVR_OK;
    const double bg[3] = {background ? background[0] : 1.0, background ? background[1] : 1.0,
                          background ? background[2] : 1.0};
    if (summary) {
        if (!c->d_desum && hipMalloc((void **)&c->d_desum, sizeof(DeltaESum)) != hipSuccess)
            return fail(c, IVR_ENOMEM, "device allocation failed");
        IVR_HIP(c, hipMemsetAsync(c->d_desum, 0, sizeof(DeltaESum), c->stream));
    }
    IVR_HIP(c, launch_delta_e(a, b, (uint64_t)n, bg, threshold, de_dev, summary ? c->d_desum : nullptr, c->n_cu,
                              c->stream));
    if (summary) {
        DeltaESum h;
        IVR_HIP(c, hipMemcpyAsync(&h, c->d_desum, sizeof h, hipMemcpyDeviceToHost, c->stream));
        IVR_HIP(c, hipStreamSynchronize(c->stream));
        float mx;
        std::memcpy(&mx, &h.max_bits, sizeof mx);
        summary->max = mx;
        summary->mean = h.sum / (double)n;
        summary->over = h.over;
    }
    c->err.clear();
    return IVR_OK;
}

ivr_status ivr_device_bytes(ivr_ctx *c, uint64_t *model_bytes, uint64_t *frame_bytes) {
    if (!c) return IVR_EINVAL;
    const size_t tiles = c->mq_tiles;
    const size_t frame = c->seg_bytes_cap + c->seg_cap * (sizeof(uint2) + sizeof(uint32_t)) +
                         c->pix_cap * sizeof(uint2) +
                         (size_t)c->mq.c_cap * ((c->mq.query ? 2 * sizeof(float4) : 0) + sizeof(uint2) + sizeof(uint32_t)) +
                         tiles * 64 * sizeof(uint2);
    if (model_bytes) *model_bytes = c->model_bytes;
    if (frame_bytes) *frame_bytes = frame;
    return IVR_OK;
}

ivr_status ivr_set_launch(ivr_ctx *c, int32_t tile_w, int32_t xcd_chunk, int32_t int_block,
                          int32_t int_waves_cu) {
    if (!c) return IVR_EINVAL;
    if (tile_w != 8 && tile_w != 16 && tile_w != 32) return fail(c, IVR_EINVAL, "tile_w must be 8, 16 or 32");
    if (int_block != 64 && int_block != 128 && int_block != 256)
        return fail(c, IVR_EINVAL, "int_block must be 64, 128 or 256");
    if (int_waves_cu < 0 || int_waves_cu > 64) return fail(c, IVR_EINVAL, "int_waves_cu outside 0..64");
    if (xcd_chunk < 0 || xcd_chunk > 4096) return fail(c, IVR_EINVAL, "xcd_chunk outside 0..4096");
    c->lc = {tile_w, xcd_chunk, int_block, int_waves_cu};
    drop_graphs(c);
    c->err.clear();
    return IVR_OK;
}

// ---------------------------------------------------------------- learned initialiser

static uint32_t host_pcg_hash(uint32_t v) {   // same published hash as the device side
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

void ivr_default_mlp_opts(ivr_mlp_opts *o) {
    if (!o) return;
    o->samples_per_patch = 65536;
    o->steps = 2000;
    o->lr = 1e-3;
    o->seed = 5005;
    o->log_every = 100;
    o->batch = kMlpBatch;
}

static Model model_of(ivr_ctx *c) {
    Model m;
    std::memset(&m, 0, sizeof m);
    m.patches = c->d_patches; m.cp32 = c->d_cp32; m.rho32 = c->d_rho32; m.cp64 = c->d_cp64;
    m.rho64 = c->d_rho64; m.knots32 = c->d_knots32; m.knots64 = c->d_knots64; m.elems = c->d_elems;
    m.tiles = c->d_tiles; m.btab = c->d_btab; m.mlp_wb = c->mlp.wb; m.mlp_norm = c->mlp.norm;
    m.disp32 = c->d_disp32; m.disp64 = c->d_disp64;
    m.npatch = c->npatch; m.scale = (float)c->scale; m.scaled = c->scale;
    return m;
}

ivr_status ivr_train_inverse_mlp(ivr_ctx *c, const ivr_mlp_opts *opts, ivr_mlp_report *report) {
    if (!c) return IVR_EINVAL;
    if (!c->has_model) return fail(c, IVR_ESTATE, "no model uploaded");
    ivr_mlp_opts o;
    ivr_default_mlp_opts(&o);
    if (opts) o = *opts;
    if (o.samples_per_patch < kMlpBatch || o.samples_per_patch > (1 << 22))
        return fail(c, IVR_EINVAL, "samples_per_patch outside 128..4194304");
    if (o.steps < 1 || o.steps > 1000000) return fail(c, IVR_EINVAL, "steps outside 1..1000000");
    if (!(o.lr > 0 && o.lr < 1)) return fail(c, IVR_EINVAL, "lr outside (0,1)");
    if (o.log_every < 1) return fail(c, IVR_EINVAL, "log_every must be >= 1");
    if (o.batch < 16 || o.batch > kMlpBatch || o.batch % 16)
        return fail(c, IVR_EINVAL, "batch must be a multiple of 16 in 16..128");
    IVR_HIP(c, hipSetDevice(c->device));
    const int np = c->npatch;
    free_mlp(c);
    const size_t nw = (size_t)np * kMlpStride;
    if (hipMalloc((void **)&c->mlp.w, nw * 4) != hipSuccess || hipMalloc((void **)&c->mlp.m, nw * 4) != hipSuccess ||
        hipMalloc((void **)&c->mlp.v, nw * 4) != hipSuccess || hipMalloc((void **)&c->mlp.wb, (size_t)np * kMlpWbStride * 2) != hipSuccess ||
        hipMalloc((void **)&c->mlp.norm, (size_t)np * 12 * 4) != hipSuccess) {
        free_mlp(c);
        return fail(c, IVR_ENOMEM, "MLP allocation failed");
    }
    // Glorot-uniform initialisation (biases 0) from the hash of (seed, block, index)
    std::vector<float> hw(nw, 0.0f), hn((size_t)np * 12, 0.0f);
    for (int q = 0; q < np; ++q) {
        float *W = hw.data() + (size_t)q * kMlpStride;
        auto uni = [&](int idx, float a) {
            const uint32_t h = host_pcg_hash(o.seed ^ host_pcg_hash((uint32_t)q * 0x9E3779B9u ^ host_pcg_hash((uint32_t)idx)));
            return a * (2.0f * ((float)(h >> 8) * (1.0f / 16777216.0f)) - 1.0f);
        };
        const float a1 = std::sqrt(6.0f / (3 + 64)), a2 = std::sqrt(6.0f / (64 + 64)), a3 = std::sqrt(6.0f / (64 + 3));
        for (int i = 0; i < 192; ++i) W[kOffW1 + i] = uni(kOffW1 + i, a1);
        for (int i = 0; i < 4096; ++i) W[kOffW2 + i] = uni(kOffW2 + i, a2);
        for (int i = 0; i < 192; ++i) W[kOffW3 + i] = uni(kOffW3 + i, a3);
        const float *box = c->hpatch[q].box;
        for (int d = 0; d < 3; ++d) {
            const float half = std::max(0.5f * (box[3 + d] - box[d]), 1e-20f);
            hn[12 * q + d] = box[d];
            hn[12 * q + 3 + d] = 1.0f / half;
            hn[12 * q + 6 + d] = 0.5f * (box[3 + d] + box[d]);
        }
    }
    IVR_HIP(c, hipMemcpy(c->mlp.w, hw.data(), nw * 4, hipMemcpyHostToDevice));
    IVR_HIP(c, hipMemset(c->mlp.m, 0, nw * 4));
    IVR_HIP(c, hipMemset(c->mlp.v, 0, nw * 4));
    IVR_HIP(c, hipMemcpy(c->mlp.norm, hn.data(), hn.size() * 4, hipMemcpyHostToDevice));
    const int ns = o.samples_per_patch, nhold = 4096;
    const int nlog = std::min(64, (o.steps + o.log_every - 1) / o.log_every);
    float4 *xs = nullptr, *ps = nullptr, *hx = nullptr, *hpz = nullptr;
    float *loss = nullptr, *err = nullptr;
    auto cleanup = [&]() { dfree(xs); dfree(ps); dfree(hx); dfree(hpz); dfree(loss); dfree(err); };
    if (hipMalloc((void **)&xs, (size_t)np * ns * 16) != hipSuccess || hipMalloc((void **)&ps, (size_t)np * ns * 16) != hipSuccess ||
        hipMalloc((void **)&hx, (size_t)np * nhold * 16) != hipSuccess || hipMalloc((void **)&hpz, (size_t)np * nhold * 16) != hipSuccess ||
        hipMalloc((void **)&loss, (size_t)np * std::max(nlog, 1) * 4) != hipSuccess ||
        hipMalloc((void **)&err, (size_t)np * nhold * 4) != hipSuccess) {
        cleanup();
        free_mlp(c);
        return fail(c, IVR_ENOMEM, "MLP sample allocation failed");
    }
    const Model m = model_of(c);
    MlpTrainParams tp;
    tp.steps = o.steps; tp.samples = ns; tp.log_every = o.log_every; tp.npatch = np; tp.batch = o.batch;
    tp.lr = (float)o.lr; tp.beta1 = 0.9f; tp.beta2 = 0.999f; tp.eps = 1e-8f; tp.seed = o.seed * 2654435761u + 17u;
    hipError_t e = hipEventRecord(c->ev[0], c->stream);
    if (e == hipSuccess) e = launch_mlp_samples(m, c->mlp, np, ns, o.seed, xs, ps, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[1], c->stream);
    if (e == hipSuccess) e = launch_mlp_train(c->mlp, tp, xs, ps, loss, nlog, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev[2], c->stream);
    if (e == hipSuccess) e = launch_mlp_samples(m, c->mlp, np, nhold, o.seed ^ 0x5A5A5A5Au, hx, hpz, c->stream);
    if (e == hipSuccess) e = launch_mlp_heldout(c->mlp, np, nhold, hx, hpz, err, c->stream);
    std::vector<float> herr((size_t)np * nhold), hloss((size_t)np * std::max(nlog, 1));
    if (e == hipSuccess) e = hipMemcpyAsync(herr.data(), err, herr.size() * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hloss.data(), loss, hloss.size() * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        cleanup();
        free_mlp(c);
        return fail(c, IVR_EDEVICE, std::string("MLP training: ") + hipGetErrorString(e));
    }
    if (report) {
        std::memset(report, 0, sizeof *report);
        report->n_loss = nlog;
        for (int k = 0; k < nlog; ++k) {
            double acc = 0;
            for (int q = 0; q < np; ++q) acc += hloss[(size_t)q * nlog + k];
            report->loss[k] = (float)(acc / np);
        }
        double sum = 0, mx = 0;
        for (float v : herr) { sum += v; mx = std::max(mx, (double)v); }
        report->heldout_mean_err = sum / herr.size();
        report->heldout_max_err = mx;
        float ms = 0;
        if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) report->ms_samples = ms;
        if (hipEventElapsedTime(&ms, c->ev[1], c->ev[2]) == hipSuccess) report->ms_train = ms;
    }
    cleanup();
    c->mlp_trained = true;
    c->err.clear();
    drop_graphs(c);   // the graphs hold the MLP weight pointers
    return IVR_OK;
}

ivr_status ivr_mlp_forward_backward(ivr_ctx *c, const float *params, const float *x, const float *p,
                                    int32_t n, float *loss, float *grad) {
    if (!c || !params || !x || !p || !loss || !grad) return fail(c, IVR_EINVAL, "NULL argument");
    if (n < 16 || n > kMlpBatch || n % 16) return fail(c, IVR_EINVAL, "n must be a multiple of 16 in 16..128");
    IVR_HIP(c, hipSetDevice(c->device));
    float *dw = nullptr, *dx = nullptr, *dp = nullptr, *dout = nullptr;
    auto cleanup = [&]() { dfree(dw); dfree(dx); dfree(dp); dfree(dout); };
    if (hipMalloc((void **)&dw, kMlpStride * 4) != hipSuccess || hipMalloc((void **)&dx, n * 12) != hipSuccess ||
        hipMalloc((void **)&dp, n * 12) != hipSuccess || hipMalloc((void **)&dout, (kMlpParams + 1) * 4) != hipSuccess) {
        cleanup();
        return fail(c, IVR_ENOMEM, "allocation failed");
    }
    MlpState st = {dw, nullptr, nullptr, nullptr, nullptr};
    MlpTrainParams tp;
    std::memset(&tp, 0, sizeof tp);
    tp.batch = n;
    hipError_t e = hipMemcpy(dw, params, kMlpParams * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dx, x, n * 12, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dp, p, n * 12, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_mlp_grad(st, tp, dx, dp, dout, c->stream);
    std::vector<float> out(kMlpParams + 1);
    if (e == hipSuccess) e = hipMemcpyAsync(out.data(), dout, out.size() * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    cleanup();
    if (e != hipSuccess) return fail(c, IVR_EDEVICE, std::string("MLP gradient: ") + hipGetErrorString(e));
    std::memcpy(grad, out.data(), kMlpParams * 4);
    *loss = out[kMlpParams];
    return IVR_OK;
}

ivr_status ivr_mlp_get_weights(ivr_ctx *c, int32_t patch, float *out) {
    if (!c || !out) return IVR_EINVAL;
    if (!c->mlp_trained) return fail(c, IVR_ESTATE, "no inverse-map MLP has been trained");
    if (patch < 0 || patch >= c->npatch) return fail(c, IVR_EINVAL, "patch out of range");
    IVR_HIP(c, hipSetDevice(c->device));
    IVR_HIP(c, hipStreamSynchronize(c->stream));
    IVR_HIP(c, hipMemcpy(out, c->mlp.w + (size_t)patch * kMlpStride, kMlpParams * 4, hipMemcpyDeviceToHost));
    return IVR_OK;
}

ivr_status ivr_mlp_infer(ivr_ctx *c, const int32_t *patch, const float *x, int32_t n, float *p_out) {
    if (!c || !patch || !x || !p_out || n < 1) return fail(c, IVR_EINVAL, "bad arguments");
    if (!c->mlp_trained) return fail(c, IVR_ESTATE, "no inverse-map MLP has been trained");
    for (int i = 0; i < n; ++i)
        if (patch[i] < 0 || patch[i] >= c->npatch) return fail(c, IVR_EINVAL, "patch out of range");
    IVR_HIP(c, hipSetDevice(c->device));
    int *dq = nullptr;
    float *dx = nullptr, *dp = nullptr;
    auto cleanup = [&]() { dfree(dq); dfree(dx); dfree(dp); };
    if (hipMalloc((void **)&dq, (size_t)n * 4) != hipSuccess || hipMalloc((void **)&dx, (size_t)n * 12) != hipSuccess ||
        hipMalloc((void **)&dp, (size_t)n * 12) != hipSuccess) {
        cleanup();
        return fail(c, IVR_ENOMEM, "allocation failed");
    }
    hipError_t e = hipMemcpy(dq, patch, (size_t)n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dx, x, (size_t)n * 12, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_mlp_infer(c->mlp, dq, dx, n, dp, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(p_out, dp, (size_t)n * 12, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    cleanup();
    if (e != hipSuccess) return fail(c, IVR_EDEVICE, std::string("MLP inference: ") + hipGetErrorString(e));
    return IVR_OK;
}

ivr_status ivr_phase_times(ivr_ctx *c, double *ms_out, int32_t cap, int32_t *n_out) {
    if (!c || !n_out || cap < 0 || (cap > 0 && !ms_out)) return fail(c, IVR_EINVAL, "bad arguments");
    IVR_HIP(c, hipSetDevice(c->device));
    const int n = c->n_timed;
    for (int r = 0; r < n && r < cap; ++r) {
        IVR_HIP(c, hipEventSynchronize(c->tev[4 * r + 3]));
        for (int k = 0; k < 3; ++k) {
            float ms = 0.f;
            IVR_HIP(c, hipEventElapsedTime(&ms, c->tev[4 * r + k], c->tev[4 * r + k + 1]));
            ms_out[3 * r + k] = ms;
        }
    }
    *n_out = n;
    c->n_timed = 0;
    c->err.clear();
    return IVR_OK;
}

}  // extern "C"
