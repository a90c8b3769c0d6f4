/*
 * FP64 CPU oracle — TEST INFRASTRUCTURE ONLY (see ivr_oracle.h).
 *
 * Plain, slow, obviously-correct definitions.  Every function names the passage
 * of the paper it follows.  Nothing here is blocked, fused or reordered beyond
 * what the definition states; the only shortcuts are skipping terms that are
 * exactly zero (local support of B-splines, bounding boxes that the ray misses).
 */
#include "ivr_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define MAXP 3                         /* highest supported degree            */
#define MAXN 4096                      /* highest control-point count per dir */
#define FRAG_CAP 1024

/* ------------------------------------------------------------------ basis
 * Eq. (Bspline): "the recursively defined i-th B-spline of degree p".
 * Cox-de Boor recursion with 0/0 := 0.  Degree-0 functions are indicator
 * functions of half-open knot intervals, except that the last non-empty
 * interval is closed so the basis is complete at u = 1.                     */
static double cox_de_boor(const double *t, int nk, int i, int p, double u)
{
    if (p == 0) {
        if (t[i] <= u && u < t[i + 1]) return 1.0;
        if (u == t[nk - 1] && t[i] < t[i + 1] && t[i + 1] == t[nk - 1]) return 1.0;
        return 0.0;
    }
    if (u < t[i] || u > t[i + p + 1]) return 0.0;     /* outside the support */
    double r = 0.0;
    double d1 = t[i + p] - t[i], d2 = t[i + p + 1] - t[i + 1];
    if (d1 > 0.0) r += (u - t[i]) / d1 * cox_de_boor(t, nk, i, p - 1, u);
    if (d2 > 0.0) r += (t[i + p + 1] - u) / d2 * cox_de_boor(t, nk, i + 1, p - 1, u);
    return r;
}

/* Derivative of the recursively defined basis:
   N'_{i,p} = p/(t_{i+p}-t_i) N_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) N_{i+1,p-1}. */
static double cox_de_boor_deriv(const double *t, int nk, int i, int p, double u)
{
    if (p == 0) return 0.0;
    if (u < t[i] || u > t[i + p + 1]) return 0.0;
    double r = 0.0;
    double d1 = t[i + p] - t[i], d2 = t[i + p + 1] - t[i + 1];
    if (d1 > 0.0) r += p / d1 * cox_de_boor(t, nk, i, p - 1, u);
    if (d2 > 0.0) r -= p / d2 * cox_de_boor(t, nk, i + 1, p - 1, u);
    return r;
}

/* Second derivative, the same rule applied to the first derivatives:
   N''_{i,p} = p/(t_{i+p}-t_i) N'_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) N'_{i+1,p-1}. */
static double cox_de_boor_deriv2(const double *t, int nk, int i, int p, double u)
{
    if (p <= 1) return 0.0;
    if (u < t[i] || u > t[i + p + 1]) return 0.0;
    double r = 0.0;
    double d1 = t[i + p] - t[i], d2 = t[i + p + 1] - t[i + 1];
    if (d1 > 0.0) r += p / d1 * cox_de_boor_deriv(t, nk, i, p - 1, u);
    if (d2 > 0.0) r -= p / d2 * cox_de_boor_deriv(t, nk, i + 1, p - 1, u);
    return r;
}

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

int32_t orc_basis(const double *t, int32_t nk, int32_t p, double u, double *N, double *dN)
{
    int n = nk - p - 1;
    if (p < 0 || n < 1) return -1;
    for (int i = 0; i < n; ++i) {
        N[i] = cox_de_boor(t, nk, i, p, u);
        if (dN) dN[i] = cox_de_boor_deriv(t, nk, i, p, u);
    }
    return n;
}

/* ------------------------------------------------------------------ evaluation
 * Eq. (Bspline) for phi (control points in R^3) and rho (scalar coefficients),
 * on the same parameter domain (Fig. "raycasting").  For NURBS the tensor-product
 * sum runs over homogeneous points (w x, w) and rho shares the rational basis.
 * The Jacobian is evaluated together with phi (Sec. "Root Finding Based
 * Algorithm": J_phi reuses the evaluation of phi).                           */
int32_t orc_eval(const orc_patch *P, const double pin[3], double x[3], double J[9], double *rho)
{
    double Nb[3][MAXN], dNb[3][MAXN];
    double p[3];
    for (int d = 0; d < 3; ++d) {
        if (P->ncp[d] > MAXN || P->deg[d] > MAXP) return -1;
        p[d] = clamp01(pin[d]);
        orc_basis(P->knots[d], P->ncp[d] + P->deg[d] + 1, P->deg[d], p[d], Nb[d], dNb[d]);
    }
    const int n0 = P->ncp[0], n1 = P->ncp[1], n2 = P->ncp[2];
    double A[4] = {0, 0, 0, 0}, dA[3][4] = {{0}}, R = 0.0;
    for (int k = 0; k < n2; ++k) {
        if (Nb[2][k] == 0.0 && dNb[2][k] == 0.0) continue;
        for (int j = 0; j < n1; ++j) {
            if (Nb[1][j] == 0.0 && dNb[1][j] == 0.0) continue;
            for (int i = 0; i < n0; ++i) {
                if (Nb[0][i] == 0.0 && dNb[0][i] == 0.0) continue;
                const double *c = P->cp + 4 * ((size_t)i + (size_t)n0 * (j + (size_t)n1 * k));
                const double s = P->scalar[i + (size_t)n0 * (j + (size_t)n1 * k)];
                const double w = P->rational ? c[3] : 1.0;
                const double b = Nb[0][i] * Nb[1][j] * Nb[2][k];
                const double bd[3] = {dNb[0][i] * Nb[1][j] * Nb[2][k],
                                      Nb[0][i] * dNb[1][j] * Nb[2][k],
                                      Nb[0][i] * Nb[1][j] * dNb[2][k]};
                for (int r = 0; r < 3; ++r) A[r] += b * w * c[r];
                A[3] += b * w;
                R += b * w * s;
                for (int q = 0; q < 3; ++q) {
                    for (int r = 0; r < 3; ++r) dA[q][r] += bd[q] * w * c[r];
                    dA[q][3] += bd[q] * w;
                }
            }
        }
    }
    if (P->rational) {
        /* quotient rule: phi = A/W, d phi = (dA - phi dW)/W */
        for (int r = 0; r < 3; ++r) x[r] = A[r] / A[3];
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) J[r * 3 + q] = (dA[q][r] - x[r] * dA[q][3]) / A[3];
        if (rho) *rho = R / A[3];
    } else {
        for (int r = 0; r < 3; ++r) x[r] = A[r];
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) J[r * 3 + q] = dA[q][r];
        if (rho) *rho = R;
    }
    return 0;
}

/* ------------------------------------------------------------------ Hessian
 * H_phi of Sec. "ODE Based Algorithm" (the order-3 tensor in the Jacobian of
 * the implicit Euler step): H[r*9 + a*3 + b] = d^2 phi_r / dp_a dp_b, with phi
 * and J.  Tensor-product sums of the basis and its first and second
 * derivatives; for NURBS, phi = A/w differentiated twice:
 *   phi_ab = (A_ab - phi_a w_b - phi_b w_a - phi w_ab) / w.                  */
int32_t orc_eval_hessian(const orc_patch *P, const double pin[3], double x[3], double J[9], double H[27])
{
    static __thread double Nb[3][MAXN], dNb[3][MAXN], ddNb[3][MAXN];
    double p[3];
    for (int d = 0; d < 3; ++d) {
        if (P->ncp[d] > MAXN || P->deg[d] > MAXP) return -1;
        p[d] = clamp01(pin[d]);
        const int nk = P->ncp[d] + P->deg[d] + 1;
        for (int i = 0; i < P->ncp[d]; ++i) {
            Nb[d][i] = cox_de_boor(P->knots[d], nk, i, P->deg[d], p[d]);
            dNb[d][i] = cox_de_boor_deriv(P->knots[d], nk, i, P->deg[d], p[d]);
            ddNb[d][i] = cox_de_boor_deriv2(P->knots[d], nk, i, P->deg[d], p[d]);
        }
    }
    const int n0 = P->ncp[0], n1 = P->ncp[1], n2 = P->ncp[2];
    /* A[c], dA[a][c], ddA[a][b][c]: homogeneous sums (c = 3 the weight) */
    double A[4] = {0}, dA[3][4] = {{0}}, ddA[3][3][4] = {{{0}}};
    for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) {
                const double f[3] = {Nb[0][i], Nb[1][j], Nb[2][k]};
                const double df[3] = {dNb[0][i], dNb[1][j], dNb[2][k]};
                const double ddf[3] = {ddNb[0][i], ddNb[1][j], ddNb[2][k]};
                if (f[0] == 0 && df[0] == 0 && ddf[0] == 0) continue;
                if (f[1] == 0 && df[1] == 0 && ddf[1] == 0) continue;
                if (f[2] == 0 && df[2] == 0 && ddf[2] == 0) continue;
                const double *c = P->cp + 4 * ((size_t)i + (size_t)n0 * (j + (size_t)n1 * k));
                const double w = P->rational ? c[3] : 1.0;
                const double hv[4] = {w * c[0], w * c[1], w * c[2], w};
                /* basis products: direction a differentiated once (and b once more) */
                for (int a = 0; a < 3; ++a) {
                    double ba = 1.0;
                    for (int e = 0; e < 3; ++e) ba *= e == a ? df[e] : f[e];
                    for (int q = 0; q < 4; ++q) dA[a][q] += ba * hv[q];
                    for (int b = 0; b < 3; ++b) {
                        double bab = 1.0;
                        for (int e = 0; e < 3; ++e) {
                            const int order = (e == a) + (e == b);
                            bab *= order == 0 ? f[e] : (order == 1 ? df[e] : ddf[e]);
                        }
                        for (int q = 0; q < 4; ++q) ddA[a][b][q] += bab * hv[q];
                    }
                }
                const double b0 = f[0] * f[1] * f[2];
                for (int q = 0; q < 4; ++q) A[q] += b0 * hv[q];
            }
    const double w = A[3];
    for (int r = 0; r < 3; ++r) x[r] = A[r] / w;
    for (int r = 0; r < 3; ++r)
        for (int a = 0; a < 3; ++a) J[r * 3 + a] = (dA[a][r] - x[r] * dA[a][3]) / w;
    for (int r = 0; r < 3; ++r)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                H[r * 9 + a * 3 + b] = (ddA[a][b][r] - J[r * 3 + a] * dA[b][3] - J[r * 3 + b] * dA[a][3] -
                                        x[r] * ddA[a][b][3]) / w;
    return 0;
}

/* ------------------------------------------------------------------ pixel accuracy
 * Definition "Pixel-Accurate Approximation of Geometry": a sample phi(p_i)
 * must project into the pixel of its ray, Delta P = 2 |pi_s(phi(p_i)) - c|_inf
 * <= 1 (Eq. (deltaP)) with c the pixel centre and pi_s the projection to the
 * screen (in pixel units), and the samples' projections onto the ray must not
 * go back towards the eye ("covering accuracy").                             */
static double norm3(const double v[3]);

double orc_delta_p(const orc_camera *c, int64_t pixel, const double g[3])
{
    double f[3], r[3], u[3], v[3];
    for (int q = 0; q < 3; ++q) f[q] = c->target[q] - c->eye[q];
    const double nf = norm3(f);
    for (int q = 0; q < 3; ++q) f[q] /= nf;
    r[0] = f[1] * c->up[2] - f[2] * c->up[1];
    r[1] = f[2] * c->up[0] - f[0] * c->up[2];
    r[2] = f[0] * c->up[1] - f[1] * c->up[0];
    const double nr = norm3(r);
    for (int q = 0; q < 3; ++q) r[q] /= nr;
    u[0] = r[1] * f[2] - r[2] * f[1];
    u[1] = r[2] * f[0] - r[0] * f[2];
    u[2] = r[0] * f[1] - r[1] * f[0];
    for (int q = 0; q < 3; ++q) v[q] = g[q] - c->eye[q];
    const double z = v[0] * f[0] + v[1] * f[1] + v[2] * f[2];
    const double th = tan(0.5 * c->fov_y_deg * M_PI / 180.0), aspect = (double)c->width / (double)c->height;
    const double sx = (v[0] * r[0] + v[1] * r[1] + v[2] * r[2]) / z;
    const double sy = (v[0] * u[0] + v[1] * u[1] + v[2] * u[2]) / z;
    const double X = (sx / (th * aspect) + 1.0) * 0.5 * c->width, Y = (1.0 - sy / th) * 0.5 * c->height;
    const double cx = (double)(pixel % c->width) + 0.5, cy = (double)(pixel / c->width) + 0.5;
    return 2.0 * fmax(fabs(X - cx), fabs(Y - cy));
}

/* Per-pixel pixel-accuracy record of the method mode's interior samples. */
typedef struct {
    const orc_camera *cam;
    int64_t pixel;
    const double *o, *d;
    double dp_max, t_prev;
    int order_bad;
} pix_diag_t;

static void diag_sample(pix_diag_t *dg, const orc_patch *P, const double p[3])
{
    if (!dg) return;
    double x[3], J[9];
    orc_eval(P, p, x, J, NULL);
    const double dp = orc_delta_p(dg->cam, dg->pixel, x);
    if (dp > dg->dp_max) dg->dp_max = dp;
    const double t = (x[0] - dg->o[0]) * dg->d[0] + (x[1] - dg->o[1]) * dg->d[1] + (x[2] - dg->o[2]) * dg->d[2];
    if (t < dg->t_prev) ++dg->order_bad;
    dg->t_prev = t;
}

/* ------------------------------------------------------------------ derived fields
 * Sec. "Parametrization Quality of Geometry", Eq. (paramQuality): the quality
 * of the parametrisation is det J_phi / ||J_phi||_F.
 * Structural analysis, Eq. (vonMises): a displacement field u on P (a spline on
 * the basis of phi: u = sum R_i u_i with the rational basis R_i of a NURBS
 * block).  The Jacobian X of u o phi^-1 at g = phi(p) solves
 * J_phi(p)^T X = J_u(p)^T, column by column (that is the transpose of the
 * chain rule's J_u J_phi^-1, which the symmetrisation below removes); the
 * tensor e = (X + X^T)/2, and the value
 *   sqrt(((e11-e22)^2 + (e22-e33)^2 + (e33-e11)^2 + 6 (e12^2 + e23^2 + e31^2)) / 2),
 * the von Mises form, whose squares and root the printed formula lacks.      */
static int solve3(const double Min[9], const double bin[3], double xout[3]);

/* J_u[r*3 + a] = d u_r / dp_a of the displacement spline at p */
static int eval_disp_jacobian(const orc_patch *P, const double pin[3], double Ju[9])
{
    static __thread double Nb[3][MAXN], dNb[3][MAXN];
    double p[3];
    if (!P->disp) return -1;
    for (int d = 0; d < 3; ++d) {
        p[d] = clamp01(pin[d]);
        orc_basis(P->knots[d], P->ncp[d] + P->deg[d] + 1, P->deg[d], p[d], Nb[d], dNb[d]);
    }
    const int n0 = P->ncp[0], n1 = P->ncp[1], n2 = P->ncp[2];
    double U[4] = {0, 0, 0, 0}, dU[3][4] = {{0}};   /* homogeneous (w u, w) */
    for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) {
                const double b = Nb[0][i] * Nb[1][j] * Nb[2][k];
                const double bd[3] = {dNb[0][i] * Nb[1][j] * Nb[2][k], Nb[0][i] * dNb[1][j] * Nb[2][k],
                                      Nb[0][i] * Nb[1][j] * dNb[2][k]};
                if (b == 0.0 && bd[0] == 0.0 && bd[1] == 0.0 && bd[2] == 0.0) continue;
                const size_t li = i + (size_t)n0 * (j + (size_t)n1 * k);
                const double w = P->rational ? P->cp[4 * li + 3] : 1.0;
                const double hv[4] = {w * P->disp[3 * li], w * P->disp[3 * li + 1], w * P->disp[3 * li + 2], w};
                for (int q = 0; q < 4; ++q) {
                    U[q] += b * hv[q];
                    for (int a = 0; a < 3; ++a) dU[a][q] += bd[a] * hv[q];
                }
            }
    for (int r = 0; r < 3; ++r) {
        const double u = U[r] / U[3];
        for (int a = 0; a < 3; ++a) Ju[r * 3 + a] = (dU[a][r] - u * dU[a][3]) / U[3];
    }
    return 0;
}

int32_t orc_field(const orc_patch *P, const double p[3], int32_t field, double *value)
{
    double x[3], J[9], rho;
    if (orc_eval(P, p, x, J, &rho) != 0) return -1;
    if (field == ORC_FIELD_SCALAR) {
        *value = rho;
        return 0;
    }
    if (field == ORC_FIELD_PARAM_QUALITY) {
        const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                           J[2] * (J[3] * J[7] - J[4] * J[6]);
        double fro = 0.0;
        for (int i = 0; i < 9; ++i) fro += J[i] * J[i];
        *value = det / sqrt(fro);
        return 0;
    }
    if (field != ORC_FIELD_VON_MISES) return -1;
    double Ju[9], JT[9], X[9];
    if (eval_disp_jacobian(P, p, Ju) != 0) return -1;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) JT[r * 3 + c] = J[c * 3 + r];
    for (int col = 0; col < 3; ++col) {
        /* column col of J_u^T is row col of J_u */
        double rhs[3] = {Ju[col * 3], Ju[col * 3 + 1], Ju[col * 3 + 2]}, xc[3];
        if (solve3(JT, rhs, xc) != 0) return -1;
        for (int r = 0; r < 3; ++r) X[r * 3 + col] = xc[r];
    }
    double e[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) e[r][c] = 0.5 * (X[r * 3 + c] + X[c * 3 + r]);
    const double a = e[0][0] - e[1][1], b = e[1][1] - e[2][2], c = e[2][2] - e[0][0];
    *value = sqrt(0.5 * (a * a + b * b + c * c + 6.0 * (e[0][1] * e[0][1] + e[1][2] * e[1][2] + e[2][0] * e[2][0])));
    return 0;
}

/* ------------------------------------------------------------------ linear solve
 * 3x3 systems of Eq. (newtonsmethod) and Eq. (VgVp).  The paper names a QR
 * factorisation; any exact direct method solves the same system.  Gaussian
 * elimination with partial pivoting, FP64.  Returns 0, or -1 if singular.    */
static int solve3(const double Min[9], const double bin[3], double xout[3])
{
    double M[3][4];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) M[r][c] = Min[r * 3 + c];
        M[r][3] = bin[r];
    }
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
        if (M[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int q = 0; q < 4; ++q) { double tmp = M[c][q]; M[c][q] = M[piv][q]; M[piv][q] = tmp; }
        for (int r = c + 1; r < 3; ++r) {
            double f = M[r][c] / M[c][c];
            for (int q = c; q < 4; ++q) M[r][q] -= f * M[c][q];
        }
    }
    for (int r = 2; r >= 0; --r) {
        double s = M[r][3];
        for (int q = r + 1; q < 3; ++q) s -= M[r][q] * xout[q];
        xout[r] = s / M[r][r];
    }
    for (int r = 0; r < 3; ++r)
        if (!isfinite(xout[r])) return -1;
    return 0;
}

static double norm3(const double v[3]) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* ------------------------------------------------------------------ inversion
 * Sec. "Root Finding Based Algorithm": F_g(p) = phi(p) - g (Eq. (F)), Newton's
 * method J_F(x_n)(x_{n+1}-x_n) = -F(x_n) (Eq. (newtonsmethod)), iterates clamped
 * to the parameter domain [0,1]^3 with a line search.  Stops when
 * ||F|| <= 1e-12 * scale.                                                    */
int32_t orc_invert(const orc_patch *P, const double g[3], const double seed[3], double scale,
                   double p_out[3], int32_t *iterations)
{
    const double tol = 1e-12 * scale;
    double p[3] = {clamp01(seed[0]), clamp01(seed[1]), clamp01(seed[2])};
    double x[3], J[9], F[3];
    orc_eval(P, p, x, J, NULL);
    for (int r = 0; r < 3; ++r) F[r] = x[r] - g[r];
    double nF = norm3(F);
    int it = 0;
    for (; it < 60 && nF > tol; ++it) {
        double step[3], negF[3] = {-F[0], -F[1], -F[2]};
        if (solve3(J, negF, step) != 0) break;
        double lam = 1.0;
        int accepted = 0;
        for (int ls = 0; ls < 40; ++ls, lam *= 0.5) {
            double q[3], xq[3], Jq[9], Fq[3];
            for (int r = 0; r < 3; ++r) q[r] = clamp01(p[r] + lam * step[r]);
            orc_eval(P, q, xq, Jq, NULL);
            for (int r = 0; r < 3; ++r) Fq[r] = xq[r] - g[r];
            double nq = norm3(Fq);
            if (nq < nF) {
                memcpy(p, q, sizeof p);
                memcpy(J, Jq, sizeof J);
                memcpy(F, Fq, sizeof F);
                nF = nq;
                accepted = 1;
                break;
            }
        }
        if (!accepted) break;
    }
    memcpy(p_out, p, sizeof p);
    if (iterations) *iterations = it;
    return nF <= tol ? 0 : -1;
}

/* Newton from the given seed, then (on failure) from a 3x3x3 grid of seeds. */
static int invert_with_restarts(const orc_patch *P, const double g[3], const double seed[3],
                                double scale, double p_out[3])
{
    if (orc_invert(P, g, seed, scale, p_out, NULL) == 0) return 0;
    static const double grid[3] = {0.1, 0.5, 0.9};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                double s[3] = {grid[a], grid[b], grid[c]};
                if (orc_invert(P, g, s, scale, p_out, NULL) == 0) return 0;
            }
    return -1;
}

/* ------------------------------------------------------------------ camera
 * Pinhole camera; pixel centres at (i+1/2, j+1/2), row 0 at the top, vertical
 * field of view fov_y.  The view ray is gamma(s) = eye + s d, |d| = 1.       */
void orc_camera_ray(const orc_camera *c, double px, double py, double o[3], double d[3])
{
    double f[3], r[3], u[3];
    for (int q = 0; q < 3; ++q) f[q] = c->target[q] - c->eye[q];
    double nf = norm3(f);
    for (int q = 0; q < 3; ++q) f[q] /= nf;
    r[0] = f[1] * c->up[2] - f[2] * c->up[1];
    r[1] = f[2] * c->up[0] - f[0] * c->up[2];
    r[2] = f[0] * c->up[1] - f[1] * c->up[0];
    double nr = norm3(r);
    for (int q = 0; q < 3; ++q) r[q] /= nr;
    u[0] = r[1] * f[2] - r[2] * f[1];
    u[1] = r[2] * f[0] - r[0] * f[2];
    u[2] = r[0] * f[1] - r[1] * f[0];
    double th = tan(0.5 * c->fov_y_deg * M_PI / 180.0);
    double aspect = (double)c->width / (double)c->height;
    double sx = (2.0 * px / c->width - 1.0) * th * aspect;
    double sy = (1.0 - 2.0 * py / c->height) * th;
    for (int q = 0; q < 3; ++q) d[q] = f[q] + sx * r[q] + sy * u[q];
    double nd = norm3(d);
    for (int q = 0; q < 3; ++q) { d[q] /= nd; o[q] = c->eye[q]; }
}

/* ------------------------------------------------------------------ transfer function
 * Eq. (emissionabsorption): emission and absorption are functions of rho.  The
 * paper leaves the form open; here a piecewise-linear RGBA table over the
 * normalised value n = clamp((rho-lo)/(hi-lo)), kappa = extinction * A.      */
void orc_transfer(const orc_tf *tf, double rho, double out[4])
{
    double n = (rho - tf->domain[0]) / (tf->domain[1] - tf->domain[0]);
    n = clamp01(n);
    int k = 0;
    while (k < tf->n - 2 && n > tf->x[k + 1]) ++k;
    double w = tf->x[k + 1] > tf->x[k] ? (n - tf->x[k]) / (tf->x[k + 1] - tf->x[k]) : 0.0;
    w = clamp01(w);
    for (int c = 0; c < 4; ++c)
        out[c] = (1.0 - w) * tf->rgba[4 * k + c] + w * tf->rgba[4 * (k + 1) + c];
    out[3] *= tf->extinction;
}

/* ------------------------------------------------------------------ faces
 * Sec. "View-Ray Intersections with Surfaces": all 6 boundary faces of every
 * block.  With clamped knots a face is the bivariate spline of the boundary
 * layer of control points.  Each face is split into Bezier elements by knot
 * insertion (Boehm), every element is culled by the bounding box of its
 * control points (convex hull; positive weights keep it valid for NURBS) and
 * subdivided by de Casteljau until small, then solved by Newton in FP64.    */

typedef struct {
    int patch, face;
    int m, n;                  /* Bezier degrees in the face directions a, b */
    double a0, a1, b0, b1;     /* element rectangle in face parameters       */
    double Q[(MAXP + 1) * (MAXP + 1) * 4];   /* homogeneous control points, a fastest */
    double lo[3], hi[3];       /* bounding box of the projected points        */
} bez_elem;

struct orc_scene {
    orc_patch *patches;
    int npatch;
    double scale;
    bez_elem *elems;
    int nelem;
    double (*pbox)[6];         /* per-patch box of control points             */
    int *elem_begin;           /* elements of patch i: [elem_begin[i], elem_begin[i+1]) */
};

/* face f: fixed direction f/2 at value f%2; in-face directions (a, b) */
static void face_dirs(int f, int *dn, int *da, int *db)
{
    *dn = f / 2;
    *da = (*dn == 0) ? 1 : 0;
    *db = (*dn == 2) ? 1 : 2;
}

/* Boehm knot insertion of u into a curve of `n` homogeneous points. */
static void insert_knot(const double *t, int nk, int p, const double *Q, int n, double u,
                        double *t2, double *Q2)
{
    int k = p;
    while (k + 1 < nk && t[k + 1] <= u) ++k;           /* t[k] <= u < t[k+1] */
    for (int i = 0; i <= n; ++i) {
        if (i <= k - p) {
            memcpy(Q2 + 4 * i, Q + 4 * i, 4 * sizeof(double));
        } else if (i >= k + 1) {
            memcpy(Q2 + 4 * i, Q + 4 * (i - 1), 4 * sizeof(double));
        } else {
            double a = (u - t[i]) / (t[i + p] - t[i]);
            for (int c = 0; c < 4; ++c) Q2[4 * i + c] = (1.0 - a) * Q[4 * (i - 1) + c] + a * Q[4 * i + c];
        }
    }
    for (int i = 0; i <= k; ++i) t2[i] = t[i];
    t2[k + 1] = u;
    for (int i = k + 1; i < nk; ++i) t2[i + 1] = t[i];
}

/* Raise every interior knot of a curve to multiplicity p.  Returns the new
   point count; writes the distinct breakpoints to brk (count in *nbrk).      */
static int bezier_extract_curve(const double *t, int nk, int p, const double *Q, int n,
                                double *Qout, double *brk, int *nbrk)
{
    double *tc = malloc(sizeof(double) * (nk + (size_t)p * nk + 8));
    double *tn = malloc(sizeof(double) * (nk + (size_t)p * nk + 8));
    double *Qc = malloc(sizeof(double) * 4 * (n + (size_t)p * nk + 8));
    double *Qn = malloc(sizeof(double) * 4 * (n + (size_t)p * nk + 8));
    memcpy(tc, t, sizeof(double) * nk);
    memcpy(Qc, Q, sizeof(double) * 4 * n);
    int ncur = n, nkcur = nk;
    *nbrk = 0;
    brk[(*nbrk)++] = t[p];
    for (int i = p + 1; i < nk - p - 1; ) {
        double u = t[i];
        int mult = 0;
        while (i + mult < nk - p - 1 && t[i + mult] == u) ++mult;
        for (int r = mult; r < p; ++r) {
            insert_knot(tc, nkcur, p, Qc, ncur, u, tn, Qn);
            ++nkcur; ++ncur;
            double *sw = tc; tc = tn; tn = sw;
            sw = Qc; Qc = Qn; Qn = sw;
        }
        brk[(*nbrk)++] = u;
        i += mult;
    }
    brk[(*nbrk)++] = t[nk - p - 1];
    memcpy(Qout, Qc, sizeof(double) * 4 * ncur);
    free(tc); free(tn); free(Qc); free(Qn);
    return ncur;
}

static void proj_box(const double *Q, int cnt, double lo[3], double hi[3])
{
    for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
    for (int i = 0; i < cnt; ++i)
        for (int c = 0; c < 3; ++c) {
            double v = Q[4 * i + c] / Q[4 * i + 3];
            if (v < lo[c]) lo[c] = v;
            if (v > hi[c]) hi[c] = v;
        }
}

orc_scene *orc_prepare(const orc_patch *patches, int32_t n, double scale)
{
    orc_scene *s = calloc(1, sizeof *s);
    s->npatch = n;
    s->scale = scale;
    s->patches = malloc(sizeof(orc_patch) * n);
    memcpy(s->patches, patches, sizeof(orc_patch) * n);
    s->pbox = malloc(sizeof(double[6]) * n);
    s->elem_begin = malloc(sizeof(int) * (n + 1));
    int cap = 1024;
    s->elems = malloc(sizeof(bez_elem) * cap);
    for (int pi = 0; pi < n; ++pi) {
        const orc_patch *P = &patches[pi];
        s->elem_begin[pi] = s->nelem;
        int N = P->ncp[0] * P->ncp[1] * P->ncp[2];
        double *Qh = malloc(sizeof(double) * 4 * N);
        for (int i = 0; i < N; ++i) {
            double w = P->rational ? P->cp[4 * i + 3] : 1.0;
            for (int c = 0; c < 3; ++c) Qh[4 * i + c] = w * P->cp[4 * i + c];
            Qh[4 * i + 3] = w;
        }
        proj_box(Qh, N, s->pbox[pi], s->pbox[pi] + 3);
        for (int f = 0; f < 6; ++f) {
            int dn, da, db;
            face_dirs(f, &dn, &da, &db);
            int na = P->ncp[da], nb = P->ncp[db], pa = P->deg[da], pb = P->deg[db];
            int fix = (f % 2) ? P->ncp[dn] - 1 : 0;
            /* face net, a fastest */
            double *F = malloc(sizeof(double) * 4 * na * nb);
            for (int jb = 0; jb < nb; ++jb)
                for (int ia = 0; ia < na; ++ia) {
                    int idx[3];
                    idx[dn] = fix; idx[da] = ia; idx[db] = jb;
                    size_t li = idx[0] + (size_t)P->ncp[0] * (idx[1] + (size_t)P->ncp[1] * idx[2]);
                    memcpy(F + 4 * ((size_t)jb * na + ia), Qh + 4 * li, 4 * sizeof(double));
                }
            int nka = na + pa + 1, nkb = nb + pb + 1;
            int cap_a = na + pa * nka + 8, cap_b = nb + pb * nkb + 8;
            double *brka = malloc(sizeof(double) * (nka + 2)), *brkb = malloc(sizeof(double) * (nkb + 2));
            int nbrka = 0, nbrkb = 0;
            /* extract along a for every row */
            double *Fa = malloc(sizeof(double) * 4 * (size_t)cap_a * nb);
            int na2 = 0;
            for (int jb = 0; jb < nb; ++jb)
                na2 = bezier_extract_curve(P->knots[da], nka, pa, F + 4 * (size_t)jb * na, na,
                                           Fa + 4 * (size_t)jb * cap_a, brka, &nbrka);
            /* extract along b for every column */
            double *col = malloc(sizeof(double) * 4 * nb), *colx = malloc(sizeof(double) * 4 * cap_b);
            double *Fab = malloc(sizeof(double) * 4 * (size_t)na2 * cap_b);
            int nb2 = 0;
            for (int ia = 0; ia < na2; ++ia) {
                for (int jb = 0; jb < nb; ++jb)
                    memcpy(col + 4 * jb, Fa + 4 * ((size_t)jb * cap_a + ia), 4 * sizeof(double));
                nb2 = bezier_extract_curve(P->knots[db], nkb, pb, col, nb, colx, brkb, &nbrkb);
                for (int jb = 0; jb < nb2; ++jb)
                    memcpy(Fab + 4 * ((size_t)jb * na2 + ia), colx + 4 * jb, 4 * sizeof(double));
            }
            for (int eb = 0; eb + 1 < nbrkb; ++eb)
                for (int ea = 0; ea + 1 < nbrka; ++ea) {
                    if (s->nelem == cap) { cap *= 2; s->elems = realloc(s->elems, sizeof(bez_elem) * cap); }
                    bez_elem *E = &s->elems[s->nelem++];
                    E->patch = pi; E->face = f; E->m = pa; E->n = pb;
                    E->a0 = brka[ea]; E->a1 = brka[ea + 1];
                    E->b0 = brkb[eb]; E->b1 = brkb[eb + 1];
                    for (int jb = 0; jb <= pb; ++jb)
                        for (int ia = 0; ia <= pa; ++ia)
                            memcpy(E->Q + 4 * (jb * (pa + 1) + ia),
                                   Fab + 4 * ((size_t)(eb * pb + jb) * na2 + (ea * pa + ia)),
                                   4 * sizeof(double));
                    proj_box(E->Q, (pa + 1) * (pb + 1), E->lo, E->hi);
                }
            free(F); free(brka); free(brkb); free(Fa); free(col); free(colx); free(Fab);
        }
        free(Qh);
    }
    s->elem_begin[n] = s->nelem;
    return s;
}

void orc_free(orc_scene *s)
{
    if (!s) return;
    free(s->patches); free(s->elems); free(s->pbox); free(s->elem_begin); free(s);
}

/* ------------------------------------------------------------------ point location
 * For brute-force tests of the fragment finder: is g inside block alpha, i.e.
 * does F_g of Eq. (F) have a root in P_alpha?  By the argument of Sec. "Root
 * Finding Based Algorithm" (|F_g(p)| is the distance to the preimage, so
 * Newton with line search converges from interior seeds when a preimage
 * exists), Newton with clamping and line search (orc_invert) is run from the
 * hint (the previous point's parameters, when *block >= 0 on entry) and then
 * from nine interior seeds, over every block whose control-point box holds g.
 * block[i] = -2 on entry takes point i-1's result as the hint (points along a
 * ray).  Uses no part of the boundary-face machinery.  On return block[i] is the
 * first block that holds g[i] (-1: none), p[3i..] its parameters and rho[i]
 * the scalar there.                                                          */
int32_t orc_locate(const orc_scene *s, const double *g, int64_t n, int32_t *block, double *p,
                   double *rho)
{
    static const double seeds[9][3] = {{0.5, 0.5, 0.5}, {0.25, 0.25, 0.25}, {0.75, 0.25, 0.25},
                                       {0.25, 0.75, 0.25}, {0.75, 0.75, 0.25}, {0.25, 0.25, 0.75},
                                       {0.75, 0.25, 0.75}, {0.25, 0.75, 0.75}, {0.75, 0.75, 0.75}};
    for (int64_t i = 0; i < n; ++i) {
        const double *gi = g + 3 * i;
        const int chain = block[i] == -2 && i > 0;
        const int hint = chain ? block[i - 1] : block[i];
        const double *hsrc = chain ? p + 3 * (i - 1) : p + 3 * i;
        double hp[3] = {hsrc[0], hsrc[1], hsrc[2]};
        int found = -1;
        double q[3];
        for (int pi = 0; pi < s->npatch && found < 0; ++pi) {
            const double *bx = s->pbox[pi];
            const double pad = 1e-9 * s->scale;
            if (gi[0] < bx[0] - pad || gi[1] < bx[1] - pad || gi[2] < bx[2] - pad || gi[0] > bx[3] + pad ||
                gi[1] > bx[4] + pad || gi[2] > bx[5] + pad)
                continue;
            const orc_patch *P = &s->patches[pi];
            if (pi == hint && orc_invert(P, gi, hp, s->scale, q, NULL) == 0) {
                found = pi;
                break;
            }
            for (int k = 0; k < 9; ++k)
                if (orc_invert(P, gi, seeds[k], s->scale, q, NULL) == 0) {
                    found = pi;
                    break;
                }
        }
        block[i] = found;
        if (found >= 0) {
            double x[3], J[9], r;
            orc_eval(&s->patches[found], q, x, J, &r);
            p[3 * i] = q[0]; p[3 * i + 1] = q[1]; p[3 * i + 2] = q[2];
            if (rho) rho[i] = r;
        }
    }
    return 0;
}

/* slab test of the ray (t >= 0) against a padded box */
static int ray_box(const double o[3], const double d[3], const double lo[3], const double hi[3],
                   double pad)
{
    double t0 = 0.0, t1 = INFINITY;
    for (int c = 0; c < 3; ++c) {
        double l = lo[c] - pad, h = hi[c] + pad;
        if (fabs(d[c]) < 1e-300) {
            if (o[c] < l || o[c] > h) return 0;
            continue;
        }
        double ta = (l - o[c]) / d[c], tb = (h - o[c]) / d[c];
        if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

static double binom(int n, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

/* Bernstein polynomial B_i^n(a) = C(n,i) a^i (1-a)^(n-i). */
static double bernstein(int n, int i, double a)
{
    if (i < 0 || i > n) return 0.0;
    return binom(n, i) * pow(a, i) * pow(1.0 - a, n - i);
}

/* Rational Bezier patch value and first derivatives in local (a,b) in [0,1]^2. */
static void bez_eval(const double *Q, int m, int n, double a, double b,
                     double S[3], double Sa[3], double Sb[3])
{
    double H[4] = {0}, Ha[4] = {0}, Hb[4] = {0};
    for (int j = 0; j <= n; ++j)
        for (int i = 0; i <= m; ++i) {
            const double *q = Q + 4 * (j * (m + 1) + i);
            double B = bernstein(m, i, a) * bernstein(n, j, b);
            /* d/da B_i^m = m (B_{i-1}^{m-1} - B_i^{m-1}) */
            double Ba = m * (bernstein(m - 1, i - 1, a) - bernstein(m - 1, i, a)) * bernstein(n, j, b);
            double Bb = bernstein(m, i, a) * n * (bernstein(n - 1, j - 1, b) - bernstein(n - 1, j, b));
            for (int c = 0; c < 4; ++c) {
                H[c] += B * q[c];
                Ha[c] += Ba * q[c];
                Hb[c] += Bb * q[c];
            }
        }
    for (int c = 0; c < 3; ++c) {
        S[c] = H[c] / H[3];
        Sa[c] = (Ha[c] - S[c] * Ha[3]) / H[3];
        Sb[c] = (Hb[c] - S[c] * Hb[3]) / H[3];
    }
}

/* de Casteljau split of the net at parameter 1/2 in direction a (dir 0) or b. */
static void bez_split(const double *Q, int m, int n, int dir, double *L, double *R)
{
    int deg = dir == 0 ? m : n, rows = dir == 0 ? n + 1 : m + 1;
    for (int r = 0; r < rows; ++r) {
        double tmp[MAXP + 1][4];
        for (int i = 0; i <= deg; ++i) {
            int idx = dir == 0 ? r * (m + 1) + i : i * (m + 1) + r;
            memcpy(tmp[i], Q + 4 * idx, 4 * sizeof(double));
        }
        for (int lvl = 0; lvl <= deg; ++lvl) {
            int il = lvl, ir = deg - lvl;
            int idxl = dir == 0 ? r * (m + 1) + il : il * (m + 1) + r;
            int idxr = dir == 0 ? r * (m + 1) + ir : ir * (m + 1) + r;
            memcpy(L + 4 * idxl, tmp[0], 4 * sizeof(double));
            memcpy(R + 4 * idxr, tmp[deg - lvl], 4 * sizeof(double));
            for (int i = 0; i < deg - lvl; ++i)
                for (int c = 0; c < 4; ++c) tmp[i][c] = 0.5 * (tmp[i][c] + tmp[i + 1][c]);
        }
    }
}

typedef struct {
    const double *o, *d;
    double scale;
    int patch, face;
    double hits[64][3];        /* (a, b, t) in face parameters */
    int nhits;
} leaf_ctx;

static void subdivide_solve(const double *Q, int m, int n, double a0, double a1, double b0,
                            double b1, int depth, leaf_ctx *cx)
{
    double lo[3], hi[3];
    proj_box(Q, (m + 1) * (n + 1), lo, hi);
    if (!ray_box(cx->o, cx->d, lo, hi, 1e-12 * cx->scale)) return;
    double dg[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    if (norm3(dg) <= 1e-3 * cx->scale || depth >= 48) {
        /* Newton on (a, b, t): S(a,b) - (o + t d) = 0 */
        double a = 0.5, b = 0.5, S[3], Sa[3], Sb[3];
        bez_eval(Q, m, n, a, b, S, Sa, Sb);
        double t = (S[0] - cx->o[0]) * cx->d[0] + (S[1] - cx->o[1]) * cx->d[1] +
                   (S[2] - cx->o[2]) * cx->d[2];
        for (int it = 0; it < 40; ++it) {
            double F[3];
            for (int c = 0; c < 3; ++c) F[c] = S[c] - cx->o[c] - t * cx->d[c];
            if (norm3(F) <= 1e-12 * cx->scale) {
                if (a >= -1e-9 && a <= 1.0 + 1e-9 && b >= -1e-9 && b <= 1.0 + 1e-9 && t > 0.0 &&
                    cx->nhits < 64) {
                    a = clamp01(a); b = clamp01(b);
                    cx->hits[cx->nhits][0] = a0 + a * (a1 - a0);
                    cx->hits[cx->nhits][1] = b0 + b * (b1 - b0);
                    cx->hits[cx->nhits][2] = t;
                    cx->nhits++;
                }
                return;
            }
            double M[9] = {Sa[0], Sb[0], -cx->d[0], Sa[1], Sb[1], -cx->d[1], Sa[2], Sb[2], -cx->d[2]};
            double negF[3] = {-F[0], -F[1], -F[2]}, st[3];
            if (solve3(M, negF, st) != 0) return;
            a += st[0]; b += st[1]; t += st[2];
            if (a < -1.0 || a > 2.0 || b < -1.0 || b > 2.0) return;
            bez_eval(Q, m, n, a, b, S, Sa, Sb);
        }
        return;
    }
    double L[(MAXP + 1) * (MAXP + 1) * 4], R[(MAXP + 1) * (MAXP + 1) * 4];
    /* split the parametric direction with the larger world extent of its control polygon */
    double ea = 0.0, eb = 0.0;
    for (int j = 0; j <= n; ++j)
        for (int i = 0; i < m; ++i) {
            double v[3];
            for (int c = 0; c < 3; ++c)
                v[c] = Q[4 * (j * (m + 1) + i + 1) + c] / Q[4 * (j * (m + 1) + i + 1) + 3] -
                       Q[4 * (j * (m + 1) + i) + c] / Q[4 * (j * (m + 1) + i) + 3];
            ea += norm3(v);
        }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= m; ++i) {
            double v[3];
            for (int c = 0; c < 3; ++c)
                v[c] = Q[4 * ((j + 1) * (m + 1) + i) + c] / Q[4 * ((j + 1) * (m + 1) + i) + 3] -
                       Q[4 * (j * (m + 1) + i) + c] / Q[4 * (j * (m + 1) + i) + 3];
            eb += norm3(v);
        }
    if (ea / (n + 1) >= eb / (m + 1)) {
        bez_split(Q, m, n, 0, L, R);
        double am = 0.5 * (a0 + a1);
        subdivide_solve(L, m, n, a0, am, b0, b1, depth + 1, cx);
        subdivide_solve(R, m, n, am, a1, b0, b1, depth + 1, cx);
    } else {
        bez_split(Q, m, n, 1, L, R);
        double bm = 0.5 * (b0 + b1);
        subdivide_solve(L, m, n, a0, a1, b0, bm, depth + 1, cx);
        subdivide_solve(R, m, n, a0, a1, bm, b1, depth + 1, cx);
    }
}

static int cmp_frag(const void *x, const void *y)
{
    double a = ((const orc_fragment *)x)->t, b = ((const orc_fragment *)y)->t;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Entering test: the ray enters block alpha at a point of face f iff the
   parameter-space velocity J^-1 d points into P across that face. */
static int classify(const orc_patch *P, const double p[3], int face, const double d[3],
                    int *entering)
{
    double x[3], J[9], v[3];
    orc_eval(P, p, x, J, NULL);
    int dn = face / 2;
    double sgn = (face % 2) ? -1.0 : 1.0;
    if (solve3(J, d, v) == 0) {
        double s = sgn * v[dn];
        if (fabs(s) <= 1e-12 * norm3(v)) return -1;      /* grazing */
        *entering = s > 0.0;
        return 0;
    }
    /* singular J on the face: use the face normal with the orientation just inside */
    int da, db, dnn;
    face_dirs(face, &dnn, &da, &db);
    double q[3] = {p[0], p[1], p[2]};
    q[dn] += sgn * 1e-6;
    double xq[3], Jq[9];
    orc_eval(P, q, xq, Jq, NULL);
    double det = Jq[0] * (Jq[4] * Jq[8] - Jq[5] * Jq[7]) - Jq[1] * (Jq[3] * Jq[8] - Jq[5] * Jq[6]) +
                 Jq[2] * (Jq[3] * Jq[7] - Jq[4] * Jq[6]);
    double ta[3] = {J[0 + da], J[3 + da], J[6 + da]}, tb[3] = {J[0 + db], J[3 + db], J[6 + db]};
    double nrm[3] = {ta[1] * tb[2] - ta[2] * tb[1], ta[2] * tb[0] - ta[0] * tb[2],
                     ta[0] * tb[1] - ta[1] * tb[0]};
    double s = nrm[0] * d[0] + nrm[1] * d[1] + nrm[2] * d[2];
    /* J^-1 d along dn equals (t_a x t_b).d / det J (Cramer), here with the sign of
       the interior det and the face's inward direction */
    double val = sgn * s * (det > 0 ? 1.0 : -1.0);
    if (fabs(val) <= 1e-14 * norm3(nrm) || det == 0.0) return -1;
    *entering = val > 0.0;
    return 0;
}

int32_t orc_ray_fragments(const orc_scene *s, const double o[3], const double d[3],
                          orc_fragment *out, int32_t cap)
{
    int nout = 0;
    for (int pi = 0; pi < s->npatch; ++pi) {
        if (!ray_box(o, d, s->pbox[pi], s->pbox[pi] + 3, 1e-9 * s->scale)) continue;
        const orc_patch *P = &s->patches[pi];
        int first = nout;
        for (int e = s->elem_begin[pi]; e < s->elem_begin[pi + 1]; ++e) {
            const bez_elem *E = &s->elems[e];
            if (!ray_box(o, d, E->lo, E->hi, 1e-9 * s->scale)) continue;
            leaf_ctx cx;
            cx.o = o; cx.d = d; cx.scale = s->scale; cx.patch = pi; cx.face = E->face; cx.nhits = 0;
            subdivide_solve(E->Q, E->m, E->n, E->a0, E->a1, E->b0, E->b1, 0, &cx);
            for (int h = 0; h < cx.nhits; ++h) {
                int dn, da, db;
                face_dirs(E->face, &dn, &da, &db);
                orc_fragment fr;
                memset(&fr, 0, sizeof fr);
                fr.p[dn] = (E->face % 2) ? 1.0 : 0.0;
                fr.p[da] = cx.hits[h][0];
                fr.p[db] = cx.hits[h][1];
                fr.t = cx.hits[h][2];
                fr.patch = pi;
                fr.face = E->face;
                int ent;
                if (classify(P, fr.p, E->face, d, &ent) != 0) continue;
                fr.entering = ent;
                /* merge duplicates (element borders, block edges and corners) */
                int dup = 0;
                for (int q = first; q < nout; ++q)
                    if (out[q].entering == fr.entering && fabs(out[q].t - fr.t) <= 1e-9 * s->scale) {
                        dup = 1;
                        break;
                    }
                if (dup) continue;
                if (nout >= cap) return -2;
                out[nout++] = fr;
            }
        }
    }
    qsort(out, nout, sizeof(orc_fragment), cmp_frag);
    return nout;
}

/* ------------------------------------------------------------------ pairing
 * Algorithm "Blockwise depth-sorting": repeatedly take the unused exit nearest
 * to the screen, then the unused entry nearest to the screen of the same
 * block (read here with t_in <= t_out + teq); stop when no exit is left.  teq
 * is the tolerance within which two crossings are one (the duplicate merge
 * above): where a ray passes through an edge or corner of a block, its entry
 * and exit there come from roots on different faces, which agree only to
 * rounding, so either may come first.                                       */
static int pair_fragments(const orc_fragment *fr, int n, double teq, int near, int (*segs)[2], int *anomalies)
{
    int used[FRAG_CAP] = {0};
    int nseg = 0;
    *anomalies = 0;
    for (;;) {
        int ib = -1;
        for (int i = 0; i < n; ++i)
            if (!used[i] && !fr[i].entering && (ib < 0 || fr[i].t < fr[ib].t)) ib = i;
        if (ib < 0) break;
        int ifr = -1;
        for (int i = 0; i < n; ++i)
            if (!used[i] && fr[i].entering && fr[i].patch == fr[ib].patch && fr[i].t <= fr[ib].t + teq &&
                (ifr < 0 || fr[i].t < fr[ifr].t))
                ifr = i;
        used[ib] = 1;
        if (ifr < 0) {
            /* Sec. "Cutting and Near Clip Planes": with a near plane, an exit of a
               block without an entry in front of it means the near plane lies
               inside that block: the segment starts there (entry index -1) */
            if (near) {
                segs[nseg][0] = -1;
                segs[nseg][1] = ib;
                ++nseg;
            } else {
                ++*anomalies;
            }
            continue;
        }
        used[ifr] = 1;
        segs[nseg][0] = ifr;
        segs[nseg][1] = ib;
        ++nseg;
    }
    for (int i = 0; i < n; ++i)
        if (!used[i]) ++*anomalies;
    return nseg;
}

/* ------------------------------------------------------------------ quadrature
 * Eq. (volRenderIntegral) with I(0) = 0: C = int kappa E exp(-tau) ds and
 * alpha = 1 - exp(-tau).  Panels of width h with kappa and E taken at the
 * midpoint; each panel composited front to back by Algorithm "Front-to-back
 * compositing" with (1 - alpha_src)^(ds/xi) = exp(-kappa ds).  The preimage of
 * each midpoint is found by Newton, continued from the previous midpoint.    */
static int segment_integral(const orc_patch *P, const orc_tf *tf, const double o[3],
                            const double d[3], double t0, double t1, const double p0[3],
                            double scale, int npan, int field, double out[4], int *fails)
{
    double h = (t1 - t0) / npan, C[3] = {0, 0, 0}, A = 0.0, p[3] = {p0[0], p0[1], p0[2]};
    for (int m = 0; m < npan; ++m) {
        double s = t0 + (m + 0.5) * h, g[3], q[3];
        for (int c = 0; c < 3; ++c) g[c] = o[c] + s * d[c];
        if (invert_with_restarts(P, g, p, scale, q) != 0) ++*fails;
        memcpy(p, q, sizeof p);
        double rho, te[4];
        if (orc_field(P, p, field, &rho) != 0) {
            ++*fails;
            rho = 0.0;
        }
        orc_transfer(tf, rho, te);
        double T = exp(-te[3] * h);
        for (int c = 0; c < 3; ++c) C[c] += (1.0 - T) * (1.0 - A) * te[c];
        A += (1.0 - T) * (1.0 - A);
    }
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = A;
    return 0;
}

typedef struct {
    double t0, t1;             /* ray parameters of the segment's ends            */
    const double *p0;          /* parameter point of the entry, NULL if unknown   */
    int patch;
} seg_t;

static int cmp_seg(const void *x, const void *y)
{
    double a = ((const seg_t *)x)->t0, b = ((const seg_t *)y)->t0;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static void render_one(const orc_scene *s, const orc_camera *cam, const orc_tf *tf,
                       const orc_opts *opts, int64_t pix, double rgba[4], double *depth,
                       orc_pixel_diag *dg, orc_fragment *fr)
{
    int64_t col = pix % cam->width, row = pix / cam->width;
    double o[3], d[3];
    orc_camera_ray(cam, col + 0.5, row + 0.5, o, d);
    memset(dg, 0, sizeof *dg);
    rgba[0] = rgba[1] = rgba[2] = rgba[3] = 0.0;
    *depth = INFINITY;
    int n = orc_ray_fragments(s, o, d, fr, FRAG_CAP);
    if (n < 0) { dg->n_anomalies = -1; return; }
    /* Sec. "Cutting and Near Clip Planes": the near plane lies near_clip in front
       of the eye along the view direction; crossings in front of it are dropped */
    const int near = opts->near_clip > 0.0;
    double t_near = 0.0;
    if (near) {
        double f[3], nf = 0.0, fd = 0.0;
        for (int c = 0; c < 3; ++c) {
            f[c] = cam->target[c] - cam->eye[c];
            nf += f[c] * f[c];
        }
        for (int c = 0; c < 3; ++c) fd += d[c] * f[c] / sqrt(nf);
        t_near = opts->near_clip / fd;
        int m = 0;
        for (int i = 0; i < n; ++i)
            if (fr[i].t >= t_near) fr[m++] = fr[i];
        n = m;
    }
    dg->n_fragments = n;
    static const int SEGCAP = FRAG_CAP;
    int (*pairs)[2] = malloc(sizeof(int[2]) * SEGCAP);
    seg_t *segs = malloc(sizeof(seg_t) * SEGCAP);
    int anomalies = 0;
    int npair = pair_fragments(fr, n, 1e-9 * s->scale, near, pairs, &anomalies);
    dg->n_anomalies = anomalies;
    /* the segments, clipped to the cutting plane's kept half-space
       n . (g - g0) >= 0; an end moved to the plane has no known parameter point */
    int nseg = 0;
    for (int k = 0; k < npair; ++k) {
        seg_t sg;
        sg.t0 = pairs[k][0] < 0 ? t_near : fr[pairs[k][0]].t;
        sg.p0 = pairs[k][0] < 0 ? NULL : fr[pairs[k][0]].p;
        sg.t1 = fr[pairs[k][1]].t;
        sg.patch = fr[pairs[k][1]].patch;
        if (opts->cut) {
            double s0 = 0.0, sd = 0.0;
            for (int c = 0; c < 3; ++c) {
                s0 += opts->cut_normal[c] * (o[c] - opts->cut_point[c]);
                sd += opts->cut_normal[c] * d[c];
            }
            if (sd == 0.0) {
                if (s0 < 0.0) continue;
            } else {
                const double ts = -s0 / sd;
                if (sd > 0.0 && ts > sg.t0) {       /* kept beyond the plane */
                    sg.t0 = ts;
                    sg.p0 = NULL;
                } else if (sd < 0.0 && ts < sg.t1) { /* kept in front of it */
                    sg.t1 = ts;
                }
            }
            if (!(sg.t1 > sg.t0)) continue;
        }
        segs[nseg++] = sg;
    }
    dg->n_segments = nseg;
    /* front to back by entry depth */
    qsort(segs, nseg, sizeof(seg_t), cmp_seg);
    double C[3] = {0, 0, 0}, A = 0.0;
    for (int k = 0; k < nseg; ++k) {
        const seg_t *sg = &segs[k];
        const orc_patch *P = &s->patches[sg->patch];
        if (k == 0) {
            *depth = sg->t0;
            dg->first_chord = sg->t1 - sg->t0;
        }
        double p0[3] = {0.5, 0.5, 0.5};
        if (sg->p0) {
            memcpy(p0, sg->p0, sizeof p0);
        } else {
            /* an entry on a clip plane: its preimage by Newton (Eq. (F)) from the
               block centre, as the seed of the quadrature's continuation */
            double g[3], q[3];
            for (int c = 0; c < 3; ++c) g[c] = o[c] + sg->t0 * d[c];
            if (invert_with_restarts(P, g, p0, s->scale, q) != 0) ++dg->n_newton_fail;
            memcpy(p0, q, sizeof p0);
        }
        double L = sg->t1 - sg->t0;
        int npan = (int)ceil(L * opts->panels_per_scale / s->scale);
        if (npan < 1) npan = 1;
        double I1[4], res[4];
        int fails = 0;
        segment_integral(P, tf, o, d, sg->t0, sg->t1, p0, s->scale, npan, opts->field, I1, &fails);
        if (opts->richardson) {
            /* halve the panels until |I_h - I_{h/2}| <= self_tol (at most 4 times) */
            double I2[4], err = 0.0;
            for (int refine = 0;; ++refine) {
                segment_integral(P, tf, o, d, sg->t0, sg->t1, p0, s->scale, 2 * npan, opts->field, I2, &fails);
                err = 0.0;
                for (int c = 0; c < 4; ++c)
                    if (fabs(I1[c] - I2[c]) > err) err = fabs(I1[c] - I2[c]);
                if (err <= opts->self_tol || refine >= 4) break;
                memcpy(I1, I2, sizeof I1);
                npan *= 2;
            }
            for (int c = 0; c < 4; ++c) res[c] = (4.0 * I2[c] - I1[c]) / 3.0;
            if (err > dg->self_error) dg->self_error = err;
        } else {
            memcpy(res, I1, sizeof res);
        }
        dg->n_newton_fail += fails;
        /* front-to-back over operator across segments */
        for (int c = 0; c < 3; ++c) C[c] += (1.0 - A) * res[c];
        A += (1.0 - A) * res[3];
    }
    free(pairs);
    free(segs);
    rgba[0] = C[0]; rgba[1] = C[1]; rgba[2] = C[2]; rgba[3] = A;
}

typedef struct {
    const orc_scene *s;
    const orc_camera *cam;
    const orc_tf *tf;
    const orc_opts *opts;
    const int64_t *pixels;
    int64_t npix;
    double *rgba, *depth;
    orc_pixel_diag *diag;
    int tid, nthreads;
} job_t;

static void *worker(void *arg)
{
    job_t *j = arg;
    orc_fragment *fr = malloc(sizeof(orc_fragment) * FRAG_CAP);
    for (int64_t i = j->tid; i < j->npix; i += j->nthreads) {
        int64_t pix = j->pixels ? j->pixels[i] : i;
        orc_pixel_diag dg;
        render_one(j->s, j->cam, j->tf, j->opts, pix, j->rgba + 4 * i, j->depth + i, &dg, fr);
        if (j->diag) j->diag[i] = dg;
    }
    free(fr);
    return NULL;
}

int32_t orc_render_pixels(const orc_scene *s, const orc_camera *cam, const orc_tf *tf,
                          const orc_opts *opts, const int64_t *pixels, int64_t npix,
                          double *rgba, double *depth, orc_pixel_diag *diag)
{
    if (!s || !cam || !tf || !opts || !rgba || !depth || tf->n < 2) return -1;
    int nt = opts->nthreads > 0 ? opts->nthreads : (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1) nt = 1;
    if (nt > 256) nt = 256;
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < nt; ++t) {
        jobs[t] = (job_t){s, cam, tf, opts, pixels, npix, rgba, depth, diag, t, nt};
        pthread_create(&th[t], NULL, worker, &jobs[t]);
    }
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    return 0;
}

/* ------------------------------------------------------------------ convergence study
 * Sec. "Convergence study": phi(x,y) = (2x, y + 0.3(1-x) sin(10 pi x)),
 * p_In = (0, 0.3), p_Out = (1, 0.7).  The pulled-back field W solves
 * J_phi W = V(phi(p)) (Eq. (VgVp)) with V = V_par + c V_perp (Eq. (vec2));
 * N = round(L/ds) uniform explicit RK steps; the error is the largest distance
 * of phi(p_i) from the view ray (caption of the table).                      */
/* Runge-Kutta-Fehlberg 4(5): stages A_rkf, 5th-order weights b_rkf (the
   solution carried on), 4th-order weights b4_rkf (the embedded estimate).    */
static const double A_rkf[6][6] = {{0},
                                   {1.0 / 4},
                                   {3.0 / 32, 9.0 / 32},
                                   {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197},
                                   {439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104},
                                   {-8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40}};
static const double b_rkf[6] = {16.0 / 135, 0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55};
static const double b4_rkf[6] = {25.0 / 216, 0, 1408.0 / 2565, 2197.0 / 4104, -1.0 / 5, 0};

/* The explicit family of the study, by its Butcher tableaux (stages, a in the
   lower triangle, b): 1 explicit Euler, 2 midpoint, 3 Kutta's third order,
   4 the classic fourth order, 5 the 3/8 rule, 6 Fehlberg's fifth order. */
static const double A_rk1[1][6] = {{0}};
static const double b_rk1[6] = {1};
static const double A_rk2[2][6] = {{0}, {0.5}};
static const double b_rk2[6] = {0, 1};
static const double A_rk3[3][6] = {{0}, {0.5}, {-1, 2}};
static const double b_rk3[6] = {1.0 / 6, 2.0 / 3, 1.0 / 6};
static const double A_rk4[4][6] = {{0}, {0.5}, {0, 0.5}, {0, 0, 1}};
static const double b_rk4[6] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
static const double A_38[4][6] = {{0}, {1.0 / 3}, {-1.0 / 3, 1}, {1, -1, 1}};
static const double b_38[6] = {1.0 / 8, 3.0 / 8, 3.0 / 8, 1.0 / 8};
static const struct {
    int stages;
    const double (*A)[6];
    const double *b;
} rk_family[7] = {{0, NULL, NULL},   {1, A_rk1, b_rk1}, {2, A_rk2, b_rk2}, {3, A_rk3, b_rk3},
                  {4, A_rk4, b_rk4}, {4, A_38, b_38},   {6, A_rkf, b_rkf}};

static void t1_phi(const double p[2], double g[2], double J[4])
{
    double x = p[0], y = p[1];
    g[0] = 2.0 * x;
    g[1] = y + 0.3 * (1.0 - x) * sin(10.0 * M_PI * x);
    J[0] = 2.0; J[1] = 0.0;
    J[2] = -0.3 * sin(10.0 * M_PI * x) + 0.3 * (1.0 - x) * 10.0 * M_PI * cos(10.0 * M_PI * x);
    J[3] = 1.0;
}

static void t1_W(const double p[2], const double gin[2], const double vpar[2], double c,
                 double w[2])
{
    double g[2], J[4];
    t1_phi(p, g, J);
    double r[2] = {gin[0] - g[0], gin[1] - g[1]};
    double dot = r[0] * vpar[0] + r[1] * vpar[1];
    double V[2] = {vpar[0] + c * (r[0] - dot * vpar[0]), vpar[1] + c * (r[1] - dot * vpar[1])};
    double det = J[0] * J[3] - J[1] * J[2];
    w[0] = (J[3] * V[0] - J[1] * V[1]) / det;
    w[1] = (-J[2] * V[0] + J[0] * V[1]) / det;
}

/* d^2 phi_2 / dx^2 of the test map (the only non-zero second derivative) */
static double t1_phi2_xx(double x)
{
    const double k = 10.0 * M_PI;
    return 0.3 * (-2.0 * k * cos(k * x) - (1.0 - x) * k * k * sin(k * x));
}

/* One implicit Euler step (Eq. (implicitEuler)) on the 2-D map: Newton on
   G(z) = z - h W(p + z) (Eq. (newtonimpliciteuler)) from the explicit Euler
   predictor, with the exact Jacobian of Eq. (JacG):
     J_phi J_G = H_phi (z - G) + (I - h J_V) J_phi,  J_V = c (v v^T - I),
   so that each Newton update solves (J_phi J_G) dz = -J_phi G, where
   J_phi G = J_phi z - h V(phi(p + z)) (Eq. (newtonimpliciteulerReformulated)).
   Returns the Newton iterations taken (-1: no convergence in 50). */
static int t1_irk1_step(double p[2], double h, const double gin[2], const double v[2], double c)
{
    double z[2], w0[2];
    t1_W(p, gin, v, c, w0);
    z[0] = h * w0[0];
    z[1] = h * w0[1];
    for (int it = 1; it <= 50; ++it) {
        const double q[2] = {p[0] + z[0], p[1] + z[1]};
        double g[2], J[4], w[2];
        t1_phi(q, g, J);
        t1_W(q, gin, v, c, w);
        const double r[2] = {gin[0] - g[0], gin[1] - g[1]};
        const double rv = r[0] * v[0] + r[1] * v[1];
        const double V[2] = {v[0] + c * (r[0] - rv * v[0]), v[1] + c * (r[1] - rv * v[1])};
        /* z - G(z) = h W(q); H_phi applied to it: column a of the matrix is
           sum_b d^2 phi / dp_a dp_b (h W)_b; only phi_2,xx is non-zero */
        const double hw[2] = {h * w[0], h * w[1]};
        double M[4];
        const double hxx = t1_phi2_xx(q[0]);
        /* (I - h J_V) = (1 + h c) I - h c v v^T */
        for (int i = 0; i < 2; ++i)
            for (int a = 0; a < 2; ++a) {
                double s = (1.0 + h * c) * J[i * 2 + a];
                for (int m = 0; m < 2; ++m) s -= h * c * v[i] * v[m] * J[m * 2 + a];
                M[i * 2 + a] = s;
            }
        M[1 * 2 + 0] += hxx * hw[0];
        const double rhs[2] = {-(J[0] * z[0] + J[1] * z[1] - h * V[0]), -(J[2] * z[0] + J[3] * z[1] - h * V[1])};
        const double det = M[0] * M[3] - M[1] * M[2];
        const double dz[2] = {(M[3] * rhs[0] - M[1] * rhs[1]) / det, (-M[2] * rhs[0] + M[0] * rhs[1]) / det};
        z[0] += dz[0];
        z[1] += dz[1];
        if (fmax(fabs(dz[0]), fabs(dz[1])) <= 1e-15) {
            p[0] += z[0];
            p[1] += z[1];
            return it;
        }
    }
    p[0] += z[0];
    p[1] += z[1];
    return -1;
}

double orc_table1_newton(int32_t method, double ds, double c, int32_t *max_newton);

double orc_table1(int32_t method, double ds, double c)
{
    return orc_table1_newton(method, ds, c, NULL);
}

/* As orc_table1; method 7 is the implicit Euler method, and *max_newton (if
   given) the most Newton iterations of any of its steps (-1: one failed). */
double orc_table1_newton(int32_t method, double ds, double c, int32_t *max_newton)
{
    const double(*A)[6] = NULL;
    const double *b = NULL;
    int st = 0;
    if (method >= 1 && method <= 6) {
        A = rk_family[method].A;
        b = rk_family[method].b;
        st = rk_family[method].stages;
    } else if (method != 7) {
        return -1.0;
    }
    if (max_newton) *max_newton = 0;
    double pin[2] = {0.0, 0.3}, pout[2] = {1.0, 0.7}, gin[2], gout[2], Jd[4];
    t1_phi(pin, gin, Jd);
    t1_phi(pout, gout, Jd);
    double vpar[2] = {gout[0] - gin[0], gout[1] - gin[1]};
    double L = sqrt(vpar[0] * vpar[0] + vpar[1] * vpar[1]);
    vpar[0] /= L; vpar[1] /= L;
    int N = (int)lround(L / ds);
    double h = L / N, p[2] = {pin[0], pin[1]}, err = 0.0;
    for (int n = 0; n < N; ++n) {
        double k[6][2];
        if (method == 7) {
            const int it = t1_irk1_step(p, h, gin, vpar, c);
            if (max_newton && (it < 0 || (*max_newton >= 0 && it > *max_newton))) *max_newton = it;
        }
        for (int i = 0; i < st; ++i) {
            double q[2] = {p[0], p[1]};
            for (int j = 0; j < i; ++j) {
                q[0] += h * A[i][j] * k[j][0];
                q[1] += h * A[i][j] * k[j][1];
            }
            t1_W(q, gin, vpar, c, k[i]);
        }
        for (int i = 0; i < st; ++i) {
            p[0] += h * b[i] * k[i][0];
            p[1] += h * b[i] * k[i][1];
        }
        double g[2];
        t1_phi(p, g, Jd);
        double r[2] = {gin[0] - g[0], gin[1] - g[1]};
        double dot = r[0] * vpar[0] + r[1] * vpar[1];
        double e = hypot(r[0] - dot * vpar[0], r[1] - dot * vpar[1]);
        if (e > err) err = e;
    }
    return err;
}

/* ------------------------------------------------------------------ method mode
 * The method itself in FP64, as a diagnostic and as the like-for-like CPU
 * baseline of the GPU path: for each segment of Algorithm "Blockwise
 * depth-sorting" the ray preimage ODE p' = W(p), J_phi(p) W = V_par + c V_perp
 * (Eqs. (odepar), (VgVp), (vec2), V_perp towards the view ray), integrated by
 * the Fehlberg 4(5) pair carrying the 5th-order solution: error
 * max_c |p5 - p4| <= tol, h <- h clamp(0.8 (tol/err)^(1/5), 0.2, 2.5) (no growth
 * right after a rejection), h <= h_max and h <= rho_step / |dn/ds|, iterates
 * clamped to P.  rho is sampled at every accepted step; between two samples it
 * is the cubic Hermite interpolant of the values and d rho/ds = grad rho . W
 * (hermite) or linear, and the interval is supersampled (Sec. "Quadrature of
 * volume render integral") with the midpoints of
 * max(n_super, span/dn, span * slope/tf_step) equal sub-steps (at most 128),
 * span the change of n over the interval, dn half the smallest knot gap of the
 * transfer function within [1/64, 1/16] and slope the transfer function's
 * largest slope over the interval's range of n; each sub-step composited by
 * Algorithm "Front-to-back compositing" with T = exp(-kappa ds).  The last step
 * ends on the exit, closing with rho there.                                  */

/* phi, J (J[r*3+q] = d phi_r / d p_q), rho and its parameter gradient at p. */
static void eval_rho_grad(const orc_patch *P, const double pin[3], double x[3], double J[9], double *rho,
                          double g[3])
{
    double Nb[3][MAXN], dNb[3][MAXN], p[3];
    for (int d = 0; d < 3; ++d) {
        p[d] = clamp01(pin[d]);
        orc_basis(P->knots[d], P->ncp[d] + P->deg[d] + 1, P->deg[d], p[d], Nb[d], dNb[d]);
    }
    const int n0 = P->ncp[0], n1 = P->ncp[1], n2 = P->ncp[2];
    double A[4] = {0, 0, 0, 0}, dA[3][4] = {{0}}, R = 0.0, dR[3] = {0, 0, 0};
    for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) {
                const double b = Nb[0][i] * Nb[1][j] * Nb[2][k];
                const double bd[3] = {dNb[0][i] * Nb[1][j] * Nb[2][k], Nb[0][i] * dNb[1][j] * Nb[2][k],
                                      Nb[0][i] * Nb[1][j] * dNb[2][k]};
                if (b == 0.0 && bd[0] == 0.0 && bd[1] == 0.0 && bd[2] == 0.0) continue;
                const size_t li = i + (size_t)n0 * (j + (size_t)n1 * k);
                const double *c = P->cp + 4 * li;
                const double w = P->rational ? c[3] : 1.0, sc = P->scalar[li];
                for (int r = 0; r < 3; ++r) A[r] += b * w * c[r];
                A[3] += b * w;
                R += b * w * sc;
                for (int q = 0; q < 3; ++q) {
                    for (int r = 0; r < 3; ++r) dA[q][r] += bd[q] * w * c[r];
                    dA[q][3] += bd[q] * w;
                    dR[q] += bd[q] * w * sc;
                }
            }
    /* quotient rule (the denominator is 1 for B-splines) */
    for (int r = 0; r < 3; ++r) x[r] = A[r] / A[3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) J[r * 3 + q] = (dA[q][r] - x[r] * dA[q][3]) / A[3];
    *rho = R / A[3];
    for (int q = 0; q < 3; ++q) g[q] = (dR[q] - *rho * dA[q][3]) / A[3];
}

/* W(p) of Eq. (VgVp); rho, grad rho at p.  Returns -1 if J is singular. */
static int method_W(const orc_patch *P, const double p[3], const double gin[3], const double d[3], double c,
                    double W[3], double *rho, double g[3])
{
    double x[3], J[9], r[3], V[3];
    eval_rho_grad(P, p, x, J, rho, g);
    for (int q = 0; q < 3; ++q) r[q] = gin[q] - x[q];
    const double rd = r[0] * d[0] + r[1] * d[1] + r[2] * d[2];
    for (int q = 0; q < 3; ++q) V[q] = d[q] + c * (r[q] - rd * d[q]);
    return solve3(J, V, W);
}

/* the transfer function's largest slope (any channel; A without the extinction)
   on interval k of n, and over the intervals of n that meet [lo, hi] together
   with their neighbours (the bound the sub-steps are counted with) */
static double tf_interval_slope(const orc_tf *tf, int k)
{
    double m = 0.0;
    if (k < 0 || k + 1 >= tf->n) return 0.0;
    for (int c = 0; c < 4; ++c) {
        const double s = fabs(tf->rgba[4 * (k + 1) + c] - tf->rgba[4 * k + c]) / (tf->x[k + 1] - tf->x[k]);
        if (s > m) m = s;
    }
    return m;
}

/* The sub-step count is an integer that floating point decides: its thresholds
   (the slope bounds, the knots, the range of n, dn and tf_step) are taken in
   binary32, the precision the GPU path holds them in, so that both sides count
   alike.  f32() rounds to it. */
static double f32(double v) { return (double)(float)v; }

static double tf_slope(const orc_tf *tf, double lo, double hi)
{
    double m = 0.0;
    lo = f32(lo);
    hi = f32(hi);
    for (int k = 0; k + 1 < tf->n; ++k) {
        /* interval k is [x_k, x_{k+1}); the first reaches down and the last up */
        const double a = k == 0 ? -INFINITY : f32(tf->x[k]), b = k + 2 == tf->n ? INFINITY : f32(tf->x[k + 1]);
        if (b <= lo || a > hi) continue;
        for (int q = k - 1; q <= k + 1; ++q) m = fmax(m, f32(tf_interval_slope(tf, q)));
    }
    return m;
}

static void method_interval(const orc_tf *tf, const orc_method_opts *mo, double ra, double ma, double rb,
                            double mb, double len, double C[3], double *A)
{
    const double inv = 1.0 / (tf->domain[1] - tf->domain[0]);
    const double sa = mo->hermite ? ma * len : rb - ra, sb = mo->hermite ? mb * len : rb - ra;
    const double span = fmax(fabs(rb - ra), 0.5 * (fabs(sa) + fabs(sb))) * inv;
    double gap = 1.0;
    for (int k = 0; k + 1 < tf->n; ++k) gap = fmin(gap, tf->x[k + 1] - tf->x[k]);
    const double dn = f32(fmin(1.0 / 16.0, fmax(1.0 / 64.0, 0.5 * gap)));
    const double na = (ra - tf->domain[0]) * inv, nb = (rb - tf->domain[0]) * inv;
    const double over = 0.25 * (fabs(sa) + fabs(sb)) * inv;
    const double slope = tf_slope(tf, fmin(na, nb) - over, fmax(na, nb) + over);
    int ns = (int)ceil(fmax(span / dn, span * slope / f32(mo->tf_step)));
    if (ns < mo->n_super) ns = mo->n_super;
    if (ns > 128) ns = 128;
    const double ds = len / ns;
    for (int j = 0; j < ns; ++j) {
        const double u = (j + 0.5) / ns, u2 = u * u, u3 = u2 * u;
        const double rho = (2 * u3 - 3 * u2 + 1) * ra + (u3 - 2 * u2 + u) * sa + (3 * u2 - 2 * u3) * rb +
                           (u3 - u2) * sb;
        double e[4];
        orc_transfer(tf, rho, e);
        const double T = exp(-e[3] * ds);
        for (int c = 0; c < 3; ++c) C[c] += (1.0 - T) * (1.0 - *A) * e[c];
        *A += (1.0 - T) * (1.0 - *A);
    }
}

/* One implicit Euler step (Eq. (implicitEuler)) from p with step h: Newton on
   G(z) = z - h W(p + z) (Eq. (newtonimpliciteuler)) from the explicit Euler
   predictor z = h W(p), each update solving (J_phi J_G) dz = -J_phi G with
     J_phi J_G = H_phi (h W(q)) + (I - h J_V) J_phi,   J_V = c (d d^T - I),
     J_phi G = J_phi z - h V(phi(q)),                   q = p + z
   (Eqs. (newtonimpliciteulerReformulated), (JacG)); every iterate p + z is
   projected onto P, so that a step that would leave P stops on its boundary.
   On return p is the new point; the Newton iterations are returned (-1: the
   iterate still moved by more than 1e-13 after 30). */
static int irk1_step(const orc_patch *P, double p[3], double h, const double gin[3], const double d[3],
                     double c, const double W0[3])
{
    double z[3] = {h * W0[0], h * W0[1], h * W0[2]};
    for (int it = 1; it <= 30; ++it) {
        double q[3], x[3], J[9], H[27], r[3], V[3], hV[3], hw[3], M[9], rhs[3], dz[3];
        for (int e = 0; e < 3; ++e) q[e] = clamp01(p[e] + z[e]);
        orc_eval_hessian(P, q, x, J, H);
        for (int e = 0; e < 3; ++e) r[e] = gin[e] - x[e];
        const double rd = r[0] * d[0] + r[1] * d[1] + r[2] * d[2];
        for (int e = 0; e < 3; ++e) {
            V[e] = d[e] + c * (r[e] - rd * d[e]);
            hV[e] = h * V[e];
        }
        if (solve3(J, hV, hw) != 0) break;
        for (int i = 0; i < 3; ++i)
            for (int a = 0; a < 3; ++a) {
                double m = (1.0 + h * c) * J[i * 3 + a];
                for (int k = 0; k < 3; ++k) m -= h * c * d[i] * d[k] * J[k * 3 + a];
                for (int b = 0; b < 3; ++b) m += H[i * 9 + a * 3 + b] * hw[b];
                M[i * 3 + a] = m;
            }
        for (int i = 0; i < 3; ++i) rhs[i] = -(J[i * 3] * z[0] + J[i * 3 + 1] * z[1] + J[i * 3 + 2] * z[2] - hV[i]);
        if (solve3(M, rhs, dz) != 0) break;
        /* the iterate projected onto P; converged once it moves by <= 1e-13 */
        double mv = 0.0;
        for (int e = 0; e < 3; ++e) {
            const double zn = clamp01(p[e] + z[e] + dz[e]) - p[e];
            mv = fmax(mv, fabs(zn - z[e]));
            z[e] = zn;
        }
        if (mv <= 1e-13) {
            for (int e = 0; e < 3; ++e) p[e] = clamp01(p[e] + z[e]);
            return it;
        }
    }
    for (int e = 0; e < 3; ++e) p[e] = clamp01(p[e] + z[e]);
    return -1;
}

/* The fixed-step methods of Sec. "ODE Based Algorithm" (method 1..6 the
   explicit family, 7 implicit Euler) and Sec. "Root Finding Based Algorithm"
   (8: every sample's preimage by Newton on phi(p) = g, from the previous
   sample's p moved along J^-1 d).  No error control: every step is h_max,
   shortened where rho changes by more than rho_step in n (h >= h_min) and at
   the exit; each step's end is sampled (rho, d rho/ds) and the interval
   composited as in the adaptive mode.  Explicit stages and steps are clamped
   to P. */
static void method_fixed_steps(const orc_patch *P, const orc_tf *tf, const orc_method_opts *mo, double scale,
                               double hmax, double hmin, double L, double gin[3], const double d[3], double p[3],
                               double W[3], double rho_a, double m_a, double rho_out, double m_out, double C[3],
                               double *A, long long *steps, pix_diag_t *dg)
{
    const double inv = 1.0 / (tf->domain[1] - tf->domain[0]);
    const int method = mo->method;
    const double c = method == 8 ? 0.0 : mo->c_perp;
    double s = 0.0, rho, g[3];
    for (int it = 0; it < 200000 && *A < 1.0 - 1e-4; ++it) {
        const double hf = mo->rho_step / (fabs(m_a) * inv + 1e-300);
        double hh = hmax < hf ? hmax : fmax(hf, hmin);
        hh = fmin(hh, L - s);
        ++*steps;
        if (L - s - hh <= 1e-6 * L) {   /* the step ends on the exit */
            method_interval(tf, mo, rho_a, m_a, rho_out, m_out, hh, C, A);
            return;
        }
        if (method >= 1 && method <= 6) {
            const int st = rk_family[method].stages;
            double k[6][3];
            for (int i = 0; i < st; ++i) {
                double q[3], rr, gg[3];
                if (i == 0) {
                    for (int e = 0; e < 3; ++e) k[0][e] = W[e];
                    continue;
                }
                for (int e = 0; e < 3; ++e) {
                    q[e] = p[e];
                    for (int j = 0; j < i; ++j) q[e] += hh * rk_family[method].A[i][j] * k[j][e];
                    q[e] = clamp01(q[e]);
                }
                method_W(P, q, gin, d, c, k[i], &rr, gg);
            }
            for (int e = 0; e < 3; ++e) {
                double v = p[e];
                for (int i = 0; i < st; ++i) v += hh * rk_family[method].b[i] * k[i][e];
                p[e] = clamp01(v);
            }
        } else if (method == 7) {
            irk1_step(P, p, hh, gin, d, c, W);
        } else {
            double x[3], J[9], Wt[3], pred[3], gn[3], pr[3];
            eval_rho_grad(P, p, x, J, &rho, g);
            if (solve3(J, d, Wt) != 0) Wt[0] = Wt[1] = Wt[2] = 0.0;
            for (int e = 0; e < 3; ++e) {
                pred[e] = clamp01(p[e] + hh * Wt[e]);
                gn[e] = gin[e] + hh * d[e];
            }
            orc_invert(P, gn, pred, scale, pr, NULL);
            for (int e = 0; e < 3; ++e) p[e] = pr[e];
        }
        for (int e = 0; e < 3; ++e) gin[e] += hh * d[e];
        s += hh;
        diag_sample(dg, P, p);
        method_W(P, p, gin, d, c, W, &rho, g);
        const double m_b = g[0] * W[0] + g[1] * W[1] + g[2] * W[2];
        method_interval(tf, mo, rho_a, m_a, rho, m_b, hh, C, A);
        rho_a = rho;
        m_a = m_b;
    }
}

/* The convergence study on a block of a spline model: the ray from phi(p_in) to
   phi(p_out), N = round(L/ds) uniform steps of method 1..6 (explicit family)
   or 7 (implicit Euler) with V = V_par + c V_perp; the error is the largest
   distance of phi(p_i) from the ray (the measure of Table
   "2dcomparisonefficiency").  *max_newton as in orc_table1_newton.          */
double orc_path_error(const orc_patch *P, const double p_in[3], const double p_out[3], int32_t method, double ds,
                      double c, int32_t *max_newton)
{
    if (!((method >= 1 && method <= 7) && ds > 0)) return -1.0;
    double x0[3], x1[3], J[9], rho, g[3], d[3], gin[3], p[3], W[3];
    eval_rho_grad(P, p_in, x0, J, &rho, g);
    eval_rho_grad(P, p_out, x1, J, &rho, g);
    for (int e = 0; e < 3; ++e) d[e] = x1[e] - x0[e];
    const double L = norm3(d);
    for (int e = 0; e < 3; ++e) {
        d[e] /= L;
        gin[e] = x0[e];
        p[e] = p_in[e];
    }
    const int N = (int)lround(L / ds);
    const double h = L / N;
    double err = 0.0;
    if (max_newton) *max_newton = 0;
    for (int n = 0; n < N; ++n) {
        method_W(P, p, gin, d, c, W, &rho, g);
        if (method == 7) {
            const int it = irk1_step(P, p, h, gin, d, c, W);
            if (max_newton && (it < 0 || (*max_newton >= 0 && it > *max_newton))) *max_newton = it;
        } else {
            const int st = rk_family[method].stages;
            double k[6][3];
            for (int e = 0; e < 3; ++e) k[0][e] = W[e];
            for (int i = 1; i < st; ++i) {
                double q[3], rr, gg[3];
                for (int e = 0; e < 3; ++e) {
                    q[e] = p[e];
                    for (int j = 0; j < i; ++j) q[e] += h * rk_family[method].A[i][j] * k[j][e];
                }
                method_W(P, q, gin, d, c, k[i], &rr, gg);
            }
            for (int e = 0; e < 3; ++e)
                for (int i = 0; i < st; ++i) p[e] += h * rk_family[method].b[i] * k[i][e];
        }
        double x[3], r[3];
        eval_rho_grad(P, p, x, J, &rho, g);
        for (int e = 0; e < 3; ++e) r[e] = gin[e] - x[e];
        const double rd = r[0] * d[0] + r[1] * d[1] + r[2] * d[2];
        for (int e = 0; e < 3; ++e) r[e] -= rd * d[e];
        err = fmax(err, norm3(r));
    }
    return err;
}

static void method_segment(const orc_patch *P, const orc_tf *tf, const orc_method_opts *mo, double scale,
                           const double o[3], const double d[3], const orc_fragment *fi, const orc_fragment *fo,
                           double out[4], long long *steps, pix_diag_t *dg)
{
    if (dg) dg->t_prev = fi->t;
    const double L = fo->t - fi->t, hmax = mo->h_max > 0 ? mo->h_max : scale / 32.0;
    const double hmin = fmin(hmax, 1.5625e-6 * scale);
    double gin[3], p[3], W[3], rho, g[3], C[3] = {0, 0, 0}, A = 0.0;
    for (int q = 0; q < 3; ++q) {
        gin[q] = o[q] + fi->t * d[q];
        p[q] = fi->p[q];
    }
    method_W(P, p, gin, d, mo->c_perp, W, &rho, g);
    double rho_a = rho, m_a = g[0] * W[0] + g[1] * W[1] + g[2] * W[2];
    double rho_out, m_out, Wo[3], go[3];
    {
        double x[3], J[9];
        eval_rho_grad(P, fo->p, x, J, &rho_out, go);
        if (solve3(J, d, Wo) != 0) Wo[0] = Wo[1] = Wo[2] = 0.0;
        m_out = go[0] * Wo[0] + go[1] * Wo[1] + go[2] * Wo[2];
    }
    const double inv = 1.0 / (tf->domain[1] - tf->domain[0]);
    if (mo->method != 0) {
        method_fixed_steps(P, tf, mo, scale, hmax, hmin, L, gin, d, p, W, rho_a, m_a, rho_out, m_out, C, &A, steps,
                           dg);
        if (dg && fo->t < dg->t_prev) ++dg->order_bad;
        out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = A;
        return;
    }
    double s = 0.0, h = fmin(L, hmax);
    int rejected = 0;
    for (int it = 0; it < 200000 && s < L && A < 1.0 - 1e-4; ++it) {
        const double hf = mo->rho_step / (fabs(m_a) * inv + 1e-300);
        if (h > hf) h = fmax(hf, hmin);
        const double hh = fmin(h, L - s);
        double k[6][3], p5[3], err = 0.0;
        for (int i = 0; i < 6; ++i) {
            double q[3], rr, gg[3];
            for (int c = 0; c < 3; ++c) {
                q[c] = p[c];
                for (int j = 0; j < i; ++j) q[c] += hh * A_rkf[i][j] * k[j][c];
                q[c] = clamp01(q[c]);
            }
            if (i == 0) {
                for (int c = 0; c < 3; ++c) k[0][c] = W[c];
            } else {
                method_W(P, q, gin, d, mo->c_perp, k[i], &rr, gg);
            }
        }
        for (int c = 0; c < 3; ++c) {
            double a5 = p[c], a4 = p[c];
            for (int i = 0; i < 6; ++i) {
                a5 += hh * b_rkf[i] * k[i][c];
                a4 += hh * b4_rkf[i] * k[i][c];
            }
            p5[c] = a5;
            if (fabs(a5 - a4) > err) err = fabs(a5 - a4);
        }
        ++*steps;
        const int accept = err <= mo->tol || hh <= hmin;
        if (accept) {
            s += hh;
            if (L - s <= 1e-6 * L) {
                method_interval(tf, mo, rho_a, m_a, rho_out, m_out, hh, C, &A);
                break;
            }
            for (int c = 0; c < 3; ++c) p[c] = clamp01(p5[c]);
            diag_sample(dg, P, p);
            method_W(P, p, gin, d, mo->c_perp, W, &rho, g);
            const double m_b = g[0] * W[0] + g[1] * W[1] + g[2] * W[2];
            method_interval(tf, mo, rho_a, m_a, rho, m_b, hh, C, &A);
            rho_a = rho;
            m_a = m_b;
        }
        double fac = err > 0.0 ? 0.8 * pow(mo->tol / err, 0.2) : 2.5;
        fac = fac < 0.2 ? 0.2 : (fac > 2.5 ? 2.5 : fac);
        if (accept && rejected && fac > 1.0) fac = 1.0;
        rejected = !accept;
        h = fmin(hmax, fmax(hmin, hh * fac));
    }
    if (dg && fo->t < dg->t_prev) ++dg->order_bad;
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = A;
}

typedef struct {
    const orc_scene *s;
    const orc_camera *cam;
    const orc_tf *tf;
    const orc_method_opts *mo;
    const int64_t *pixels;
    int64_t npix;
    double *rgba;
    double *dp;
    int32_t *order_bad;
    long long steps;
    int tid, nthreads;
} mjob_t;

static void *method_worker(void *arg)
{
    mjob_t *j = arg;
    orc_fragment *fr = malloc(sizeof(orc_fragment) * FRAG_CAP);
    int (*pairs)[2] = malloc(sizeof(int[2]) * FRAG_CAP);
    for (int64_t i = j->tid; i < j->npix; i += j->nthreads) {
        const int64_t pix = j->pixels ? j->pixels[i] : i;
        double o[3], d[3], *out = j->rgba + 4 * i;
        orc_camera_ray(j->cam, pix % j->cam->width + 0.5, pix / j->cam->width + 0.5, o, d);
        out[0] = out[1] = out[2] = out[3] = 0.0;
        const int n = orc_ray_fragments(j->s, o, d, fr, FRAG_CAP);
        if (n <= 0) continue;
        int anom = 0;
        const int np = pair_fragments(fr, n, 1e-9 * j->s->scale, 0, pairs, &anom);
        /* front to back by entry depth */
        for (int a = 1; a < np; ++a)
            for (int b = a; b > 0 && fr[pairs[b][0]].t < fr[pairs[b - 1][0]].t; --b) {
                int t0 = pairs[b][0], t1 = pairs[b][1];
                pairs[b][0] = pairs[b - 1][0]; pairs[b][1] = pairs[b - 1][1];
                pairs[b - 1][0] = t0; pairs[b - 1][1] = t1;
            }
        double C[3] = {0, 0, 0}, A = 0.0;
        pix_diag_t dgv = {j->cam, pix, o, d, 0.0, 0.0, 0};
        pix_diag_t *dg = (j->dp || j->order_bad) ? &dgv : NULL;
        for (int k = 0; k < np && A < 1.0 - 1e-4; ++k) {
            double r[4];
            const orc_fragment *fi = &fr[pairs[k][0]], *fo = &fr[pairs[k][1]];
            method_segment(&j->s->patches[fo->patch], j->tf, j->mo, j->s->scale, o, d, fi, fo, r, &j->steps, dg);
            for (int c = 0; c < 3; ++c) C[c] += (1.0 - A) * r[c];
            A += (1.0 - A) * r[3];
        }
        out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = A;
        if (j->dp) j->dp[i] = dgv.dp_max;
        if (j->order_bad) j->order_bad[i] = dgv.order_bad;
    }
    free(fr);
    free(pairs);
    return NULL;
}

int32_t orc_render_pixels_method(const orc_scene *s, const orc_camera *cam, const orc_tf *tf,
                                 const orc_method_opts *mo, const int64_t *pixels, int64_t npix, double *rgba,
                                 int64_t *rk_steps, double *dp, int32_t *order_bad)
{
    if (!s || !cam || !tf || !mo || !rgba || tf->n < 2 || !(mo->tol > 0)) return -1;
    int nt = mo->nthreads > 0 ? mo->nthreads : (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1) nt = 1;
    if (nt > 256) nt = 256;
    pthread_t th[256];
    mjob_t jobs[256];
    for (int t = 0; t < nt; ++t) {
        jobs[t] = (mjob_t){s, cam, tf, mo, pixels, npix, rgba, dp, order_bad, 0, t, nt};
        pthread_create(&th[t], NULL, method_worker, &jobs[t]);
    }
    long long total = 0;
    for (int t = 0; t < nt; ++t) {
        pthread_join(th[t], NULL);
        total += jobs[t].steps;
    }
    if (rk_steps) *rk_steps = total;
    return 0;
}
