/*
 * FP64 CPU oracle for isogeometric volume rendering (Fuchs & Hjelmervik,
 * "Interactive Isogeometric Volume Visualization with Pixel-Accurate Geometry").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU library; the two meet only through the seeded
 * scene generators.
 *
 * What it computes (per pixel, for the ray e + s*d, s > 0):
 *   - every crossing of the ray with the six boundary faces of every block
 *     (Sec. "View-Ray Intersections with Surfaces"), found by Bezier extraction,
 *     convex-hull culling and subdivision, then FP64 Newton;
 *   - the entry/exit pairs of Algorithm "Blockwise depth-sorting";
 *   - the emission-absorption integral of Eq. (volRenderIntegral) with
 *     rho_gamma(s) = rho(phi^-1(gamma(s))) of Eq. (rhoPhiInv), by the midpoint
 *     rule on fine panels (Algorithm "Front-to-back compositing" applied to
 *     constant panels, which is exact for them) with the preimage of every panel
 *     midpoint found by Newton's method of Eq. (newtonsmethod), plus one
 *     Richardson extrapolation;
 *   - the explicit Runge-Kutta family of Sec. "ODE Based Algorithm" on the
 *     analytic map of the convergence study (Table "2dcomparisonefficiency").
 * All arithmetic is IEEE double.  Errors are returned as negative ints.
 */
#ifndef IVR_ORACLE_H
#define IVR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t deg[3];
    int32_t ncp[3];
    const double *knots[3];   /* ncp[d]+deg[d]+1 values, clamped, on [0,1] */
    const double *cp;         /* ncp0*ncp1*ncp2 x (x,y,z,w), i fastest     */
    const double *scalar;     /* ncp0*ncp1*ncp2 coefficients of rho         */
    int32_t rational;         /* 1: NURBS (w used), 0: plain B-spline       */
    const double *disp;       /* NULL, or ncp0*ncp1*ncp2 x (u_x,u_y,u_z): the
                                 displacement spline u on the same basis      */
} orc_patch;

/* Scalar field sampled along the ray (orc_opts.field): the block's scalar
   spline rho, or a field derived from the maps on the fly. */
#define ORC_FIELD_SCALAR 0
#define ORC_FIELD_PARAM_QUALITY 1   /* Eq. (paramQuality): det J_phi / |J_phi|_F */
#define ORC_FIELD_VON_MISES 2       /* Eq. (vonMises), read with its squares and
                                       root, of the symmetrised J_{u o phi^-1}   */

typedef struct {
    int32_t n;                /* number of knots of the transfer function   */
    const double *x;          /* n abscissae on [0,1], increasing           */
    const double *rgba;       /* n x (R,G,B,A)                              */
    double extinction;        /* kappa = extinction * A                     */
    double domain[2];         /* rho -> (rho - lo) / (hi - lo), clamped     */
} orc_tf;

typedef struct {
    double eye[3], target[3], up[3];
    double fov_y_deg;
    int32_t width, height;
} orc_camera;

typedef struct {
    double panels_per_scale;  /* panel width = scale / panels_per_scale      */
    int32_t richardson;       /* 1: combine h and h/2 as (4 I_{h/2} - I_h)/3 */
    int32_t nthreads;         /* 0: all online cores                         */
    double self_tol;          /* halve the panels while |I_h - I_{h/2}| > this */
    /* Sec. "Cutting and Near Clip Planes".  Cutting plane (cut != 0): only
       points g with cut_normal . (g - cut_point) >= 0 are rendered.  Near clip
       plane (near_clip > 0): only points at least near_clip in front of the eye
       along the view direction; a block that the near plane cuts is entered
       there.                                                                   */
    int32_t cut;
    double cut_point[3], cut_normal[3];
    double near_clip;
    int32_t field;            /* ORC_FIELD_*                                  */
} orc_opts;

typedef struct orc_scene orc_scene;

/* Fragment record returned by orc_ray_fragments. */
typedef struct {
    double t;                 /* ray parameter (unit direction)             */
    double p[3];              /* parameter point on the block boundary      */
    int32_t patch, face;      /* face 0..5 = u0,u1,v0,v1,w0,w1              */
    int32_t entering;         /* 1: ray enters the block here               */
    int32_t pad;
} orc_fragment;

/* Per-pixel diagnostics. */
typedef struct {
    int32_t n_fragments, n_segments, n_anomalies, n_newton_fail;
    double self_error;        /* max |I_h - I_{h/2}| over channels/segments  */
    double first_chord;       /* t_out - t_in of the first segment (0: none) */
} orc_pixel_diag;

orc_scene *orc_prepare(const orc_patch *patches, int32_t n, double scale);
void orc_free(orc_scene *s);

/* All B-spline basis functions N_{i,p}(u) and their derivatives, i=0..nk-p-2. */
int32_t orc_basis(const double *t, int32_t nk, int32_t p, double u, double *N, double *dN);
/* phi, its Jacobian (row-major J[r*3+c] = d phi_r / d p_c) and rho at p. */
int32_t orc_eval(const orc_patch *P, const double p[3], double x[3], double J[9], double *rho);
/* Newton preimage of g with line search and clamping to [0,1]^3. */
int32_t orc_invert(const orc_patch *P, const double g[3], const double seed[3], double scale,
                   double p_out[3], int32_t *iterations);
/* Brute-force point location (tests only): for each of n points g[3i..], the
   first block whose map reaches it by Newton inversion (hint: block[i] >= 0 and
   p[3i..] on entry; block[i] = -2: point i-1's result), -1 if none; its
   parameters p[3i..] and rho[i] (rho may be NULL). */
int32_t orc_locate(const orc_scene *s, const double *g, int64_t n, int32_t *block, double *p,
                   double *rho);
/* Pinhole ray through pixel position (px, py) (pixel centres at i+0.5). */
void orc_camera_ray(const orc_camera *c, double px, double py, double o[3], double d[3]);
/* Transfer function at rho: (R,G,B,kappa). */
void orc_transfer(const orc_tf *tf, double rho, double out[4]);
/* Every non-grazing boundary crossing of the ray, sorted by t. Returns count or <0. */
int32_t orc_ray_fragments(const orc_scene *s, const double o[3], const double d[3],
                          orc_fragment *out, int32_t cap);
/* Render a list of pixels (linear index row*width+col); NULL list = whole image. */
int32_t orc_render_pixels(const orc_scene *s, const orc_camera *cam, const orc_tf *tf,
                          const orc_opts *opts, const int64_t *pixels, int64_t npix,
                          double *rgba, double *depth, orc_pixel_diag *diag);
/* Method mode: the GPU path's method in FP64 (ray preimage ODE by adaptive
   RKF45 or a fixed-step method, Hermite or linear rho between samples,
   supersampling, Algorithm "Front-to-back compositing"), a diagnostic and the
   like-for-like CPU baseline.  Writes RGBA per pixel and the steps (attempts)
   in all. */
typedef struct {
    double tol, h_max, c_perp, rho_step, tf_step;  /* h_max <= 0: scale/32       */
    int32_t n_super, hermite, nthreads;
    /* 0 adaptive RKF45; fixed steps: 1..6 the explicit family of the
       convergence study (Euler, midpoint, Kutta, classic, 3/8, Fehlberg 5th),
       7 implicit Euler, 8 root finding (Sec. "Root Finding Based Algorithm") */
    int32_t method;
} orc_method_opts;
int32_t orc_render_pixels_method(const orc_scene *s, const orc_camera *cam, const orc_tf *tf,
                                 const orc_method_opts *mo, const int64_t *pixels, int64_t npix, double *rgba,
                                 int64_t *rk_steps, double *dp, int32_t *order_bad);
/* Eq. (deltaP): 2 |pi_s(g) - pixel centre|_inf in pixels for point g and the
   pixel (row*width + col) of camera c.  The method mode writes per pixel (when
   dp / order_bad are not NULL) the largest Delta P of the interior samples and
   the number of samples whose projection onto the ray lies before the previous
   one's (the segment's entry and exit included as the first and last). */
double orc_delta_p(const orc_camera *c, int64_t pixel, const double g[3]);
/* Convergence study: error of an RK method on the analytic 2-D map.
   method 1 Euler, 2 midpoint, 3 Kutta, 4 classic, 5 3/8-rule, 6 Fehlberg (5th),
   7 implicit Euler. */
double orc_table1(int32_t method, double ds, double c);
/* method 7: implicit Euler (Eq. (implicitEuler)) by Newton with the exact J_G of
   Eq. (JacG); *max_newton: most Newton iterations of a step (-1: one failed). */
double orc_table1_newton(int32_t method, double ds, double c, int32_t *max_newton);
/* The convergence study on block P: the ray from phi(p_in) to phi(p_out) by
   N = round(L/ds) uniform steps of method 1..7; largest distance of phi(p_i)
   from the ray.  *max_newton as in orc_table1_newton. */
double orc_path_error(const orc_patch *P, const double p_in[3], const double p_out[3], int32_t method, double ds,
                      double c, int32_t *max_newton);
/* The value of field ORC_FIELD_* at parameter point p of block P (0, or -1
   where the field needs a displacement the block does not have or J_phi is
   singular). */
int32_t orc_field(const orc_patch *P, const double p[3], int32_t field, double *value);
/* phi, J and the Hessian H[r*9 + a*3 + b] = d^2 phi_r / dp_a dp_b at p. */
int32_t orc_eval_hessian(const orc_patch *P, const double p[3], double x[3], double J[9], double H[27]);

#ifdef __cplusplus
}
#endif
#endif
