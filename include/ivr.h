/*
 * ivr — isogeometric volume rendering on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the per-pixel hot path of Fuchs & Hjelmervik, "Interactive
 * Isogeometric Volume Visualization with Pixel-Accurate Geometry" (IEEE TVCG
 * 2015).  For every pixel the library
 *   1. finds every crossing of the view ray with the six boundary faces of every
 *      block (Sec. "View-Ray Intersections with Surfaces"; here by Newton on the
 *      face equations of Eq. (F)/(newtonsmethod), FP32 iterations followed by an
 *      FP64 refinement), recording {depth, parameter, block, front-facing};
 *   2. pairs them per block by Algorithm "Blockwise depth-sorting";
 *   3. integrates the parameter-space ray p' = W(p), J_phi(p) W(p) = V(phi(p))
 *      with V = V_par + c V_perp (Eqs. (odepar), (VgVp), (vec2)) from each entry
 *      to its exit with an adaptive embedded Runge-Kutta-Fehlberg 4(5) scheme;
 *   4. samples rho at every accepted step, applies the transfer function with
 *      supersampling (Sec. "Quadrature of volume render integral") and composites
 *      front to back by Algorithm "Front-to-back compositing";
 *   5. merges the per-segment results of a pixel front to back.
 *
 * Conventions
 *   - All functions return ivr_status: 0 on success, a negative code on error.
 *     A failing call leaves the context as it was; ivr_last_error() describes
 *     the failure.  No C++ exception or abort crosses this interface.
 *   - A context belongs to one device and one HIP stream and is not thread-safe.
 *   - Host arrays passed in are copied before the call returns; the caller keeps
 *     ownership.  Output buffers are caller-owned device memory; results are
 *     written asynchronously on the context's stream.
 */
#ifndef IVR_H
#define IVR_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ivr_status;
#define IVR_OK 0
#define IVR_EINVAL (-1)     /* invalid argument                               */
#define IVR_ENOMEM (-2)     /* device allocation failed                       */
#define IVR_EDEVICE (-3)    /* no usable gfx950 device / HIP runtime error    */
#define IVR_ESTATE (-4)     /* call not valid in the current state            */
#define IVR_EOVERFLOW (-5)  /* a fixed capacity was exceeded                  */

typedef struct ivr_ctx ivr_ctx;

/* One block (patch) of the model, Eq. (Bspline) and Sec. "Approach and
 * Implementation" (blocks G_alpha with phi_alpha and rho_alpha on P_alpha).
 *   degree[d]   polynomial degree per direction, 1..3; a block whose directions
 *               differ is raised at upload to its largest degree in every
 *               direction (exact degree elevation: knot multiplicities grow by
 *               the difference, coefficients by collocation), which the kernels
 *               then evaluate; a block is also split (exactly) at every interior
 *               knot of full multiplicity, where it is only C0, into blocks
 *               that meet there as at any conforming interface, so that the
 *               integrator meets smooth blocks only.  Block indices used by the
 *               MLP functions count the blocks after these splits (the same as
 *               the input's when no block has such a knot)
 *   ncp[d]      control points per direction, >= degree+1
 *   knots[d]    ncp[d]+degree[d]+1 non-decreasing values, clamped (first and last
 *               value repeated degree+1 times); mapped affinely onto [0,1]
 *   cp          ncp0*ncp1*ncp2 records (x, y, z, w), i fastest then j then k;
 *               w > 0 is used only when rational != 0
 *   scalar      ncp0*ncp1*ncp2 coefficients of rho (same layout); for NURBS rho
 *               uses the same rational basis as the geometry                   */
typedef struct {
    int32_t degree[3];
    int32_t ncp[3];
    const double *knots[3];
    const double *cp;
    const double *scalar;
    int32_t rational;
    const double *displacement;   /* NULL, or ncp0*ncp1*ncp2 x (u_x,u_y,u_z): a
                                     displacement spline u on the block's own
                                     (rational) basis, for IVR_FIELD_VON_MISES */
} ivr_patch_desc;

/* Pinhole camera: the ray of pixel (i, j), row 0 at the top, passes through the
 * pixel centre (i+1/2, j+1/2); vertical field of view fov_y_deg. */
typedef struct {
    double eye[3], target[3], up[3];
    double fov_y_deg;
    int32_t width, height;
} ivr_camera;

/* Transfer function (Eq. (emissionabsorption)): piecewise-linear RGBA over the
 * normalised value n = clamp((rho - domain[0]) / (domain[1] - domain[0]), 0, 1)
 * with n_knots (2..16) increasing abscissae x[] from 0 to 1 and rgba[4*n_knots];
 * extinction kappa = extinction * A, emission RGB (not premultiplied). */
typedef struct {
    int32_t n_knots;
    const double *x;
    const double *rgba;
    double extinction;
    double domain[2];
} ivr_transfer_fn;

#define IVR_PRECISION_FP32 0   /* FP32 kernels, FP64 boundary-root refinement  */
#define IVR_PRECISION_FP64 1   /* every step in FP64                           */
#define IVR_SEED_PLAIN 0       /* face Newton from the element centre              */
#define IVR_SEED_MLP 1         /* from the block's trained inverse-map MLP         */
#define IVR_SEED_BOX 2         /* from the ray's passage through the element box   */
#define IVR_RHO_LINEAR 0       /* rho linear between samples (as in the paper)  */
#define IVR_RHO_HERMITE 1      /* cubic Hermite from rho and d rho/ds           */
#define IVR_INTERIOR_ODE 0     /* the ray preimage ODE by adaptive RKF45 (Sec. "ODE
                                  Based Algorithm")                               */
#define IVR_INTERIOR_RF 1      /* every sample's preimage by Newton, seeded from the
                                  previous sample (Sec. "Root Finding Based
                                  Algorithm"); steps bounded as for the ODE        */
/* The fixed-step methods of the convergence study (Sec. "ODE Based Algorithm",
   Table "2dcomparisonefficiency") on the same ODE: no error control; every step
   is h_max, shortened where rho changes by more than rho_step and at the exit
   (as for IVR_INTERIOR_RF), and each step's end is a sample.                  */
#define IVR_INTERIOR_RK1 2     /* explicit Euler, Eq. (explicitEuler)              */
#define IVR_INTERIOR_RK2 3     /* midpoint rule (second order)                     */
#define IVR_INTERIOR_RK3 4     /* Kutta's third-order method                       */
#define IVR_INTERIOR_RK4 5     /* the classic fourth-order method                  */
#define IVR_INTERIOR_RK4_38 6  /* the 3/8 rule (fourth order)                      */
#define IVR_INTERIOR_RKF5 7    /* Fehlberg's fifth-order solution, fixed step       */
#define IVR_INTERIOR_IRK1 8    /* implicit Euler, Eq. (implicitEuler): Newton on
                                  G(z) = z - h W(p + z) with the exact J_G of
                                  Eq. (JacG) (Hessian of the map), iterates
                                  projected onto P; a step whose Newton does not
                                  converge in 16 iterations is taken as it
                                  stands and flagged RESTART_FAIL               */

/* The value sampled along the ray.  The derived fields are computed from the
   maps at every sample. */
#define IVR_FIELD_SCALAR 0         /* the blocks' scalar splines rho              */
#define IVR_FIELD_PARAM_QUALITY 1  /* det J_phi / |J_phi|_F, Sec. "Parametrization
                                      Quality of Geometry", Eq. (paramQuality)  */
#define IVR_FIELD_VON_MISES 2      /* von Mises value of the symmetrised Jacobian
                                      of u o phi^-1 for the blocks' displacement
                                      splines u (Eq. (vonMises), with the squares
                                      and root its print lacks); every block must
                                      carry one                                 */

/* Stopping rule of the Newton iteration of a root-finding sample (Sec. "Root
   Finding Based Algorithm"). */
#define IVR_NEWTON_STOP_TOL 0      /* |phi(p) - g| <= 2e-6 of the scale (FP32) or
                                      1e-12 (FP64)                              */
#define IVR_NEWTON_STOP_FRUSTUM 1  /* the paper's pixel-accurate rule: |phi(p) - g|
                                      at most g's distance to the boundary of the
                                      pixel's frustum (not below the TOL rule)  */

/* Render options (ivr_default_opts fills the defaults given in brackets). */
typedef struct {
    int32_t precision;          /* IVR_PRECISION_*                          [FP32] */
    double rk_tol;              /* RKF45 local error bound on p (inf-norm) [1e-5] */
    double h_max;               /* largest step, in world units along the ray;
                                   <= 0: scale/32; half of it on a segment
                                   with a singular end                      [0]   */
    double c_perp;              /* weight c of V_perp in Eq. (vec2)         [1]   */
    int32_t n_super;            /* supersampling sub-steps per RK step      [4]   */
    double det_fp64_threshold;  /* |det J| below it: the 3x3 solve of W (and of
                                   a Newton step) in FP64               [1e-6] */
    int32_t max_fragments;      /* boundary crossings kept per ray, 2..64   [64]  */
    int32_t seed_mode;          /* IVR_SEED_*: first Newton seed of a face root [BOX]*/
    double early_term;          /* stop a segment once alpha >= 1-early_term [1e-4]*/
    int32_t max_newton_iter;    /* FP32 Newton iterations per face root     [16]  */
    int32_t rho_interp;         /* IVR_RHO_*: rho between two samples  [HERMITE] */
    int32_t timing;             /* 1: record HIP events around every phase of
                                   this render for ivr_phase_times (no sync) [0] */
    double tf_step;             /* largest change of the transfer function's
                                   output per supersampling sub-step: more
                                   sub-steps where it is steep       [0.025] */
    double rho_step;            /* largest change of rho per step, as a
                                   fraction of the transfer function's domain:
                                   limits h where rho changes fast     [0.1] */
    int32_t cand_per_pixel;     /* capacity of the candidate list (element
                                   boxes a ray hits, solved 64 at a time across
                                   rays) per pixel on average, 0..64: the rays
                                   of a 64-pixel tile whose candidates do not
                                   fit are traversed again and solved ray by
                                   ray (0: every ray); same image       [8]   */
    double det_singular;        /* |det J_phi| below it at a segment end makes
                                   the end singular, Eq. (degeneracyfix): a
                                   singular entry is moved along the ray and
                                   found again by Newton, the integration stops
                                   short of a singular exit            [1e-6] */
    double drift_tol;           /* largest distance of phi(p) from the ray point
                                   of its arc length, as a fraction of the
                                   model's scale, checked before every sample:
                                   beyond it the point is found again by Newton
                                   from p (from the block's network with MLP
                                   seeds) before it is sampled; 0: no check [1e-4] */
    int32_t interior;           /* IVR_INTERIOR_*: how a segment's samples find
                                   their parameter points                 [ODE] */
    int32_t cut;                /* 1: a cutting plane (Sec. "Cutting and Near Clip
                                   Planes"): only points g with
                                   cut_normal . (g - cut_point) >= 0 are
                                   rendered; a segment cut by it starts or ends
                                   on it, that end's parameter point found by
                                   Newton (from the block centre, or the block's
                                   network with MLP seeds)                  [0] */
    double cut_point[3], cut_normal[3];
    double near_clip;           /* > 0: the near plane, this far in front of the
                                   eye along the view direction; only points
                                   beyond it are rendered, and a block it cuts is
                                   entered there (an exit without an entry in
                                   front); 0: none                          [0] */
    int32_t newton_stop;        /* IVR_NEWTON_STOP_*: when a root-finding
                                   sample's Newton stops                [TOL] */
    int32_t field;              /* IVR_FIELD_*: the value sampled along the ray;
                                   a derived field comes with its exact
                                   gradient (from the Hessian of the maps), so
                                   rho_interp and the step bounds work as for
                                   the scalar field; derived fields run with
                                   the ODE and RF interior methods   [SCALAR] */
} ivr_render_opts;

/* Per-pixel flags (ivr_view.flags_dev): OR of the events of the pixel's ray. */
#define IVR_FLAG_ANOMALY 1u              /* a crossing left unpaired              */
#define IVR_FLAG_FRAGMENT_OVERFLOW 2u    /* crossings dropped (max_fragments)     */
#define IVR_FLAG_SEGMENT_OVERFLOW 4u     /* segments dropped (capacity)           */
#define IVR_FLAG_ITER_CAP 8u             /* a segment stopped at the RK step cap  */
#define IVR_FLAG_DRIFT_RESTART 16u       /* a segment drifted off the ray and was
                                            put back on it by Newton             */
#define IVR_FLAG_RESTART_FAIL 32u        /* such a Newton did not converge (also
                                            a root-finding sample's or an
                                            implicit Euler step's Newton)        */
#define IVR_FLAG_DEGENERATE 64u          /* a segment end with singular J_phi     */
#define IVR_FLAG_DEPTH_ORDER 128u        /* samples out of depth order (ivr_view
                                            dp_dev given)                        */

/* Counters of one render (filled when a non-NULL ivr_stats* is passed; that
 * forces a stream synchronisation). */
typedef struct {
    uint64_t rays;              /* pixels rendered                               */
    uint64_t segments;          /* entry/exit pairs integrated                   */
    uint64_t fragments;         /* boundary crossings kept                       */
    uint64_t anomalies;         /* crossings left unpaired by the pairing        */
    uint64_t fragment_overflow; /* crossings dropped (fixed capacities)           */
    uint64_t segment_overflow;  /* segments dropped (per-pixel capacity)         */
    uint64_t box_tests;         /* ray/box slab tests                            */
    uint64_t face_newton;       /* candidates solved (face Newton started; a
                                   second search on one element counts once)    */
    uint64_t face_newton_iter;  /* FP32 face Newton iterations                   */
    uint64_t fp64_polish_iter;  /* FP64 refinement iterations                    */
    uint64_t rk_steps;          /* RKF45 attempts (6 evaluations of W each)      */
    uint64_t rk_rejected;       /* rejected attempts                             */
    uint64_t samples;           /* accepted steps (rho + transfer function)      */
    uint64_t w_evals;           /* evaluations of phi, J_phi and W               */
    uint64_t fp64_solves;       /* 3x3 solves done in FP64 (small det J)         */
    uint64_t rk_iter_cap;       /* segments stopped at the iteration cap         */
    uint64_t mlp_queries;       /* MLP seed evaluations                          */
    uint64_t subsamples;        /* supersampling sub-steps (transfer function)   */
    uint64_t degenerate;        /* segment ends with singular J (|det J| below
                                   det_singular), shrunk by Eq. (degeneracyfix) */
    uint64_t mlp_restarts;      /* shrunk entries whose Newton the network seeded */
    uint64_t drift_restarts;    /* samples put back on the ray by Newton (drift_tol) */
    uint64_t restart_fail;      /* of which Newton did not converge               */
    uint64_t dp_over;           /* interior samples with Delta P > 1 (views with
                                   dp_dev only)                                   */
    uint64_t order_violations;  /* samples out of depth order (same)             */
    double ms_fragments, ms_integrate, ms_merge;  /* event times per phase: the
                                   fragment launches with the block sort that
                                   follows them, the integrator launches, the
                                   merge                                       */
} ivr_stats;

/* Creates a context on `device` using `hip_stream` (a hipStream_t; NULL = the
 * null stream).  IVR_EDEVICE if the device is not a gfx950. */
ivr_status ivr_create(ivr_ctx **out, int32_t device, void *hip_stream);

/* Fills *o with the defaults listed at ivr_render_opts. */
void ivr_default_opts(ivr_render_opts *o);

/* Replaces the model with n >= 1 blocks (Sec. "Approach and Implementation":
 * knots and control points are all the method stores).  Validates every block
 * (degrees, counts, clamped non-decreasing knots, finite values, positive
 * weights) and returns IVR_EINVAL without touching the current model on
 * failure.  Packs FP32 and FP64 copies, bounding boxes of every block, face and
 * face element (convex hull of their control points), and uploads them.  A new
 * model invalidates a trained MLP. */
ivr_status ivr_upload_patches(ivr_ctx *ctx, const ivr_patch_desc *patches, int32_t n);

/* Uploads several models into one context (replacing the current ones): model m
 * is the model_sizes[m] consecutive blocks that follow model m-1's in patches[].
 * Views of a batch name the model they look at; blocks of different models never
 * see each other (faces shared between blocks are only matched within a model).
 * ivr_upload_patches(ctx, p, n) is ivr_upload_models with one model of n blocks.
 * At most 2^20-1 blocks in all.  Same validation and failure behaviour as
 * ivr_upload_patches. */
ivr_status ivr_upload_models(ivr_ctx *ctx, const ivr_patch_desc *patches, int32_t n,
                             const int32_t *model_sizes, int32_t n_models);

/* Renders one view.  rgba_dev: width*height*4 floats (premultiplied RGBA over
 * transparent black, row-major, row 0 at the top); depth_dev: width*height
 * floats (ray parameter of the first entry, +inf where the ray misses) or NULL.
 * opts NULL = defaults.  Returns after enqueueing the work unless stats != NULL.
 * IVR_ESTATE before a model is uploaded or when opts->seed_mode is MLP and no
 * MLP has been trained. */
ivr_status ivr_render(ivr_ctx *ctx, const ivr_camera *cam, const ivr_transfer_fn *tf,
                      const ivr_render_opts *opts, float *rgba_dev, float *depth_dev,
                      ivr_stats *stats);

/* ivr_render for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same image, but every frame buffer (segments, candidate
 * list, block order, per-segment results, counters, the view record) is carved
 * out of one fixed 256 MiB device array per GPU, set up by ivr_create and held
 * until the process ends.  The call allocates nothing, host or device (a
 * non-NULL stats uses the context's pinned staging and events).
 *   - At most 1048576 pixels per call and 65536 blocks in the model, else
 *     IVR_EOVERFLOW with nothing launched; opts->timing must be 0 (IVR_EINVAL).
 *   - Segment slots are what the array holds after the fixed parts (about 2.3
 *     per pixel at 1024x1024, more for smaller views): segments beyond them are
 *     dropped and counted in stats->segment_overflow.  Candidate-list capacity
 *     is capped likewise (rays past it are traversed again; same image).
 *   - Every call on one GPU, from any context, uses that GPU's one array: calls
 *     whose work overlaps on the device (different streams, no ordering) race
 *     and must be serialised by the caller.  Calls on one stream are ordered.
 * Arguments, outputs and errors otherwise as ivr_render. */
ivr_status ivr_render_noalloc(ivr_ctx *ctx, const ivr_camera *cam, const ivr_transfer_fn *tf,
                              const ivr_render_opts *opts, float *rgba_dev, float *depth_dev,
                              ivr_stats *stats);

/* One view of a batch: camera, transfer function (NULL: the batch's), the model
 * it looks at (index into the models of the last upload) and its caller-owned
 * device outputs, laid out as for ivr_render, plus optional per-pixel flags
 * (width*height uint32 IVR_FLAG_* bits, or NULL) and an optional per-pixel
 * pixel-accuracy record (Definition "Pixel-Accurate Approximation of
 * Geometry"): dp_dev, width*height floats, receives the largest
 * Delta P = 2 |pi_s(phi(p_i)) - pixel centre|_inf (Eq. (deltaP), in pixels) over
 * the interior samples p_i of the pixel's segments (0 where there are none),
 * and the flags receive IVR_FLAG_DEPTH_ORDER where a sample's projection onto
 * the ray lies before its predecessor's (the entry and exit included).  A batch
 * with any dp_dev runs an instrumented integrator (scalar field, ODE or RF
 * interior method; IVR_EINVAL otherwise). */
typedef struct {
    ivr_camera cam;
    const ivr_transfer_fn *tf;
    int32_t model;
    float *rgba_dev;
    float *depth_dev;
    uint32_t *flags_dev;
    float *dp_dev;
} ivr_view;

/* Renders 1..64 views of possibly different sizes and models with the same
 * options in one pass of the hot path: one fragment launch over the tiles of all
 * views, one persistent integrator launch per degree class over all their
 * segments (a lane's segment may come from any view) and one merge.  Without
 * stats and timing the launches are captured once per batch shape (view sizes
 * and models, options, launch shapes) in a HIP graph and replayed; the cameras,
 * transfer functions and output pointers travel in a device view table written
 * before each replay, so a replay may change them.  With stats (or
 * opts->timing) the kernels are launched directly and the counters and phase
 * times cover the whole batch.  IVR_EINVAL for an empty or oversized batch, a
 * missing rgba buffer or transfer function, or an unknown model. */
ivr_status ivr_render_batch(ivr_ctx *ctx, const ivr_view *views, int32_t n_views,
                            const ivr_transfer_fn *tf, const ivr_render_opts *opts, ivr_stats *stats);

/* Launch shapes picked by ivr_autotune. */
typedef struct {
    int32_t tile_w, tile_h;     /* fragment-kernel tile (one 64-lane wave)            */
    int32_t xcd_chunk;          /* > 0: runs of this many consecutive tiles per XCD   */
    int32_t int_block;          /* integrator workgroup size                          */
    int32_t int_waves_cu;       /* integrator waves per CU (0: as many as fit)        */
    int32_t n_tried;
    double tried_ms[32];        /* phase time of every shape tried, in order           */
    double ms_before, ms_after; /* fragment + integrator time before and after         */
} ivr_tune_report;

/* Times the batch (three runs per shape, best kept) under every fragment tile
 * shape (8x8, 16x4, 32x2) and XCD chunk (0, 4, 16), then every integrator workgroup size
 * (64, 128, 256) and residency (all that fit, 16 or 8 waves per CU), keeps the
 * fastest of each for this context (ivr_render and ivr_render_batch use them)
 * and drops captured graphs.  Writes the views' outputs as a side effect. */
ivr_status ivr_autotune(ivr_ctx *ctx, const ivr_view *views, int32_t n_views, const ivr_transfer_fn *tf,
                        const ivr_render_opts *opts, ivr_tune_report *report);

/* Sets the launch shapes by hand (tile_w 8, 16 or 32; xcd_chunk 0..4096; int_block
 * 64, 128 or 256; int_waves_cu 0..64).  Results do not depend on them. */
ivr_status ivr_set_launch(ivr_ctx *ctx, int32_t tile_w, int32_t xcd_chunk, int32_t int_block,
                          int32_t int_waves_cu);

/* ---- learned initialiser: one 3 -> 64 -> 64 -> 3 tanh MLP per block that maps a
 * world point (normalised by the block's box to [-1,1]^3) to its parameter point;
 * a surrogate of F^-1 used to seed the Newton solves of the boundary roots
 * (seed_mode IVR_SEED_MLP).  Trained on the GPU on (F(p), p) pairs generated by
 * the forward map with BF16 MFMA forward/backward kernels and Adam (FP32 master
 * weights). */
typedef struct {
    int32_t samples_per_patch;  /* forward-map samples per block          [65536] */
    int32_t steps;              /* Adam steps                              [2000] */
    double lr;                  /* Adam step size                          [1e-3] */
    uint32_t seed;              /* sample and initialisation seed          [5005] */
    int32_t log_every;          /* record the loss every this many steps    [100] */
    int32_t batch;              /* minibatch rows per block and step: a
                                   multiple of 16 in 16..128              [128] */
} ivr_mlp_opts;

typedef struct {
    int32_t n_loss;             /* entries of loss[] written                     */
    float loss[64];             /* minibatch loss (mean over blocks) at steps
                                   0, log_every, 2*log_every, ...                 */
    double heldout_mean_err;    /* mean and max over 4096 held-out samples per   */
    double heldout_max_err;     /* block of max_c |MLP(F(p))_c - p_c|            */
    double ms_samples, ms_train;
} ivr_mlp_report;

void ivr_default_mlp_opts(ivr_mlp_opts *o);

/* Trains one MLP per uploaded block (IVR_ESTATE before an upload).  report may be
 * NULL; when given, the call waits for the training to finish. */
ivr_status ivr_train_inverse_mlp(ivr_ctx *ctx, const ivr_mlp_opts *opts, ivr_mlp_report *report);

/* Gradient check of the training kernels: one forward/backward pass of the
 * device code on n rows (a multiple of 16 in 16..128, the minibatch sizes the
 * training takes) with the given parameters (kMlpParams = 4611 floats
 * in the layout W1[3][64] b1[64] W2[64][64] b2[64] W3[64][3] b3[3]), normalised
 * inputs x (n*3) and targets p (n*3), all host arrays.  Writes the loss
 * (mean over rows of |y - p|^2) and the 4611 gradient entries.  Synchronous. */
ivr_status ivr_mlp_forward_backward(ivr_ctx *ctx, const float *params, const float *x, const float *p,
                                    int32_t n, float *loss, float *grad);

/* Copies block `patch`'s FP32 master weights (4611 floats) to host memory. */
ivr_status ivr_mlp_get_weights(ivr_ctx *ctx, int32_t patch, float *out);

/* p_out[3i..] = MLP_{patch[i]}(x[3i..]) for n world points (host arrays). */
ivr_status ivr_mlp_infer(ivr_ctx *ctx, const int32_t *patch, const float *x, int32_t n, float *p_out);

/* Phase times of the renders recorded with opts->timing = 1 since the last call:
 * waits for them, writes up to `cap` triples (fragments, integrate, merge) in
 * milliseconds to ms_out (3*cap doubles), the number of renders to *n_out, and
 * forgets them.  At most 4096 renders are kept (IVR_EOVERFLOW past that). */
ivr_status ivr_phase_times(ivr_ctx *ctx, double *ms_out, int32_t cap, int32_t *n_out);

/* Summary of an image comparison. */
typedef struct {
    double max;                 /* largest per-pixel difference                  */
    double mean;                /* mean over the pixels                          */
    uint64_t over;              /* pixels whose difference exceeds the threshold */
} ivr_delta_e_summary;

/* Image quality as the paper measures it: the CIE's year-2000 colour difference
 * (CIEDE2000, CIE 142-2001; 1 is a just noticeable difference, the paper
 * accepts up to 5) between two premultiplied RGBA device images of n_pixels
 * (4 floats each, as ivr_render writes them), each composited over the
 * background colour (3 values in [0,1]; NULL: white) and read as sRGB
 * (IEC 61966-2-1) with the D65 white, in FP64 on the device.  de_dev (device,
 * n_pixels floats, or NULL) receives the per-pixel difference; *summary (host,
 * or NULL) the largest, the mean and the count above `threshold`, which waits
 * for the stream.  IVR_EINVAL for a NULL image or n_pixels < 0. */
ivr_status ivr_delta_e2000(ivr_ctx *ctx, const float *rgba_a_dev, const float *rgba_b_dev, int64_t n_pixels,
                           const double *background, double threshold, float *de_dev,
                           ivr_delta_e_summary *summary);

/* Device memory the context holds: the uploaded model (control nets, boxes,
 * basis tables) and the frame buffers, which are sized from counts (segment
 * slots at 2.5 per pixel or 1.2 times the most per pixel a render needed,
 * candidate entries at 2 per pixel or 1.25 times the most needed) and grow but never shrink.  Either pointer may
 * be NULL. */
ivr_status ivr_device_bytes(ivr_ctx *ctx, uint64_t *model_bytes, uint64_t *frame_bytes);

/* Message for the last failing call of this context ("" if none). */
const char *ivr_last_error(const ivr_ctx *ctx);

/* Frees every device allocation of the context (waits for its stream). */
void ivr_destroy(ivr_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
