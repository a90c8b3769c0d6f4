// Data layout shared by the host library and the gfx950 kernels.
//
// Model (uploaded once, read-only while rendering):
//   DevPatch[npatch]      per-block metadata and bounding boxes (one 16-B aligned record)
//   cp32 / cp64           control points, float4 / double4 per point: (x,y,z,rho) for
//                         B-splines (the scalar coefficient rides in the fourth lane),
//                         homogeneous (wx,wy,wz,w) for NURBS; i fastest
//   rho32 / rho64         scalar coefficients (w*rho for NURBS), same order
//   knots32 / knots64     knot vectors normalised to [0,1] (only read for
//                         non-uniform directions)
//   FaceElem[nelem]       one record per non-empty knot span of every boundary face
// Frame buffers (grow-only, owned by the context):
//   Seg[cap]              entry/exit pairs written by the fragment kernel
//   queue[class][cap]     segment indices per degree class, consumed by the integrator
//   results[cap]          premultiplied (C, alpha) per segment
//   pixseg[pixels]        (first segment, count) per pixel, segments sorted by entry depth
#pragma once
#include <stdint.h>

namespace ivr {

constexpr int kMaxDegree = 3;
constexpr int kMaxTfKnots = 16;
constexpr int kClasses = 6;          // degree class = 2*(degree-1) + rational
constexpr int kFragCap = 64;         // boundary crossings kept per ray (hard cap)
constexpr int kSegCap = 32;          // segments kept per pixel
constexpr int kCandCap = 64;         // face elements whose box a ray hits (Newton seeds)

struct alignas(16) DevPatch {
    int32_t deg;           // isotropic degree 1..3
    int32_t n[3];          // control points per direction
    int32_t nspan[3];      // n - deg (number of spans when uniform)
    int32_t uniform;       // bit d: open-uniform knots in direction d
    int32_t rational;      // 1: NURBS
    int32_t cp_off;        // index of the first control point
    int32_t knot_off[3];   // offset of each knot vector in the knot arrays
    int32_t elem_off[7];   // face f owns elements [elem_off[f], elem_off[f+1])
    int32_t tile_off[7];   // face f owns tiles [tile_off[f], tile_off[f+1])
    int32_t klass;         // degree class
    float orient;          // sign of det J over the block (+1 / -1)
    float box[6];          // padded bounding box lo[3], hi[3]
    float fbox[6][6];      // padded bounding box of each face
    float inv_nspan[3];
    float pad0;
    int32_t twin[6];       // face shared with another block: 8*block + face, or -1
    int32_t face_skip;     // bit f: face f is the twin of a face tested from the other block
    int32_t btab_off;      // first float of the block's basis tables (see Model::btab)
    int32_t btab_len;      // floats of the block's basis tables
    int32_t pad2[3];
};

// Face element: oriented box around the element's control points (axes from the
// net's edge directions; the element lies in the convex hull of its points).
struct alignas(16) FaceElem {
    float c[3];            // box centre
    float ax[3][3];        // orthonormal axes (rows)
    float ext[3];          // padded half extents along the axes
    float a0, a1, b0, b1;  // parameter rectangle in the face's (a, b) directions
    int32_t face;
    int32_t patch;
    float graze;           // bound on the slope of the element against its box plane
    int32_t pad;
};

// Up to kTile x kTile neighbouring elements of one face, with an oriented box
// around all their Bezier points; its elements are contiguous.  A tile of more
// than 2 x 2 elements is split into sub-tiles of up to 2 x 2 (records of the
// same kind, [sub_begin, sub_end) of the tile array, their elements contiguous
// in the tile's order); otherwise sub_begin == sub_end.
constexpr int kTile = 4;
struct alignas(16) FaceTile {
    float c[3];
    float ax[3][3];
    float ext[3];
    int32_t elem_begin, elem_end;
    int32_t sub_begin, sub_end;
    int32_t pad;
};

template <typename R>
struct Seg {
    R t_in, t_out;         // ray parameters of entry and exit
    R p_in[3], p_out[3];   // parameter points of entry and exit
    R rho_out;             // rho at the exit
    R drho_out;            // d rho / ds at the exit (along the ray)
    uint32_t pixel;        // linear pixel index
    uint32_t patch;
};

struct Model {
    const DevPatch *patches;
    const float4 *cp32;
    const float *rho32;
    const double4 *cp64;
    const double *rho64;
    const float *knots32;
    const double *knots64;
    const FaceElem *elems;
    const FaceTile *tiles;
    // Per block, direction d (0..2) and knot span e: the deg+1 non-zero basis
    // functions on the span as polynomials in the local coordinate x in [0,1],
    // (deg+1)^2 coefficients (function i, power k at [i*(deg+1)+k]); directions
    // follow each other, spans in order.
    const float *btab;
    const uint16_t *mlp_wb;    // BF16 MLP weights per block (seed_mode MLP)
    // displacement spline u per control point as (w u, w) (w = 1 for B-splines),
    // same order as cp32 / cp64; null when the model has none
    const float4 *disp32;
    const double4 *disp64;
    const float *mlp_norm;     // per block: (unused[3], 1/half extent[3], centre[3], pad[3])
    int32_t npatch;
    float scale;           // bounding-box diagonal of the model
    double scaled;
};

// Summary of an image comparison (ivr_delta_e2000), accumulated on the device.
struct DeltaESum {
    double sum;
    unsigned long long over;
    unsigned int max_bits;   // float bits of the largest difference (non-negative)
    unsigned int pad;
};

// Device-side counters, one 64-bit slot each (ivr_stats order).
enum Counter : int {
    C_RAYS = 0, C_SEGMENTS, C_FRAGMENTS, C_ANOMALIES, C_FRAG_OVF, C_SEG_OVF, C_BOX_TESTS,
    C_FACE_NEWTON, C_FACE_NEWTON_ITER, C_FP64_POLISH, C_RK_STEPS, C_RK_REJECTED, C_SAMPLES,
    C_W_EVALS, C_FP64_SOLVES, C_RK_ITER_CAP, C_MLP_QUERIES, C_SUBSAMPLES, C_DEGENERATE,
    C_MLP_RESTARTS, C_DRIFT_RESTARTS, C_RESTART_FAIL, C_DP_OVER, C_ORDER_BAD, C_COUNT
};

// Bookkeeping written by the fragment kernel.
struct QueueState {
    uint32_t seg_total;             // segments requested (may exceed the capacity)
    uint32_t n_cands;               // candidates recorded
    uint32_t pad[6];
};

// Buffers of the two-pass fragment kernel: every wave's candidates block after
// block (element | owning lane << kCandLaneShift, seed index or ~0), per lane
// the positions of its own candidates in that list, and per lane the wave's
// base and its count.  With MLP seeds, a candidate's network query (world
// point, block) and seed sit at its position in the list.
constexpr int kCandLaneShift = 26;
constexpr uint32_t kCandElemMask = (1u << kCandLaneShift) - 1;
struct CandLists {
    float4 *query;            // x, y, z, block (as int bits)
    float4 *seed;
    uint2 *clist;
    uint32_t *plist;
    uint2 *crange;            // per lane of a fragment tile (tile * 64 + lane)
    uint32_t c_cap;
};

// What the integrator of one degree class needs to take its segments block by
// block: the block-sorted segment order, the blocks of the class as positions
// [q_begin, q_end) of pperm (blocks grouped by class), per-block base, count and
// cursor into the order, and the largest control net of the class (LDS size).
struct IntegrateArgs {
    const uint32_t *order;
    const uint32_t *pperm;
    int32_t q_begin, q_end;
    const uint32_t *pbase, *pcount;
    uint32_t *pcur;
    int32_t max_cp;
    int32_t max_tab;
};

struct FrameParams {
    // camera (FP64 and FP32 copies of the same basis)
    double eye[3], fwd[3], right[3], up[3];
    double tan_half, aspect;
    float eyef[3], fwdf[3], rightf[3], upf[3];
    float tan_halff, aspectf;
    int32_t width, height;
    // transfer function: knots x[k] and per-interval value/slope
    int32_t tf_n;
    int32_t tf_nint_max;            // most interior knots of any view of the batch
    float tf_x[kMaxTfKnots];
    float tf_v[kMaxTfKnots][4];     // value at knot k (RGB, kappa = extinction*A)
    float tf_s[kMaxTfKnots][4];     // slope on [x_k, x_{k+1}]
    float tf_lo, tf_inv_range;
    float tf_dn;                    // target change of n per supersampling sub-step
    float tf_smax[kMaxTfKnots];     // largest |slope| over channels on intervals k-1..k+1
    float tf_step;                  // largest change of the transfer function per sub-step
    float rho_step;                 // largest change of n (normalised rho) per step
    double tf_xd[kMaxTfKnots];
    double tf_vd[kMaxTfKnots][4];
    double tf_sd[kMaxTfKnots][4];
    double tf_lod, tf_inv_ranged;
    // integrator
    float rk_tol, h_max, h_min, c_perp, early_term, det_thr, det_sing, drift_tol;
    double rk_told, h_maxd, h_mind, c_perpd, early_termd, det_thrd, det_singd, drift_told;
    int32_t n_super, max_frag, max_newton, collect, hermite, seed_mode;
    int32_t interior;               // IVR_INTERIOR_*
    int32_t field;                  // IVR_FIELD_*
    int32_t newton_stop;            // IVR_NEWTON_STOP_*
    // Sec. "Cutting and Near Clip Planes": cutting plane (cut != 0) keeping
    // cut_n . (g - g0) >= 0, with cut_s0 = cut_n . (eye - g0) for this view; near
    // plane near_clip in front of the eye along fwd (0: none)
    int32_t cut;
    double cut_n[3], cut_s0, near_clip;
    float scale;
    double scaled;
};


// One view of a batch (device array).  Views may look at different models (patch
// ranges), have their own camera and transfer function; the integrator options
// of the batch are the same in every record.
constexpr int kViewShift = 20;          // Seg::patch = block | view << kViewShift
constexpr uint32_t kPatchMask = (1u << kViewShift) - 1;
constexpr int kMaxViews = 1 << (32 - kViewShift);

struct alignas(16) ViewRec {
    FrameParams fp;
    int32_t patch_begin, patch_end;     // the view's model
    uint32_t tile_begin;                // first fragment-kernel tile of the view
    uint32_t tiles_x;                   // tiles per image row
    uint32_t pix_begin;                 // first pixel of the view in the batch
    uint32_t pad;
    float *rgba;                        // width*height*4, caller-owned
    float *depth;                       // width*height or null
    uint32_t *flags;                    // width*height IVR_FLAG_* bits or null
    float *dp;                          // width*height largest Delta P, or null
    void *pad2;
};

// What the integrator keeps per view in LDS: on interval k (x[k] <= n < x[k+1])
// channel c of the transfer function is a[k].c + b[k].c * n; x[m] = +inf past the
// last interior knot; smax[k] bounds the slope on intervals k-1..k+1.
struct alignas(16) ViewLds {
    float4 a[kMaxTfKnots], b[kMaxTfKnots];
    float x[kMaxTfKnots], smax[kMaxTfKnots];
    float lo, inv_range, dn, h_max, h_min, scale;
    double inv_ranged;
};

// Launch shapes chosen by the autotuner.
struct LaunchCfg {
    int32_t tile_w;          // fragment tile width in pixels (tile_w * tile_h = 64)
    int32_t xcd_chunk;       // > 0: runs of this many consecutive tiles per XCD
    int32_t int_block;       // integrator workgroup size (64, 128 or 256)
    int32_t int_waves_cu;    // integrator waves per CU (0: as many as fit)
};

}  // namespace ivr
