/*
 * hyrf.h -- C ABI of the HyRF differentiable render step on AMD MI355X (gfx950).
 *
 * The method (Wang & Xu, "HyRF: Hybrid Radiance Fields for Memory-efficient
 * and High-quality Novel View Synthesis"): explicit compact Gaussians are
 * pre-culled against the camera (Sec. 3.3, Eqs. 8-9), their positions are
 * contracted into (0,1)^3 (Sec. 3.2 Eq. 2, App. A.1) and looked up in two
 * multi-resolution hash grids (Eq. 3) whose features two tiny MLPs decode
 * into opacity / scale / rotation and view-dependent colour (Eqs. 4-6); the
 * result is aggregated with the explicit parameters (Eq. 7), splatted with
 * the 3DGS rasterizer -- EWA projection, depth-ordered tile binning,
 * front-to-back alpha blending (Sec. 3.1, Eq. 1) -- and blended with a
 * background colour that the radiance field predicts where each pixel's ray
 * meets a sphere of radius r (Sec. 3.3 Eqs. 10-11, App. A.2).
 *
 * Conventions shared by every call
 *  - Every pointer named in a descriptor or argument is DEVICE memory owned by
 *    the caller, except the descriptor structs themselves, which are read on
 *    the host during the call and may be freed when it returns.  The library
 *    never allocates or frees device memory and keeps no state between calls
 *    (apart from a thread-local error string).
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t passed as
 *    void*; NULL = the default stream).  Inputs must stay valid, and outputs
 *    must not be read, until the stream has reached the work.
 *  - Arrays are float32 and planar (structure of arrays) unless stated.
 *    "n" is the Gaussian count, "V" the number of views, "L" the number of
 *    grid levels.  All views of one call share width and height.
 *  - Every argument is validated on the host before anything is enqueued;
 *    on failure nothing is launched or written, the call returns a non-zero
 *    hyrf_status and hyrf_last_error() describes the problem.  Device-side
 *    faults surface at the caller's next synchronisation.  NaN/Inf inputs
 *    propagate; they are not checked.
 */
#ifndef HYRF_H
#define HYRF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYRF_TILE 16          /* screen tiles are 16 x 16 pixels */
#define HYRF_MAX_VIEWS 8
#define HYRF_PE_OCTAVES 4     /* view-direction encoding: 4 octaves, sin and cos -> 24 inputs */
#define HYRF_GEO_OUT 8        /* geometry decoder: opacity, scale[3], rotation[4] */
#define HYRF_COL_OUT 3        /* colour decoder: rgb */

typedef enum {
  HYRF_OK = 0,
  HYRF_ERR_INVALID_ARGUMENT = 1,
  HYRF_ERR_UNSUPPORTED = 2,
  HYRF_ERR_CAPACITY = 3,
  HYRF_ERR_LAUNCH = 4
} hyrf_status;

typedef enum { HYRF_F32 = 0, HYRF_F16 = 1, HYRF_BF16 = 2, HYRF_U8 = 3 } hyrf_dtype;
/* RENDER: the background is added only where the final transmittance
 * exceeds tau_T (Sec. 3.3, last paragraph) and nothing is saved.
 * TRAIN: the background is added at every pixel and the state the backward
 * needs is saved. */
typedef enum { HYRF_RENDER = 0, HYRF_TRAIN = 1 } hyrf_mode;

/* Explicit compact Gaussians (Sec. 3.2, first paragraph). */
typedef struct {
  int32_t n;
  const void* pos;       /* [3][n] world position p_e: float32, or float16 when
                            pos_dtype = HYRF_F16 (see below)                       */
  const float* scale_e;  /* [3][n] scale logit s_e (paper: one value; pass equal axes) */
  const float* rot_e;    /* [4][n] rotation residual (w,x,y,z) or NULL (paper: none) */
  const float* opac_e;   /* [n]    opacity logit alpha_e                           */
  const float* col_e;    /* [3][n] colour logit c_e                                */
  /* HYRF_F32 (0, the default) or HYRF_F16: positions stored in half
   * precision, the compressed model's format (Sec. 4.3), widened to float32
   * (exactly) where the cull, the field query and the projection read them.
   * A render-only format: hyrf_render_backward and its stages reject it
   * (HYRF_ERR_UNSUPPORTED); hyrf_spatial_order takes float32 positions. */
  int32_t pos_dtype;
} hyrf_gaussians;

/* Two hash-grid fields and their decoders (Sec. 3.2, Eqs. 2-6; Sec. 4.1). */
typedef struct {
  int32_t levels;        /* L: 4, 8, 12 or 16                                       */
  int32_t features;      /* F: must be 2                                           */
  int32_t log2_T_geo;    /* geometry table rows per level, 2^log2_T_geo (10..24)    */
  int32_t log2_T_rad;    /* radiance table rows per level (10..24)                  */
  float base_res;        /* N_min (>= 2); N_l = floor(N_min * growth^l)             */
  float growth;          /* b (>= 1)                                               */
  int32_t table_dtype;   /* HYRF_F32, HYRF_F16, or HYRF_U8 (8-bit min-max codes,
                            render only; see qparams_*)                            */
  const void* table_geo; /* [L][T_geo][2]                                          */
  const void* table_rad; /* [L][T_rad][2]                                          */
  int32_t hidden;        /* MLP width: 16, 32, 48 or 64                            */
  int32_t n_hidden;      /* hidden layers: 1 or 2 (ReLU, no bias)                  */
  int32_t mlp_dtype;     /* HYRF_F32, or HYRF_BF16 (bf16 operands, fp32 accumulate; the
                            weights are still passed as float32 and rounded on load) */
  const float* mlp_geo;  /* layers concatenated, each row-major [out][in]:
                            [hidden][2L], ([hidden][hidden]), [8][hidden]            */
  const float* mlp_col;  /* [hidden][2L+24], ([hidden][hidden]), [3][hidden]        */
  float aabb_center[3];  /* scene box: p' = (p - centre) * inv_half (App. A.1 Eq. 13) */
  float aabb_inv_half[3];
  float bg_radius;       /* background sphere radius r (Sec. 4.1: 100)              */
  float tau_T;           /* render-mode background threshold (Sec. 4.1: 0.2)        */
  /* HYRF_U8 tables only (else ignored, may be NULL): per level l, the pair
   * (min_l, step_l) of that level's 8-bit min-max quantisation; an entry
   * holding code q decodes to min_l + step_l * q (Sec. 4.3, compressed model).
   * Device, [L][2] float32 each. */
  const float* qparams_geo;
  const float* qparams_rad;
  /* Non-zero: the single-field (non-decoupled) model the paper compares
   * with (Sec. 4.4, decoupling ablation): ONE hash grid, the radiance table
   * (table_rad, log2_T_rad, qparams_rad), feeds both decoders; table_geo,
   * log2_T_geo and qparams_geo are ignored, and the whole table gradient goes
   * to hyrf_grads.table_rad (hyrf_grads.table_geo is ignored). */
  int32_t single_field;
  /* Adjoint only; no effect on any result beyond float rounding.  How the
   * background points' radiance-table scatter treats corners shared by
   * consecutive grid cells: 0 = automatic (merged into one cell before the
   * atomics: fewer atomic requests, for both decoder precisions),
   * 1 = always merged, 2 = never.
   * Other values: HYRF_ERR_INVALID_ARGUMENT. */
  int32_t scatter_merge;
} hyrf_fields;

/* Pinhole camera, world -> camera p_c = R p + t (Sec. 3.3 Eq. 8), OpenCV axes
 * (x right, y down, z forward); pixel (x, y) is sampled at (x+.5, y+.5). */
typedef struct {
  float R[9];            /* row-major */
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  float z_near;          /* pre-cull: drop Gaussians with depth <= z_near            */
  float cull_tol;        /* pre-cull tolerance band "tol" of Eq. 9                   */
} hyrf_camera;

/* Output of hyrf_query_fields: the union (over views) of pre-cull survivors,
 * compacted in ascending Gaussian index, with their aggregated properties.
 * Slot k (0 <= k < *vis_count) describes Gaussian vis_idx[k]. */
typedef struct {
  int32_t* vis_count;    /* [1]                                                     */
  int32_t* vis_idx;      /* [n]                                                     */
  float* opacity;        /* [n]       sigmoid(a_n + a_e)                             */
  float* scale;          /* [3][n]    sigmoid(s_n + s_e)                             */
  float* quat;           /* [4][n]    Normalize(r_n (+ r_e)), (w,x,y,z)               */
  float* rgb;            /* [V][3][n] sigmoid(c_n + c_e) per view                    */
  float* feat_geo;       /* [n][2L] encoded geometry features, or NULL (TRAIN needs it) */
  float* feat_rad;       /* [n][2L] encoded radiance features, or NULL (TRAIN needs it) */
  uint32_t* dbg_index;   /* optional [n][2][L][8] table rows (field 0 = geometry,
                            corner k = dx + 2 dy + 4 dz), or NULL                    */
  float* feat_jac;       /* optional (TRAIN) [n][L][12] spatial derivatives of the
                            encoded features with respect to the contracted
                            position x: per level, geometry field then radiance
                            field, feature 0 then 1, d/dx, d/dy, d/dz.  Kept for the
                            backward, which then need not gather the tables again
                            for dL/dp; NULL -> the backward gathers them.  Not
                            written for 8-bit tables (render-only).                */
} hyrf_query_out;

/* Per (view, slot) splat records written by hyrf_project and read by
 * hyrf_bin_sort / hyrf_composite / hyrf_render_backward. */
typedef struct {
  int32_t n_max;         /* slots per view (>= *count; normally n)                   */
  const int32_t* count;  /* [1] valid slots (normally hyrf_query_out.vis_count)       */
  float* rec;            /* [V][n_max][12]: u, v, conic a, b, c, opacity, r, g, b,
                            depth, 0, 0  (float4-aligned; 16-byte aligned pointer)    */
  int32_t* rect;         /* [V][n_max][4]: tile rectangle x0, y0, x1, y1 (x1, y1
                            exclusive); empty when the splat is culled in this view,
                            degenerate, or cannot reach alpha 1/255 anywhere           */
  float* depth;          /* [V][n_max] camera depth rounded to float32 (> 0): ordering key */
  int64_t* total;        /* [1] sum of rectangle areas = tile entries (written by
                            hyrf_project)                                           */
} hyrf_splats;

/* Gradient accumulators (+=) -- all float32, caller-zeroed, same layouts as
 * the corresponding inputs.  Any pointer may be NULL to skip that output. */
typedef struct {
  float* pos;            /* [3][n] */
  float* scale_e;        /* [3][n] */
  float* rot_e;          /* [4][n] (ignored when hyrf_gaussians.rot_e is NULL) */
  float* opac_e;         /* [n]    */
  float* col_e;          /* [3][n] */
  float* table_geo;      /* [L][T_geo][2] float32 even for float16 tables */
  float* table_rad;      /* [L][T_rad][2] */
  float* mlp_geo;        /* same layout as hyrf_fields.mlp_geo */
  float* mlp_col;        /* same layout as hyrf_fields.mlp_col */
  /* Densification statistics (Sec. 3.1: Gaussians are densified from
   * accumulated gradients, as in 3DGS), nullable, [n] each, accumulated (+=)
   * over calls: for every view in which a Gaussian's footprint touches a tile,
   * dens_accum += |(W/2 dL/du, H/2 dL/dv)| (the gradient with respect to its
   * projected centre in normalised device coordinates) and dens_count += 1. */
  float* dens_accum;
  float* dens_count;
} hyrf_grads;

/* Forward state of a TRAIN-mode render that hyrf_render_backward reads. */
typedef struct {
  const hyrf_query_out* query;   /* with feat_geo / feat_rad filled              */
  const hyrf_splats* splats;
  const uint32_t* vals;          /* sorted splat ids from hyrf_bin_sort            */
  const uint32_t* tile_ranges;   /* [V*tiles][2]                                  */
  const float* T_final;          /* [V][H][W] from hyrf_composite                 */
  const int32_t* last;           /* [V][H][W] from hyrf_composite                 */
  const float* bg_rgb;           /* [V][3][H][W] background colours c_s           */
  const float* bg_feat;          /* [V*H*W][2L] radiance features of the sphere
                                    points from hyrf_composite, or NULL (the
                                    backward then gathers them again)           */
} hyrf_fwd_state;

/* ---- the render step ------------------------------------------------------ */

/* Pre-cull, field query, decoding and aggregation (Sec. 3.3 Eqs. 8-9, then
 * Sec. 3.2 Eqs. 2-7).  A Gaussian survives if, in at least one of the V
 * views, its camera depth exceeds z_near and its projected centre lies in the
 * image frame widened by cull_tol on every side (normalised coordinates).
 * The survivors are queried once in both fields; the colour decoder runs once
 * per view with that view's direction encoding.  ws: workspace of at least
 * hyrf_query_workspace_bytes(n) bytes (16-byte aligned). */
hyrf_status hyrf_query_fields(const hyrf_fields* fields, const hyrf_gaussians* g,
                              const hyrf_camera* cams, int32_t n_views,
                              const hyrf_query_out* out, void* ws, size_t ws_bytes,
                              void* stream);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation:
 * hyrf_query_fields with its scratch (cull flags, their exclusive scan, the
 * scan's partials) taken from a device array the library holds, instead of a
 * caller workspace.  Outputs are those of hyrf_query_fields, bit for bit.
 *  - n must be <= HYRF_QUERY_NOALLOC_MAX_GAUSSIANS; a larger n returns
 *    HYRF_ERR_CAPACITY with nothing launched.
 *  - The array, hyrf_query_noalloc_scratch_bytes() bytes (about 32 MiB), is
 *    held by every GPU the library runs on until the process ends.  The first
 *    call on a device looks up its address there once (the calling thread's
 *    current device must be the device of `stream`); no call allocates or
 *    frees memory.
 *  - Every call on one GPU uses that GPU's one array: calls that overlap on
 *    one GPU (two streams, two threads) race and must be serialised by the
 *    caller.  Nothing in it needs clearing between calls. */
#define HYRF_QUERY_NOALLOC_MAX_GAUSSIANS (1 << 22)
size_t hyrf_query_noalloc_scratch_bytes(void);
hyrf_status hyrf_query_fields_noalloc(const hyrf_fields* fields, const hyrf_gaussians* g,
                                      const hyrf_camera* cams, int32_t n_views,
                                      const hyrf_query_out* out, void* stream);

/* EWA projection of every surviving Gaussian into every view (3DGS
 * rasterizer, Sec. 3.1): 2D covariance J W Sigma W^T J^T + 0.3 I, conic,
 * centre, float32 depth key, and a conservative tile rectangle holding every
 * pixel where alpha >= 1/255 can hold.  Also writes splats->total. */
hyrf_status hyrf_project(const hyrf_gaussians* g, const hyrf_query_out* q,
                         const hyrf_camera* cams, int32_t n_views,
                         const hyrf_splats* splats, void* stream);

/* Tile binning and depth ordering (Sec. 3.1, "ordered by depth"): every
 * splat is listed once for each tile its rectangle covers, ordered by
 * (view, tile, float32 depth, slot).  vals[e] = view * n_max + slot of entry
 * e; keys[e] = view * tiles + tile (keys may be NULL); tile_ranges[2k],
 * [2k+1] = first / one-past-last entry of tile k = view*tiles + ty*tiles_x + tx.
 * capacity = length of keys / vals; returns HYRF_ERR_CAPACITY (nothing
 * launched) when n_entries > capacity, where n_entries is the caller's copy
 * of *splats->total (the one host read of the step). */
hyrf_status hyrf_bin_sort(const hyrf_splats* splats, const hyrf_camera* cams,
                          int32_t n_views, int64_t n_entries, int64_t capacity,
                          uint32_t* keys, uint32_t* vals, uint32_t* tile_ranges,
                          void* ws, size_t ws_bytes, void* stream);

/* Front-to-back alpha blending per 16x16 tile (Eq. 1 with the 3DGS rules:
 * alpha = min(0.99, o exp(-d^T conic d / 2)), skipped below 1/255, stop before
 * the transmittance falls below 1e-4), then the background
 * C = C_fg + T_final * c_s with c_s = sigmoid(colour decoder(Theta_rad at the
 * ray / sphere intersection, PE(ray direction))) (Sec. 3.3 Eqs. 10-11).
 * out_rgb [V][3][H][W]; out_T [V][H][W]; in TRAIN mode out_last [V][H][W]
 * (entries consumed up to the last contributor) and out_bg [V][3][H][W] are
 * required, in RENDER mode they may be NULL.  out_bg_feat (TRAIN mode,
 * nullable): [V*H*W][2L] float32 radiance features of every sphere point,
 * kept for the backward (hyrf_fwd_state.bg_feat) so that it need not gather
 * them again.  ws: at least
 * hyrf_composite_workspace_bytes(V, W, H) bytes. */
hyrf_status hyrf_composite(const hyrf_splats* splats, const uint32_t* vals,
                           const uint32_t* tile_ranges, const hyrf_camera* cams,
                           int32_t n_views, const hyrf_fields* fields, int32_t mode,
                           float* out_rgb, float* out_T, int32_t* out_last, float* out_bg,
                           float* out_bg_feat, void* ws, size_t ws_bytes, void* stream);

/* The train-mode background on its own (Sec. 3.3 Eqs. 10-11): c_s of every
 * pixel of every view, out_bg [V][3][H][W], and (nullable) the sphere points'
 * radiance features out_bg_feat [V*H*W][2L] kept for the backward.  It
 * depends on the cameras and fields only, so a caller may run it on a second
 * stream while the Gaussians are queried, projected, sorted and blended
 * (hyrf_composite with fields = NULL), then add it with
 * hyrf_blend_background.  The result equals hyrf_composite with fields in
 * TRAIN mode. */
hyrf_status hyrf_background(const hyrf_fields* fields, const hyrf_camera* cams, int32_t n_views, float* out_bg,
                            float* out_bg_feat, void* stream);

/* rgb[v][c][p] += T[v][p] * bg[v][c][p] over [V][3][H][W] (Eq. 10: the
 * background seen through the final transmittance). */
hyrf_status hyrf_blend_background(const float* bg, const float* T, float* rgb, int32_t n_views, int32_t width,
                                  int32_t height, void* stream);

/* Adjoint of the whole step: given dL/dC [V][3][H][W], accumulates (+=) the
 * gradients of every explicit parameter, both hash tables (background uses
 * included) and both decoders' weights.  Predicates (pre-cull, alpha
 * threshold, early stop, tau_T) and grid-cell choices are held fixed; the
 * 0.99 alpha clamp passes no gradient where it is active.  ws: at least
 * hyrf_backward_workspace_bytes(...) bytes. */
hyrf_status hyrf_render_backward(const hyrf_fields* fields, const hyrf_gaussians* g,
                                 const hyrf_camera* cams, int32_t n_views,
                                 const hyrf_fwd_state* saved, const float* dL_drgb,
                                 const hyrf_grads* grads, void* ws, size_t ws_bytes,
                                 void* stream);

/* The same adjoint split into seven stages, for callers that overlap or time
 * them.  Every stage takes the same arguments and workspace; each reads what
 * the stages it depends on left in the workspace (stage numbers are stable;
 * stage 5 is empty since stage 4 scatters its table gradients itself):
 *   0  decoder weights permuted into the operand order of the adjoint
 *   1  blending and projection adjoints (explicit-parameter gradients,
 *      densification statistics)
 *   2  decoder adjoints of the Gaussians; dL/dp through the view direction
 *      and, with saved feature derivatives, through the interpolation
 *      weights                                                    (after 0, 1)
 *   3  hash-table adjoint of the Gaussians                         (after 2)
 *   4  colour-decoder and radiance-table adjoints of the background
 *      points                                                     (after 0)
 *   5  launches nothing                                            (after 4)
 *   6  decoder weight gradients from the partials of 2 and 4   (after 2, 4)
 * The Gaussian branch (1, 2, 3) and the background branch (4, 5) touch
 * disjoint workspace regions and meet only in atomic additions to the
 * radiance-table gradient, so they may run concurrently on two streams (the
 * caller orders them with events).  hyrf_render_backward == stages 0..6 on
 * one stream. */
hyrf_status hyrf_render_backward_stage(int32_t stage, const hyrf_fields* fields, const hyrf_gaussians* g,
                                       const hyrf_camera* cams, int32_t n_views,
                                       const hyrf_fwd_state* saved, const float* dL_drgb,
                                       const hyrf_grads* grads, void* ws, size_t ws_bytes, void* stream);

/* L1 photometric term of the training loss (Sec. 3.4 Eq. 12, lambda = 0):
 * loss[0] = mean |img - target| over n values, grad[i] = sign(img - target)/n
 * (sign(0) = 0).  loss and grad are device pointers; grad may be NULL. */
hyrf_status hyrf_l1_loss(const float* img, const float* target, int64_t n,
                         float* loss, float* grad, void* ws, size_t ws_bytes, void* stream);

/* Training loss of Sec. 3.4 Eq. 12 with both terms:
 *   loss = (1 - lambda) * mean|img - target| + lambda * (1 - mean SSIM(img, target)),
 * forward and gradient fused in one pass.  SSIM follows Wang et al. 2004
 * with the settings 3DGS trains with (the paper adopts its loss): 11 x 11
 * Gaussian window of standard deviation 1.5, C1 = 0.01^2, C2 = 0.03^2
 * (dynamic range 1), statistics per plane with the image extended by zeros
 * outside its frame; the mean runs over every pixel of every plane.
 * img, target: device [planes][height][width] fp32 (planes = views x 3
 * colour channels).  loss: device float[3] <- (loss, mean L1, mean SSIM).
 * grad (device, nullable): [planes][height][width] <- dloss/dimg
 * (overwritten; sign(0) = 0 in the L1 term).  lambda in [0, 1] (3DGS: 0.2).
 * Deterministic.  Invalid arguments (NULL, non-positive sizes, lambda out of
 * range, workspace too small) return HYRF_ERR_INVALID_ARGUMENT before any
 * launch. */
hyrf_status hyrf_l1_dssim_loss(const float* img, const float* target, int32_t planes, int32_t height,
                               int32_t width, float lambda, float* loss, float* grad, void* ws,
                               size_t ws_bytes, void* stream);
size_t hyrf_l1_dssim_workspace_bytes(int32_t planes, int32_t height, int32_t width);

/* 8-bit min-max quantisation of one hash table (Sec. 4.3, compressed model),
 * decoded inside the field gather by every query when table_dtype is HYRF_U8.
 * Per level l over its T x 2 values: min_l, max_l; step_l = (max_l - min_l) / 255
 * (float32, correctly rounded); code = rint((x - min_l) / step_l) (float32
 * subtraction and division, ties to even), clamped to [0, 255]; code 0 when
 * step_l == 0.  table: device [levels][T][2] float32; codes: device
 * [levels][T][2] uint8; qparams: device [levels][2] <- (min_l, step_l).
 * Values must be finite.  Deterministic. */
hyrf_status hyrf_quantize_table(const float* table, int32_t levels, int32_t log2_T, uint8_t* codes,
                                float* qparams, void* ws, size_t ws_bytes, void* stream);
size_t hyrf_quantize_workspace_bytes(int32_t levels, int32_t log2_T);

/* ---- training-loop steps after the backward (Sec. 3.4) ---------------------- */

/* One parameter tensor of hyrf_adam_step.  param, grad, m, v: device [n]
 * float32 (m and v caller-zeroed before step 1).  param_half (nullable):
 * device [n] float16 copy written from the updated param (the float16 tables
 * of the precision variant render from it).  All pointers 16-byte aligned. */
typedef struct {
  float* param;
  float* grad;
  float* m;
  float* v;
  void* param_half;
  int64_t n;
  float lr;
} hyrf_adam_group;

#define HYRF_ADAM_MAX_GROUPS 16

/* Adam (Kingma & Ba 2015, Algorithm 1) over up to HYRF_ADAM_MAX_GROUPS
 * tensors in one launch -- the explicit Gaussians, both tables and both
 * decoders train this way (Sec. 3.4; the optimiser of 3DGS): m = b1 m +
 * (1-b1) g; v = b2 v + (1-b2) g^2; param -= lr (m / (1-b1^t)) /
 * (sqrt(v / (1-b2^t)) + eps).  step: t >= 1.  zero_grad != 0 clears grad
 * after reading it (the backward accumulates into zeroed buffers).
 * groups: HOST array of n_groups descriptors (read during the call).
 * Invalid arguments return HYRF_ERR_INVALID_ARGUMENT before any launch. */
hyrf_status hyrf_adam_step(const hyrf_adam_group* groups, int32_t n_groups, int32_t step, float beta1,
                           float beta2, float eps, int32_t zero_grad, void* stream);

/* Flags of hyrf_densify_masks. */
#define HYRF_PRUNE 1u   /* opacity below min_opacity                          */
#define HYRF_CLONE 2u   /* mean NDC gradient >= grad_threshold, small Gaussian */
#define HYRF_SPLIT 4u   /* mean NDC gradient >= grad_threshold, large Gaussian */
#define HYRF_JUDGED 8u  /* the Gaussian was in the query's visible list        */

/* Densify / prune decisions of 3DGS applied to HyRF's aggregated Gaussians
 * (Sec. 3.1 and Sec. 3.4: densify from accumulated gradients, prune
 * Gaussians with low opacity).  For every Gaussian in the visible list of q
 * (a query output: vis_count, vis_idx, opacity, scale): mean = dens_accum /
 * dens_count (0 when the count is 0); CLONE if mean >= grad_threshold and
 * max(scale) <= dense_extent, SPLIT if mean >= grad_threshold and max(scale) >
 * dense_extent; PRUNE if opacity < min_opacity; JUDGED always.  Gaussians
 * outside the list get flags 0.  flags: device [n] uint8 (overwritten).
 * n_max: the capacity q was written with (its scale stride). */
hyrf_status hyrf_densify_masks(const hyrf_query_out* q, int32_t n, int32_t n_max, const float* dens_accum,
                               const float* dens_count, float grad_threshold, float dense_extent,
                               float min_opacity, uint8_t* flags, void* stream);

/* Opacity reset of Sec. 3.4 (3DGS's periodic reset, applied to the explicit
 * opacity): opac_e[i] = min(opac_e[i], logit(value)), value in (0, 1). */
hyrf_status hyrf_reset_opacity(float* opac_e, int32_t n, float value, void* stream);

/* ---- data layout ------------------------------------------------------------ */

/* Permutation that orders the Gaussians along a Morton (Z-order) curve of
 * their contracted positions (10 bits per axis, stable for equal codes).
 * A layout utility run once, outside the render step: storing the Gaussians
 * as pos[perm[k]] -> slot k puts spatial neighbours into the same wavefront,
 * which makes the hash-grid gathers and table-gradient atomics of the coarse
 * levels coherent.  It changes no rendered value except the order of
 * equal-depth ties (ties are ordered by storage index).  perm: [n] uint32. */
hyrf_status hyrf_spatial_order(const hyrf_fields* fields, const float* pos, int32_t n, uint32_t* perm,
                               void* ws, size_t ws_bytes, void* stream);
size_t hyrf_spatial_order_workspace_bytes(int32_t n);

/* ---- sizing and errors ----------------------------------------------------- */
size_t hyrf_query_workspace_bytes(int32_t n);
size_t hyrf_bin_sort_workspace_bytes(int32_t n_views, int32_t n_max, int64_t capacity,
                                     int32_t width, int32_t height);
size_t hyrf_composite_workspace_bytes(int32_t n_views, int32_t width, int32_t height);
size_t hyrf_backward_workspace_bytes(const hyrf_fields* fields, int32_t n_views, int32_t n_max,
                                     int32_t width, int32_t height);
size_t hyrf_l1_workspace_bytes(int64_t n);
/* Message of the last failed call on this thread ("" if none). */
const char* hyrf_last_error(void);
/* Library version string. */
const char* hyrf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HYRF_H */
