/*
 * vtgs.h -- C ABI of the MI355X (gfx950) view-tied Gaussian splatting
 * renderer: the differentiable splat of VTGaussian-SLAM (arXiv 2506.02741)
 * with its tracking and mapping inner steps.
 *
 * The method (paper sections in brackets):
 *  - A view-tied Gaussian is an isotropic sphere tied to one valid depth
 *    pixel of a keyframe; its centre is that pixel back-projected with the
 *    keyframe's depth and pose, so only colour c (3), radius r and opacity o
 *    are stored and learned [Sec. 3.2].  Keyframes are grouped in sections;
 *    a view renders a slice of consecutive keyframes [Sec. 3.2-3.4].
 *  - splat({g}, p) renders RGB V', depth D' and a silhouette from the
 *    Gaussians at camera pose p [Sec. 3.3 Eq. 1, Sec. 3.4].
 *  - Tracking optimises the pose with the Gaussians fixed, minimising
 *    alpha W|V - V'|_1 + beta W|D - D'|_1 (Eq. 1) [Sec. 3.3].
 *  - Mapping optimises colour, radius and opacity of the learnable slice,
 *    minimising rho|V - V'|_1 + tau L_SSIM + sigma U|D - D'|_1 (Eq. 2)
 *    [Sec. 3.4]; learning rates from App. A.
 *
 * Renderer readings where the paper is silent: r is the std-dev of the
 * sphere; first-order projection Sigma_2D = r^2 J J^T + lowpass*I; a
 * Gaussian reaches pixels with q = d^T Sigma^-1 d <= q_cut;
 * alpha = min(alpha_max, o exp(-q/2)) and alpha < alpha_min is skipped;
 * compositing stops before transmittance would fall below t_min; order is
 * ascending depth of the centre, ties by view-local id; depth output is
 * sum z alpha T (not normalised); silhouette = 1 - T_final.
 *
 * Conventions
 *  - FP32 everywhere.  Poses are world->camera 3x4 row-major [R|t].
 *  - Pixel (u, v) = (column, row); centres at integer coordinates; images
 *    are row-major; RGB is planar [3][P].
 *  - Every pointer documented "device" is HIP device memory owned by the
 *    caller.  The library allocates no device memory: a plan's state lives in
 *    a caller-owned workspace sized by vtgs_plan_workspace_bytes(), or in the
 *    library's static scratch (vtgs_render_fwd_static).  It keeps host-side
 *    plan objects only.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *    compute calls are asynchronous on that stream and never synchronise,
 *    except vtgs_plan_status().
 *  - Errors: a negative vtgs_status.  Argument errors are detected on the
 *    host before anything is enqueued; vtgs_last_error() (thread-local)
 *    describes the last failure.  Errors found on the device (pair capacity
 *    exceeded, non-finite loss) set sticky flags in the workspace that
 *    vtgs_plan_status() reports; outputs of a flagged call are undefined.
 *    No C++ exception crosses this boundary.
 */
#ifndef VTGS_H
#define VTGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VTGS_ABI_VERSION 2

typedef enum {
  VTGS_OK = 0,
  VTGS_E_ARG = -1,        /* invalid argument, nothing enqueued            */
  VTGS_E_HIP = -2,        /* a HIP runtime call failed                     */
  VTGS_E_WORKSPACE = -3,  /* workspace missing, unbound or too small       */
  VTGS_E_CAPACITY = -4,   /* device: more (Gaussian, tile) pairs than room */
  VTGS_E_NONFINITE = -5   /* device: a loss was not finite                 */
} vtgs_status;

/* Pinhole intrinsics and image size. */
typedef struct {
  float fx, fy, cx, cy;
  int32_t width, height;
} vtgs_camera;

/* One keyframe's view-tied Gaussians in compact form (index i < n)
 * [Sec. 3.2].  Produced by vtgs_ingest_*. */
typedef struct {
  int32_t n;                 /* number of Gaussians                          */
  const uint32_t *pix;       /* device [n] row-major pixel index in the keyframe */
  float *depth;              /* device [n] z-depth of that pixel (m), > 0: the
                                Gaussian's place on its pixel's ray; map_step
                                moves it when depth_adam != NULL              */
  float *color;              /* device [3][n] planar colour c                 */
  float *opacity;            /* device [n] opacity o in (0, 1]                */
  float *radius;             /* device [n] radius r (m), > 0                  */
  float *pose;               /* device [12] world->camera of the keyframe;
                                map_step adjusts it when pose_adam != NULL    */
  vtgs_camera cam;           /* keyframe intrinsics and image size            */
  int32_t learnable;         /* 1: receives gradients / optimiser steps       */
  float *g_color;            /* device [3][n], render_bwd adds (+=); or NULL  */
  float *g_opacity;          /* device [n], or NULL                           */
  float *g_radius;           /* device [n], or NULL                           */
  float *adam;               /* device [10][n]: Adam m[5], v[5] over
                                (c0,c1,c2, logit o, log r) for map_step; or NULL */
  /* Geometry of a learnable keyframe (supplementary: Gaussians movable
   * along the ray; Sec. 3.5: bundle adjustment of a keyframe pose through
   * its tied Gaussians' centres).  Any of them non-NULL makes the backward
   * also carry dLoss/d(centre) per Gaussian. */
  float *g_depth;            /* device [n], render_bwd adds dLoss/d(depth) (+=); or NULL */
  float *g_pose;             /* device [6], render_bwd adds dLoss/d(xi) of a left
                                twist xi = (rho, phi) of the pose, pose <-
                                exp(xi^) pose, at xi = 0 (+=); or NULL         */
  float *depth_adam;         /* device [2][n]: Adam m, v of the depth for map_step; or NULL */
  float *pose_adam;          /* device [13]: Adam m[6], v[6], t of the pose twist for
                                map_step (lr_trans on rho, lr_rot on phi, then
                                pose <- exp(step^) pose); or NULL              */
} vtgs_keyframe;

/* One rendered view: keyframes [kf_first, kf_first + kf_count) of the
 * plan's keyframe array, seen through `cam` at `pose`. */
typedef struct {
  vtgs_camera cam;           /* output resolution and intrinsics              */
  float *pose;               /* device [12] world->camera; track_step updates it */
  int32_t kf_first, kf_count;
  const float *obs_rgb;      /* device [3][H*W] observed RGB (track/map), or NULL */
  const float *obs_depth;    /* device [H*W] observed depth, 0 = invalid, or NULL */
  const uint8_t *vis;        /* device [H*W] visibility mask for Eq. 1 W, or NULL = all */
  float *pose_adam;          /* device [13]: m[6], v[6], t for track_step, or NULL */
} vtgs_view;

typedef struct {
  float alpha_min;           /* skip alpha below this (default 1/255)          */
  float alpha_max;           /* clamp alpha (default 0.99)                     */
  float t_min;               /* stop before T < t_min (default 1e-4)           */
  float q_cut;               /* cut-off of q (default 11.0826 = 2 ln 255 up)   */
  float z_near;              /* cull centres with z <= z_near (default 0.01 m) */
  float lowpass;             /* added to Sigma_2D diagonal (default 0.3 px^2)  */
  float bg[3];               /* background colour (default 0)                  */
  int32_t tile;              /* 8, 16 or 32 (default 16)                       */
  int32_t batch;             /* LDS batch of Gaussians: 128, 256, 512 (default 256) */
} vtgs_params;

/* Eq. 1 weights and pose learning rates (App. A); sil_thr is the coverage
 * threshold of the mask W (default 0.5). */
typedef struct { float alpha, beta, lr_rot, lr_trans, sil_thr; } vtgs_track_cfg;

/* Eq. 2 weights and learning rates of colour, opacity, radius (App. A), of
 * the tied depths of keyframes with depth_adam, and of the poses of
 * keyframes with pose_adam (translation, rotation). */
typedef struct {
  float rho, tau, sigma, lr_color, lr_opacity, lr_radius, lr_depth, lr_trans, lr_rot;
} vtgs_map_cfg;

typedef struct vtgs_plan vtgs_plan;

/* ---- library ---- */
int32_t vtgs_abi_version(void);
const char *vtgs_last_error(void);
void vtgs_default_params(vtgs_params *out);

/* ---- keyframe ingestion [Sec. 3.2; App. A r = D / f] --------------------
 * A Gaussian is tied to every pixel (s*i, s*j) of the stride grid whose
 * depth is > 0 and finite and whose mask byte (if mask != NULL) is non-zero,
 * in row-major order.
 * vtgs_ingest_count writes that number to *count (device int32).  The
 * caller then allocates the compact arrays for n Gaussians and calls
 * vtgs_ingest_fill with the same depth/mask/stride and the same scratch
 * (whose contents count left behind), which writes pix, depth, colour (from
 * rgb_img [3][H*W], untouched if rgb_img == NULL), opacity = o_init and
 * radius = stride * depth / fx.  scratch: device, at least
 * vtgs_ingest_scratch_bytes(H, W, stride) bytes. */
int64_t vtgs_ingest_scratch_bytes(int32_t H, int32_t W, int32_t stride);
int vtgs_ingest_count(const float *depth_img, const uint8_t *mask, int32_t H, int32_t W,
                      int32_t stride, void *scratch, int64_t scratch_bytes, int32_t *count,
                      void *stream);
int vtgs_ingest_fill(const float *depth_img, const float *rgb_img, const uint8_t *mask,
                     int32_t H, int32_t W, int32_t stride, float fx, float o_init,
                     const void *scratch, int64_t scratch_bytes, int32_t n, uint32_t *pix,
                     float *depth, float *color, float *opacity, float *radius, void *stream);

/* ---- complement initialisation [Sec. 3.4] ---------------------------------
 * mask[p] = 1 where the current Gaussians leave pixel p of a frame
 * uncovered -- the silhouette of their rendering at the frame's pose,
 * sil[p] (device [n]), below thr (the paper's 0.5) -- and the frame's depth
 * depth_img[p] (device [n]) is valid (> 0 and finite); else 0.  Passed to
 * vtgs_ingest_count / vtgs_ingest_fill as their mask, it ties new
 * Gaussians to exactly those pixels.  mask: device uint8 [n].  VTGS_E_ARG
 * for NULL arrays or n < 0, nothing enqueued. */
int vtgs_uncovered_mask(const float *sil, const float *depth_img, int64_t n, float thr,
                        uint8_t *mask, void *stream);

/* ---- plans --------------------------------------------------------------
 * A plan fixes a batch of views over an array of keyframes (host copies of
 * the descriptors, device pointers inside are borrowed and must stay valid
 * while the plan is used) and the room for (Gaussian, tile) pairs.
 * pair_capacity <= 0 picks ceil(1.5 (1 + 10/tile)^2) pairs per (view,
 * Gaussian) record plus 65536, at most 2^31 - 1; an explicit pair_capacity
 * above 2^31 - 1 is VTGS_E_ARG (tile lists use 32-bit positions).  The caller
 * allocates vtgs_plan_workspace_bytes() bytes of device memory (256-byte
 * aligned) and binds it once with vtgs_plan_bind(), which uploads the
 * descriptors on `stream`.  A plan is used by one host thread at a time.
 * Output images of a plan are packed: view v occupies pixels
 * [vtgs_plan_view_offset(v), + W_v*H_v) of every plane. */
int vtgs_plan_create(const vtgs_keyframe *kfs, int32_t n_kf, const vtgs_view *views,
                     int32_t n_views, const vtgs_params *prm, int64_t pair_capacity,
                     vtgs_plan **out);
void vtgs_plan_destroy(vtgs_plan *plan);
int64_t vtgs_plan_workspace_bytes(const vtgs_plan *plan);
int64_t vtgs_plan_pixels(const vtgs_plan *plan);
int64_t vtgs_plan_view_offset(const vtgs_plan *plan, int32_t view);
int64_t vtgs_plan_records(const vtgs_plan *plan);
int64_t vtgs_plan_tiles(const vtgs_plan *plan);
int64_t vtgs_plan_pair_capacity(const vtgs_plan *plan);
int vtgs_plan_bind(vtgs_plan *plan, void *ws, int64_t ws_bytes, void *stream);
/* Synchronises `stream`; returns VTGS_OK, VTGS_E_CAPACITY (and the pairs
 * the last render needed in *pairs_needed) or VTGS_E_NONFINITE.  Clears the
 * flags when `clear` != 0. */
int vtgs_plan_status(vtgs_plan *plan, int64_t *pairs_needed, int32_t clear, void *stream);

/* ---- render_fwd: splat({g}, p) for every view of the plan [Sec. 3.3] ----
 * rgb [3][P], depth [P], sil [P] device outputs (each may be NULL).  The
 * per-pixel state the backward needs (final transmittance, last
 * contributor) stays in the workspace. */
int vtgs_render_fwd(vtgs_plan *plan, float *rgb, float *depth, float *sil, void *stream);

/* ---- render_fwd_static: render_fwd for callers that cannot allocate ------
 * For callers that cannot allocate device memory or be handed a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same forward as vtgs_render_fwd, with the plan's state
 * kept in the library's own static scratch of VTGS_STATIC_SCRATCH_BYTES on
 * the current device instead of a caller workspace.  The plan need not be
 * bound; afterwards it is bound to that scratch (render_bwd, track_step and
 * map_step then use it too) until vtgs_plan_bind rebinds it.  A plan whose
 * vtgs_plan_workspace_bytes exceeds the scratch is VTGS_E_WORKSPACE, with
 * nothing enqueued.  The call allocates no device memory.  The first call
 * with a plan on a device (or after another plan used the device's
 * scratch) uploads the plan's descriptor tables with an asynchronous
 * host-to-device copy from host memory the plan owns and clears the
 * scratch's counters with fill kernels; later calls with the same plan only
 * enqueue kernels.  Every plan on a device shares that device's scratch, so
 * calls that overlap on one device -- on different streams, or a plan's
 * state read after another plan used the scratch -- race. */
#define VTGS_STATIC_SCRATCH_BYTES (128ll << 20)
int vtgs_render_fwd_static(vtgs_plan *plan, float *rgb, float *depth, float *sil, void *stream);

/* ---- render_bwd: gradients of a scalar loss through the last render_fwd --
 * g_rgb [3][P], g_depth [P], g_sil [P]: dLoss/d(outputs), device, NULL = 0.
 * Adds dLoss/dc, dLoss/do, dLoss/dr into g_color/g_opacity/g_radius of every
 * learnable keyframe that has them, summed over views [Sec. 3.4], and
 * dLoss/d(depth) and the keyframe pose twist gradient into g_depth / g_pose
 * where given [Sec. 3.5; supplementary, Gaussians movable along the ray];
 * writes dLoss/dxi [n_views][6] into g_twist (device, or NULL) where
 * xi = (rho, phi) is a left twist of each view's world->camera pose,
 * pose <- exp(xi^) pose, taken at xi = 0 [Sec. 3.3]. */
int vtgs_render_bwd(vtgs_plan *plan, const float *g_rgb, const float *g_depth,
                    const float *g_sil, float *g_twist, void *stream);

/* ---- track_step: `iters` tracking iterations of every view [Sec. 3.3] ----
 * Each iteration renders the view's slice at view.pose, evaluates Eq. 1
 * against view.obs_rgb / view.obs_depth with W = vis & (D > 0) &
 * (silhouette > sil_thr) held fixed, back-propagates to the twist, takes an
 * Adam step on it (lr_trans on rho, lr_rot on phi; state in view.pose_adam,
 * beta = (0.9, 0.999), eps = 1e-8) and retracts pose <- exp(step^) pose.
 * loss: device [iters][n_views] (or NULL).  Everything stays on the device;
 * nothing is read back. */
int vtgs_track_step(vtgs_plan *plan, const vtgs_track_cfg *cfg, int32_t iters, float *loss,
                    void *stream);

/* ---- map_step: one mapping iteration over every view [Sec. 3.4] ----------
 * Renders each view, evaluates Eq. 2 against its observation (means over
 * pixels; SSIM with an 11x11 Gaussian window, sigma 1.5), sums the views'
 * losses, back-propagates to c, o, r of the learnable keyframes and takes
 * one Adam step on (c, logit o, log r) with lr_color, lr_opacity, lr_radius
 * (state in keyframe.adam, step counter *step on the device, incremented).
 * A learnable keyframe with depth_adam also moves its Gaussians along their
 * rays (Adam on depth, lr_depth), and one with pose_adam adjusts its pose
 * (Adam on a left twist, lr_trans / lr_rot, then pose <- exp(step^) pose;
 * its own step count in pose_adam[12]) [Sec. 3.5].  The centres move only
 * from the next iteration on.  loss: device [n_views] (or NULL). */
int vtgs_map_step(vtgs_plan *plan, const vtgs_map_cfg *cfg, int32_t *step, float *loss,
                  void *stream);

/* ---- visibility check [Sec. 3.3] ----------------------------------------
 * A frame to test against: its depth map (device [H*W], 0 = invalid), its
 * intrinsics and image size, and its world->camera pose (device [12]). */
typedef struct {
  const float *depth;
  vtgs_camera cam;
  const float *pose;
} vtgs_frame_ref;

/* The point of source pixel (u, v) with depth d > 0 (back-projected with
 * src_cam at src_pose) is visible in a target when its depth in the target
 * camera, p_z > z_near, lies within rel_tol (the paper's 1 %: 0.01) of the
 * target's depth map bilinearly interpolated at its projection, the four
 * neighbours inside the map and valid.  FP32 in a fixed operation order,
 * the back-projection and projection being those of the splat's records.
 * mask: device [H*W] of the source, 1 where the point is visible in at
 * least one target (the union Eq. 1's W takes over a section's head, middle
 * and last frames), or NULL.  counts: device int32 [n_targets], the visible
 * points per target (the overlap selection), or NULL.  Targets may have
 * other resolutions than the source.  Asynchronous on `stream`; argument
 * errors (NULL source or target arrays, bad cameras, n_targets < 1,
 * rel_tol < 0) return VTGS_E_ARG with nothing enqueued. */
int vtgs_visibility(const float *src_depth, const vtgs_camera *src_cam, const float *src_pose,
                    const vtgs_frame_ref *targets, int32_t n_targets, float rel_tol, float z_near,
                    uint8_t *mask, int32_t *counts, void *stream);

/* ---- measurement ----------------------------------------------------------
 * Stage timing: enable != 0 starts recording HIP events on the call's stream
 * around every stage the plan launches (preprocess, sort, compositing, ...);
 * with enable = R > 1 (at most 64) the two compositing stages, which only
 * overwrite what they write, are launched R times back to back between their
 * events, so that the per-launch time leaves out the events' own overhead.
 * enable == 0 stops, synchronises those events and writes, per stage index
 * s < VTGS_N_STAGES, the summed milliseconds ms[s] and launches count[s]
 * (either array may be NULL).  vtgs_stage_name(s) names stage s. */
#define VTGS_N_STAGES 10
const char *vtgs_stage_name(int32_t stage);
int vtgs_plan_timing(vtgs_plan *plan, int32_t enable, double *ms, int64_t *count);

/* ---- inspection (tests) -------------------------------------------------
 * Copies of the workspace state after vtgs_render_fwd, on `stream`:
 * records [n_rec][12] float (mx, my, qa, qb, qc, o, z, R, c0, c1, c2, r) and
 * rect [n_rec][4] int32 (tx0, ty0, tx1, ty1; tx0 > tx1 when culled);
 * ranges [n_tiles][2] uint32 (start, end) of each tile's sorted list; ids
 * [pair_capacity] uint32 view-local ids in sorted order; n_pairs (device
 * int64) the pairs of the last render.  Any pointer may be NULL. */
int vtgs_debug_state(vtgs_plan *plan, float *records, int32_t *rect, uint32_t *ranges,
                     uint32_t *ids, int64_t *n_pairs, void *stream);

/* Copies, on `stream`, of the plan's internal images (device [5][P]: RGB,
 * depth, silhouette of the last forward that track_step or map_step ran)
 * and of the upstream gradients map_step formed from Eq. 2 (device [5][P]:
 * dLoss/dRGB, dLoss/ddepth, and a zero silhouette plane) [Sec. 3.4].
 * Either pointer may be NULL. */
int vtgs_debug_images(vtgs_plan *plan, float *img, float *gimg, void *stream);

/* Adds, on `stream`, the per-Gaussian gradients (colour, opacity, radius,
 * and depth and the keyframe pose twist when the plan carries geometry) that
 * the last backward to colour/opacity/radius left in the workspace -- the
 * values map_step's Adam step used -- into g_color, g_opacity, g_radius,
 * g_depth and g_pose of every learnable keyframe that has them.  VTGS_E_ARG
 * when the plan has no learnable keyframe or no such backward ran on it yet. */
int vtgs_debug_gather(vtgs_plan *plan, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* VTGS_H */
