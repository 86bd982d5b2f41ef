/*
 * oracle.h -- plain, slow, single-threaded CPU reference of the view-tied
 * Gaussian splatting renderer (VTGaussian-SLAM, arXiv 2506.02741).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code: only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the HIP library.
 *
 * What it computes (paper section in brackets):
 *  - view-tied Gaussians: one isotropic sphere per valid depth pixel, centre
 *    back-projected from the depth with the frame's pose, 5 parameters
 *    (colour c in R^3, radius r, opacity o)                      [Sec. 3.2]
 *  - radius initialisation r = D / f                           [App. A eq.]
 *  - splat({g}, p): RGB V', depth D' and silhouette rendered from the
 *    Gaussians of a keyframe slice (a section) at camera pose p  [Sec. 3.3-3.4]
 *  - tracking loss (Eq. 1), mapping loss (Eq. 2) with the SSIM term
 *  - gradients to c, o, r (mapping) and to the camera pose (tracking)
 *
 * Precision: every decision that selects a tile or a contributor is taken in
 * FP32 with a fixed operation order and no FMA contraction (this module is
 * compiled with -ffp-contract=off); the values of images and gradients are
 * evaluated in FP64 on those FP32 decisions.
 *
 * Conventions: poses are world->camera 3x4 row-major [R|t]; pixel (u,v) =
 * (column,row) with centres at integer coordinates; depth is z-depth.
 */
#ifndef VTGS_ORACLE_H
#define VTGS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float fx, fy, cx, cy; int32_t width, height; } orc_cam;

/* One keyframe's Gaussians in compact form (index i = 0..n-1). */
typedef struct {
  int32_t n;
  const uint32_t *pix;     /* [n] row-major pixel index in the keyframe image */
  const float *depth;      /* [n] z-depth of that pixel (m)                    */
  const float *color;      /* [3][n] planar                                    */
  const float *opacity;    /* [n]                                              */
  const float *radius;     /* [n] isotropic standard deviation (m)             */
  const float *pose;       /* [12] world->camera                               */
  orc_cam cam;
} orc_kf;

/* A view renders keyframes [kf_first, kf_first + kf_count). */
typedef struct {
  orc_cam cam;
  const float *pose;       /* [12] world->camera */
  int32_t kf_first, kf_count;
} orc_view;

typedef struct {
  float alpha_min, alpha_max, t_min, q_cut, z_near, lowpass;
  float bg[3];
  int32_t tile;
} orc_params;

/* Per (view, Gaussian) FP32 record of the preprocessing. */
typedef struct {
  float px, py, pz;        /* camera-frame centre                      */
  float mx, my;            /* projected mean (pixels)                  */
  float qa, qb, qc;        /* conic = inverse 2D covariance [[qa,qb],[qb,qc]] */
  float ext;               /* integer extent R (pixels)                */
  int32_t rect[4];         /* tx0, ty0, tx1, ty1 inclusive             */
  int32_t count;           /* tiles covered; 0 = culled                */
} orc_rec;

/* Optional FP64 value inputs over the slice's local ids (NULL => the
 * keyframes' float values), plus a left twist applied to the view pose and
 * (kf_twist) to each keyframe pose of the slice.
 * geometry64 = 0: the forward composites, in FP64, the projected mean,
 * conic and depth of the pinned FP32 records (the definition both sides
 * share bit for bit); derivatives use the FP64 geometry.  geometry64 = 1:
 * every geometric quantity is recomputed in FP64 from the (overridden)
 * inputs -- a smooth function of colour, opacity, radius and twist, for
 * finite differences and closed forms. */
typedef struct {
  const double *color;     /* [3][N] */
  const double *opacity;   /* [N]    */
  const double *radius;    /* [N]    */
  double twist[6];         /* (rho, phi): pose <- exp(twist^) * pose */
  int32_t geometry64;
  const double *depth;     /* [N] tied depth (the Gaussian's place on its ray) */
  const double *kf_twist;  /* [kf_count][6]: keyframe pose <- exp(twist^) * pose */
} orc_values;

/* ---- keyframe ingestion: valid pixels -> compact Gaussian list ---- */
int32_t orc_ingest_count(const float *depth_img, const uint8_t *mask,
                         int32_t H, int32_t W, int32_t stride);
int32_t orc_ingest_fill(const float *depth_img, const float *rgb_img, const uint8_t *mask,
                        int32_t H, int32_t W, int32_t stride, float fx, float o_init,
                        int32_t n, uint32_t *pix, float *depth, float *color,
                        float *opacity, float *radius);

/* ---- FP32 preprocessing and tile lists ---- */
void orc_relpose32(const float *Tv, const float *Tk, float *M);
int32_t orc_slice_size(const orc_view *v, const orc_kf *kfs);
int32_t orc_preprocess32(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                         orc_rec *out);
int64_t orc_tile_lists(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                       uint64_t *keys, uint32_t *vals, uint32_t *ranges, int64_t cap);

/* ---- visibility (Sec. 3.3): a source frame's depth point -- pixel (u, v)
 * with depth d > 0, back-projected with the source intrinsics and moved
 * from the source pose to a target pose -- is visible in the target when
 * its target-camera depth p_z > z_near lies within rel_tol (1 %) of the
 * target depth map bilinearly interpolated at its projection (all four
 * neighbours inside the map and valid).  FP32 in a pinned order (no FMA):
 * the relative pose, back-projection, transform and projection of the
 * records, then bilinear top/bottom rows and their blend, then
 * |p_z - D| <= rel_tol * D.  vis [n_tgt][H*W] (0/1), counts [n_tgt] the
 * visible points per target (or NULL). ---- */
int orc_visibility(const float *src_depth, const orc_cam *src_cam, const float *src_pose,
                   int32_t n_tgt, const float *const *tgt_depth, const orc_cam *tgt_cam,
                   const float *const *tgt_pose, float rel_tol, float z_near, uint8_t *vis,
                   int64_t *counts);

/* ---- forward ---- */
/* Full image when n_px < 0 (outputs have P = W*H entries); otherwise only
 * the listed pixel indices (outputs have n_px entries).  rgb is planar
 * [3][P].  marginal[p] != 0 where some FP32 decision at that pixel lies
 * within a relative distance `margin` of its threshold (bit 1: a candidate
 * test, 2: the alpha_max clamp, 4: a stop decision).  Returns 0 on success
 * (1 when the superset property failed somewhere). */
int orc_render_fwd(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                   const orc_values *val, float margin, int32_t n_px, const int32_t *px_idx,
                   double *rgb, double *depth, double *sil, double *t_final,
                   int32_t *n_contrib, uint8_t *marginal);

/* The other outcomes of the listed pixels' near-tie decisions (candidate
 * tests, then stop decisions, numbered as met): variant j of pixel i takes
 * decision j the other way.  n_dec[i] receives the number of near-tie
 * decisions of pixel i; rgb [n_px][max_alt][3], depth and sil
 * [n_px][max_alt] receive variants j < min(n_dec[i], max_alt).  Returns 0
 * on success. */
int orc_render_alt(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                   const orc_values *val, float margin, int32_t n_px, const int32_t *px_idx,
                   int32_t max_alt, double *rgb, double *depth, double *sil, int32_t *n_dec);

/* ---- backward: exact derivative of the forward with the FP32 contributor
 * sets held fixed.  g_color [3][N], g_opac [N], g_rad [N] over the slice's
 * local ids (overwritten), g_twist [6] (overwritten).  g_mag (NULL or
 * [5N + 6]: colour, opacity, radius, twist) receives each gradient's sum of
 * absolute summands -- every per-pixel term, and every product and sum
 * inside it, taken in absolute value -- the scale of the rounding error of
 * any evaluation of those sums in a shorter precision.  g_kdepth (NULL or
 * [N]) receives dLoss/d(tied depth) of every Gaussian -- its centre moved
 * along its pixel's ray -- and g_kpose (NULL or [kf_count][6]) the gradient
 * of a left twist (rho, phi) of each keyframe pose of the slice, through the
 * centres of its tied Gaussians; g_kmag (NULL, or [N + 6 kf_count] when
 * g_mag is given) their sums of absolute summands. ---- */
int orc_render_bwd(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                   const orc_values *val, const double *g_rgb, const double *g_depth,
                   const double *g_sil, double *g_color, double *g_opac, double *g_rad,
                   double *g_twist, double *g_mag, double *g_kdepth, double *g_kpose,
                   double *g_kmag);

/* ---- losses ---- */
double orc_track_loss(int32_t P, const double *rgb, const double *depth, const double *sil,
                      const float *obs_rgb, const float *obs_depth, const uint8_t *vis,
                      double alpha, double beta, double sil_thr,
                      double *g_rgb, double *g_depth);
double orc_ssim(int32_t H, int32_t W, const double *x, const double *y, double *g_x);
double orc_map_loss(int32_t H, int32_t W, const double *rgb, const double *depth,
                    const float *obs_rgb, const float *obs_depth,
                    double rho, double tau, double sigma, double *g_rgb, double *g_depth);

/* ---- optimiser pieces ---- */
void orc_se3_exp(const double *xi, double *T);       /* T [12] */
void orc_adam(int64_t n, double *param, const double *grad, double *m, double *v,
              int64_t t, double lr, double b1, double b2, double eps);

#ifdef __cplusplus
}
#endif
#endif
