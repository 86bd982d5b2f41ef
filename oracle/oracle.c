/*
 * oracle.c -- plain single-threaded CPU reference of the view-tied Gaussian
 * splatting renderer (VTGaussian-SLAM, arXiv 2506.02741).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.  Written from the
 * paper (Sec. 3.2 view-tied Gaussians, Sec. 3.3 Eq. 1, Sec. 3.4 Eq. 2,
 * App. A radius initialisation and learning rates) and from the readings
 * of what the paper leaves open, which are listed in the design notes:
 * sphere = isotropic std-dev r, first-order (EWA) projection with a
 * low-pass term, cut-off q <= Q_CUT, alpha = min(alpha_max, o exp(-q/2)),
 * skip alpha < alpha_min, stop before T drops under t_min, depth order with
 * the view-local id breaking ties.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.
 * The FP32 decision path relies on IEEE single arithmetic with no
 * contraction; every value and gradient is then evaluated in FP64.
 * The same source built with -fopenmp (the all-cores timing of the CPU
 * baseline) splits the per-pixel loops over threads: the forward's pixels
 * are independent (its output is bitwise the single-threaded one); the
 * backward gives each thread a contiguous range of rows with its own
 * gradient sums, added in row order.  Without OpenMP there is one range and
 * the sums run in pixel order.
 *
 * Parity pins: see tests/test_oracle_*.py (closed forms, invariants,
 * brute force, finite differences, library SSIM).
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* keyframe ingestion (Sec. 3.2: a Gaussian at every pixel with valid depth; */
/* App. A: r = D / f; stride s > 1 keeps pixels (s*i, s*j) with r = s*D/f)   */
/* ------------------------------------------------------------------------ */

static int valid_depth(float d) { return d > 0.f && d <= FLT_MAX; }

int32_t orc_ingest_count(const float *depth_img, const uint8_t *mask,
                         int32_t H, int32_t W, int32_t stride) {
  int32_t n = 0;
  for (int32_t v = 0; v < H; v += stride)
    for (int32_t u = 0; u < W; u += stride) {
      int64_t p = (int64_t)v * W + u;
      if (valid_depth(depth_img[p]) && (!mask || mask[p])) n++;
    }
  return n;
}

int32_t orc_ingest_fill(const float *depth_img, const float *rgb_img, const uint8_t *mask,
                        int32_t H, int32_t W, int32_t stride, float fx, float o_init,
                        int32_t n, uint32_t *pix, float *depth, float *color,
                        float *opacity, float *radius) {
  int32_t i = 0;
  int64_t P = (int64_t)H * W;
  for (int32_t v = 0; v < H; v += stride)
    for (int32_t u = 0; u < W; u += stride) {
      int64_t p = (int64_t)v * W + u;
      if (!(valid_depth(depth_img[p]) && (!mask || mask[p]))) continue;
      if (i >= n) return -1;
      float d = depth_img[p];
      pix[i] = (uint32_t)p;
      depth[i] = d;
      if (rgb_img)
        for (int c = 0; c < 3; c++) color[(int64_t)c * n + i] = rgb_img[c * P + p];
      opacity[i] = o_init;
      radius[i] = ((float)stride * d) / fx;
      i++;
    }
  return i;
}

/* ------------------------------------------------------------------------ */
/* FP32 preprocessing with a fixed operation order (decides tiles)          */
/* ------------------------------------------------------------------------ */

void orc_relpose32(const float *Tv, const float *Tk, float *M) {
  /* M = Tv * Tk^-1 = [Rv Rk^T | tv - (Rv Rk^T) tk] */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      M[4 * i + j] = (Tv[4 * i + 0] * Tk[4 * j + 0] + Tv[4 * i + 1] * Tk[4 * j + 1]) +
                     Tv[4 * i + 2] * Tk[4 * j + 2];
  for (int i = 0; i < 3; i++)
    M[4 * i + 3] = Tv[4 * i + 3] -
                   ((M[4 * i + 0] * Tk[3] + M[4 * i + 1] * Tk[7]) + M[4 * i + 2] * Tk[11]);
}

int32_t orc_slice_size(const orc_view *v, const orc_kf *kfs) {
  int32_t n = 0;
  for (int32_t k = 0; k < v->kf_count; k++) n += kfs[v->kf_first + k].n;
  return n;
}

static int32_t tiles_of(int32_t len, int32_t B) { return (len + B - 1) / B; }

static void pre32(const float *M, const orc_cam *kc, const orc_cam *vc, uint32_t pix, float d,
                  float r, const orc_params *prm, int32_t tiles_x, int32_t tiles_y, orc_rec *o) {
  memset(o, 0, sizeof(*o));
  int32_t u = (int32_t)(pix % (uint32_t)kc->width), v = (int32_t)(pix / (uint32_t)kc->width);
  /* back-projection of the depth pixel in its keyframe (Sec. 3.2) */
  float xk = (((float)u - kc->cx) / kc->fx) * d;
  float yk = (((float)v - kc->cy) / kc->fy) * d;
  float zk = d;
  /* keyframe camera -> view camera */
  float px = ((M[0] * xk + M[1] * yk) + M[2] * zk) + M[3];
  float py = ((M[4] * xk + M[5] * yk) + M[6] * zk) + M[7];
  float pz = ((M[8] * xk + M[9] * yk) + M[10] * zk) + M[11];
  o->px = px; o->py = py; o->pz = pz;
  if (!(pz > prm->z_near)) return;
  /* pinhole projection of the centre */
  float mx = vc->fx * (px / pz) + vc->cx;
  float my = vc->fy * (py / pz) + vc->cy;
  /* Sigma_2D = r^2 J J^T + s I with J the projection Jacobian */
  float a = vc->fx / pz, b = vc->fy / pz;
  float zz = pz * pz;
  float jx = -(vc->fx * px) / zz, jy = -(vc->fy * py) / zz;
  float r2 = r * r;
  float s11 = r2 * (a * a + jx * jx) + prm->lowpass;
  float s12 = r2 * (jx * jy);
  float s22 = r2 * (b * b + jy * jy) + prm->lowpass;
  float det = s11 * s22 - s12 * s12;
  if (!(det > 0.f)) return;
  float mid = 0.5f * (s11 + s22);
  float lmax = mid + sqrtf(fmaxf(0.f, mid * mid - det));
  float R = ceilf(sqrtf(prm->q_cut * lmax));
  if (!(isfinite(mx) && isfinite(my) && isfinite(R))) return;
  o->mx = mx; o->my = my;
  o->qa = s22 / det; o->qb = -s12 / det; o->qc = s11 / det;
  o->ext = R;
  float invB = 1.0f / (float)prm->tile;
  float fx0 = fmaxf(floorf((mx - R) * invB), 0.f);
  float fy0 = fmaxf(floorf((my - R) * invB), 0.f);
  float fx1 = fminf(floorf((mx + R) * invB), (float)(tiles_x - 1));
  float fy1 = fminf(floorf((my + R) * invB), (float)(tiles_y - 1));
  if (fx0 > fx1 || fy0 > fy1) return;
  o->rect[0] = (int32_t)fx0; o->rect[1] = (int32_t)fy0;
  o->rect[2] = (int32_t)fx1; o->rect[3] = (int32_t)fy1;
  o->count = (o->rect[2] - o->rect[0] + 1) * (o->rect[3] - o->rect[1] + 1);
}

int32_t orc_preprocess32(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                         orc_rec *out) {
  int32_t tx = tiles_of(v->cam.width, prm->tile), ty = tiles_of(v->cam.height, prm->tile);
  int32_t id = 0;
  for (int32_t s = 0; s < v->kf_count; s++) {
    const orc_kf *k = &kfs[v->kf_first + s];
    float M[12];
    orc_relpose32(v->pose, k->pose, M);
    for (int32_t i = 0; i < k->n; i++, id++)
      pre32(M, &k->cam, &v->cam, k->pix[i], k->depth[i], k->radius[i], prm, tx, ty, &out[id]);
  }
  return id;
}

static uint32_t fbits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

typedef struct { uint64_t key; uint32_t val; } kv;

static int cmp_kv(const void *a, const void *b) {
  const kv *x = (const kv *)a, *y = (const kv *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->val > y->val) - (x->val < y->val);
}

int64_t orc_tile_lists(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                       uint64_t *keys, uint32_t *vals, uint32_t *ranges, int64_t cap) {
  int32_t N = orc_slice_size(v, kfs);
  orc_rec *rec = (orc_rec *)malloc(sizeof(orc_rec) * (size_t)(N > 0 ? N : 1));
  orc_preprocess32(v, kfs, prm, rec);
  int32_t tx = tiles_of(v->cam.width, prm->tile), ty = tiles_of(v->cam.height, prm->tile);
  int64_t K = 0;
  for (int32_t g = 0; g < N; g++) K += rec[g].count;
  kv *pairs = (kv *)malloc(sizeof(kv) * (size_t)(K > 0 ? K : 1));
  int64_t j = 0;
  /* one (tile, depth) key per tile of the Gaussian's rectangle */
  for (int32_t g = 0; g < N; g++) {
    if (!rec[g].count) continue;
    for (int32_t y = rec[g].rect[1]; y <= rec[g].rect[3]; y++)
      for (int32_t x = rec[g].rect[0]; x <= rec[g].rect[2]; x++) {
        pairs[j].key = ((uint64_t)(uint32_t)(y * tx + x) << 32) | fbits(rec[g].pz);
        pairs[j].val = (uint32_t)g;
        j++;
      }
  }
  qsort(pairs, (size_t)K, sizeof(kv), cmp_kv);
  for (int32_t t = 0; t < tx * ty; t++) ranges[2 * t] = ranges[2 * t + 1] = 0;
  for (int64_t i = 0; i < K; i++) {
    if (i < cap) { keys[i] = pairs[i].key; vals[i] = pairs[i].val; }
    uint32_t t = (uint32_t)(pairs[i].key >> 32);
    if (i == 0 || (uint32_t)(pairs[i - 1].key >> 32) != t) ranges[2 * t] = (uint32_t)i;
    ranges[2 * t + 1] = (uint32_t)(i + 1);
  }
  free(pairs);
  free(rec);
  return K;
}

/* ------------------------------------------------------------------------ */
/* visibility of a frame's depth points in other views (Sec. 3.3)            */
/* ------------------------------------------------------------------------ */

/* Bilinear interpolation of a depth map at (x, y): the four neighbours
 * must lie inside the map and hold valid (> 0) depths.  Returns 0 when the
 * interpolation is undefined. */
static int depth_bilinear(const float *D, int32_t W, int32_t H, float x, float y, float *out) {
  /* decide on the float coordinates before any conversion to int */
  if (!(x >= 0.0f && y >= 0.0f && x < (float)(W - 1) && y < (float)(H - 1))) return 0;
  float fx0 = floorf(x), fy0 = floorf(y);
  int32_t x0 = (int32_t)fx0, y0 = (int32_t)fy0;
  float d00 = D[(int64_t)y0 * W + x0], d01 = D[(int64_t)y0 * W + x0 + 1];
  float d10 = D[(int64_t)(y0 + 1) * W + x0], d11 = D[(int64_t)(y0 + 1) * W + x0 + 1];
  if (!(d00 > 0.0f && d01 > 0.0f && d10 > 0.0f && d11 > 0.0f)) return 0;
  float ax = x - fx0, ay = y - fy0;
  float top = d00 + ax * (d01 - d00);
  float bot = d10 + ax * (d11 - d10);
  *out = top + ay * (bot - top);
  return 1;
}

int orc_visibility(const float *src_depth, const orc_cam *src_cam, const float *src_pose,
                   int32_t n_tgt, const float *const *tgt_depth, const orc_cam *tgt_cam,
                   const float *const *tgt_pose, float rel_tol, float z_near, uint8_t *vis,
                   int64_t *counts) {
  int32_t W = src_cam->width, H = src_cam->height;
  int64_t P = (int64_t)W * H;
  for (int32_t t = 0; t < n_tgt; t++) {
    float M[12];
    orc_relpose32(tgt_pose[t], src_pose, M);
    const orc_cam *tc = &tgt_cam[t];
    int64_t cnt = 0;
    for (int64_t p = 0; p < P; p++) {
      uint8_t v = 0;
      float d = src_depth[p];
      if (d > 0.0f) {
        int32_t u = (int32_t)(p % W), w = (int32_t)(p / W);
        /* back-projection and transform in the pinned order of the records */
        float xk = (((float)u - src_cam->cx) / src_cam->fx) * d;
        float yk = (((float)w - src_cam->cy) / src_cam->fy) * d;
        float zk = d;
        float px = ((M[0] * xk + M[1] * yk) + M[2] * zk) + M[3];
        float py = ((M[4] * xk + M[5] * yk) + M[6] * zk) + M[7];
        float pz = ((M[8] * xk + M[9] * yk) + M[10] * zk) + M[11];
        if (pz > z_near) {
          float mx = tc->fx * (px / pz) + tc->cx;
          float my = tc->fy * (py / pz) + tc->cy;
          float Dt;
          if (depth_bilinear(tgt_depth[t], tc->width, tc->height, mx, my, &Dt))
            v = fabsf(pz - Dt) <= rel_tol * Dt;
        }
      }
      vis[(int64_t)t * P + p] = v;
      cnt += v;
    }
    if (counts) counts[t] = cnt;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* FP64 geometry of one Gaussian in one view (values and gradients)         */
/* ------------------------------------------------------------------------ */

typedef struct {
  double p[3];       /* camera-frame centre */
  double mu[2];      /* projected mean */
  double J[2][3];    /* d mu / d p */
  double dJ[3][2][3];/* d J / d p_k */
  double Q[2][2];    /* inverse of Sigma_2D */
  double r;
  double z;          /* depth composited into D' */
} geo64;

static void mat34_mul(const double *A, const double *B, double *C) {
  /* C = A * B for 3x4 rigid transforms (implicit last row 0 0 0 1) */
  for (int i = 0; i < 3; i++) {
    for (int j = 0; j < 4; j++) {
      double s = 0;
      for (int k = 0; k < 3; k++) s += A[4 * i + k] * B[4 * k + j];
      if (j == 3) s += A[4 * i + 3];
      C[4 * i + j] = s;
    }
  }
}

static void rigid_inv(const double *T, double *I) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) I[4 * i + j] = T[4 * j + i];
  for (int i = 0; i < 3; i++)
    I[4 * i + 3] = -(I[4 * i + 0] * T[3] + I[4 * i + 1] * T[7] + I[4 * i + 2] * T[11]);
}

static void view_pose64(const orc_view *v, const orc_values *val, double *Tv) {
  double T0[12];
  for (int i = 0; i < 12; i++) T0[i] = v->pose[i];
  if (val) {
    double E[12];
    orc_se3_exp(val->twist, E);
    mat34_mul(E, T0, Tv);
  } else {
    memcpy(Tv, T0, sizeof(T0));
  }
}

/* M = T_v T_k^-1 of slice keyframe sidx in FP64, with the view's and the
 * keyframe's twists of `val` applied (left: pose <- exp(twist^) pose). */
static void slice_M(const orc_view *v, const orc_kf *kfs, const orc_values *val, int32_t sidx,
                    double *M) {
  const orc_kf *k = &kfs[v->kf_first + sidx];
  double Tv[12], T0[12], Tk[12], Tki[12];
  view_pose64(v, val, Tv);
  for (int i = 0; i < 12; i++) T0[i] = k->pose[i];
  if (val && val->kf_twist) {
    double E[12];
    orc_se3_exp(val->kf_twist + 6 * sidx, E);
    mat34_mul(E, T0, Tk);
  } else {
    memcpy(Tk, T0, sizeof(T0));
  }
  rigid_inv(Tk, Tki);
  mat34_mul(Tv, Tki, M);
}

static void geo_of(const double *M, const orc_cam *kc, const orc_cam *vc, uint32_t pix, double d,
                   double r, double lowpass, geo64 *g) {
  int32_t u = (int32_t)(pix % (uint32_t)kc->width), v = (int32_t)(pix / (uint32_t)kc->width);
  double X[3] = {(u - (double)kc->cx) / kc->fx * d, (v - (double)kc->cy) / kc->fy * d, d};
  for (int i = 0; i < 3; i++)
    g->p[i] = M[4 * i] * X[0] + M[4 * i + 1] * X[1] + M[4 * i + 2] * X[2] + M[4 * i + 3];
  double fx = vc->fx, fy = vc->fy, x = g->p[0], y = g->p[1], z = g->p[2];
  g->mu[0] = fx * x / z + vc->cx;
  g->mu[1] = fy * y / z + vc->cy;
  double J[2][3] = {{fx / z, 0, -fx * x / (z * z)}, {0, fy / z, -fy * y / (z * z)}};
  memcpy(g->J, J, sizeof(J));
  memset(g->dJ, 0, sizeof(g->dJ));
  g->dJ[0][0][2] = -fx / (z * z);
  g->dJ[1][1][2] = -fy / (z * z);
  g->dJ[2][0][0] = -fx / (z * z);
  g->dJ[2][0][2] = 2 * fx * x / (z * z * z);
  g->dJ[2][1][1] = -fy / (z * z);
  g->dJ[2][1][2] = 2 * fy * y / (z * z * z);
  double S[2][2];
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) {
      double s = 0;
      for (int k = 0; k < 3; k++) s += J[i][k] * J[j][k];
      S[i][j] = r * r * s + (i == j ? lowpass : 0.0);
    }
  double det = S[0][0] * S[1][1] - S[0][1] * S[1][0];
  g->Q[0][0] = S[1][1] / det;
  g->Q[1][1] = S[0][0] / det;
  g->Q[0][1] = g->Q[1][0] = -S[0][1] / det;
  g->r = r;
  g->z = z;
}

/* q, and the pieces of its derivative, at pixel (u, v) */
static double q_at(const geo64 *g, double u, double v, double *w) {
  double d0 = u - g->mu[0], d1 = v - g->mu[1];
  w[0] = g->Q[0][0] * d0 + g->Q[0][1] * d1;
  w[1] = g->Q[1][0] * d0 + g->Q[1][1] * d1;
  return d0 * w[0] + d1 * w[1];
}

/* dq/dr and dq/dp: q = d^T Sigma^-1 d, d = pixel - mu(p),
 * Sigma = r^2 J J^T + s I.  With w = Sigma^-1 d and t = J^T w:
 *   dq/dr   = -2 r |t|^2
 *   dq/dp_k = -2 t_k - 2 r^2 (dJ_k^T w) . t                            */
static void dq_of(const geo64 *g, const double *w, double *dq_dr, double *dq_dp) {
  double t[3];
  for (int k = 0; k < 3; k++) t[k] = g->J[0][k] * w[0] + g->J[1][k] * w[1];
  *dq_dr = -2.0 * g->r * (t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  for (int k = 0; k < 3; k++) {
    double e = 0;
    for (int m = 0; m < 3; m++) e += (g->dJ[k][0][m] * w[0] + g->dJ[k][1][m] * w[1]) * t[m];
    dq_dp[k] = -2.0 * t[k] - 2.0 * g->r * g->r * e;
  }
}

/* ------------------------------------------------------------------------ */
/* shared setup of a render: FP32 records, FP64 geometry, slice lookup       */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t N;
  orc_rec *rec;        /* FP32 decisions */
  geo64 *geo;          /* FP64 values    */
  double *col, *opa;   /* FP64 colour [3][N], opacity [N] */
} scene_t;

static void scene_free(scene_t *s) {
  free(s->rec); free(s->geo); free(s->col); free(s->opa);
}

static int scene_build(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                       const orc_values *val, scene_t *s) {
  int32_t N = orc_slice_size(v, kfs);
  s->N = N;
  size_t n1 = (size_t)(N > 0 ? N : 1);
  s->rec = (orc_rec *)malloc(sizeof(orc_rec) * n1);
  s->geo = (geo64 *)malloc(sizeof(geo64) * n1);
  s->col = (double *)malloc(sizeof(double) * 3 * n1);
  s->opa = (double *)malloc(sizeof(double) * n1);
  if (!s->rec || !s->geo || !s->col || !s->opa) { scene_free(s); return -1; }
  orc_preprocess32(v, kfs, prm, s->rec);
  int32_t id = 0;
  for (int32_t sidx = 0; sidx < v->kf_count; sidx++) {
    const orc_kf *k = &kfs[v->kf_first + sidx];
    double M[12];
    slice_M(v, kfs, val, sidx, M);
    for (int32_t i = 0; i < k->n; i++, id++) {
      double r = (val && val->radius) ? val->radius[id] : k->radius[i];
      double d = (val && val->depth) ? val->depth[id] : k->depth[i];
      geo_of(M, &k->cam, &v->cam, k->pix[i], d, r, prm->lowpass, &s->geo[id]);
      if (!(val && val->geometry64) && s->rec[id].count > 0) {
        /* composite the pinned FP32 record: mean, conic, depth */
        const orc_rec *rc = &s->rec[id];
        geo64 *g = &s->geo[id];
        g->mu[0] = rc->mx;
        g->mu[1] = rc->my;
        g->Q[0][0] = rc->qa;
        g->Q[0][1] = g->Q[1][0] = rc->qb;
        g->Q[1][1] = rc->qc;
        g->z = rc->pz;
      }
      for (int c = 0; c < 3; c++)
        s->col[(size_t)c * N + id] = (val && val->color) ? val->color[(size_t)c * N + id]
                                                          : k->color[(int64_t)c * k->n + i];
      s->opa[id] = (val && val->opacity) ? val->opacity[id] : k->opacity[i];
    }
  }
  return 0;
}

static float opa32(const orc_view *v, const orc_kf *kfs, int32_t id) {
  for (int32_t s = 0; s < v->kf_count; s++) {
    const orc_kf *k = &kfs[v->kf_first + s];
    if (id < k->n) return k->opacity[id];
    id -= k->n;
  }
  return 0.f;
}

/* One candidate entry of a pixel's list. */
typedef struct { uint32_t zb; int32_t id; uint8_t clamped; } ent;

static int cmp_ent(const void *a, const void *b) {
  const ent *x = (const ent *)a, *y = (const ent *)b;
  if (x->zb != y->zb) return x->zb < y->zb ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

static int near_rel(float x, float thr, float margin) {
  return fabsf(x - thr) <= margin * fabsf(thr);
}

/* Kinds of near-tie a test reports in its flag byte. */
enum { MARG_CAND = 1, MARG_CLAMP = 2, MARG_STOP = 4 };

/* FP32 per-(pixel, Gaussian) test: q <= Q_CUT and alpha >= alpha_min.
 * Returns 1 if the Gaussian is a candidate.  ORs MARG_CAND into *marg when
 * the candidate decision is a near-tie: q within `margin` (relative) of
 * Q_CUT while the alpha test passes or ties, or alpha within `margin` of
 * alpha_min while the q test passes or ties; with flip != 0 the tied tests
 * are taken the other way.  ORs MARG_CLAMP when the alpha_max clamp ties
 * (which moves alpha by at most `margin`, not the candidate set). */
static int test32(const orc_rec *r, float o, int32_t u, int32_t v, const orc_params *prm,
                  float margin, int flip, uint8_t *clamped, uint8_t *marg) {
  float dx = (float)u - r->mx, dy = (float)v - r->my;
  /* pinned order: q = fma(qc*dy, dy, fma(2qb*dx, dy, (qa*dx)*dx)) */
  float q = (r->qa * dx) * dx;
  q = fmaf((2.0f * r->qb) * dx, dy, q);
  q = fmaf(r->qc * dy, dy, q);
  float a = o * expf(-0.5f * q);
  /* G <= 1, so the clamp can only engage (and tie) when o > alpha_max */
  if (o > prm->alpha_max && near_rel(a, prm->alpha_max, margin)) *marg |= MARG_CLAMP;
  *clamped = a > prm->alpha_max;
  if (*clamped) a = prm->alpha_max;
  int pq = q <= prm->q_cut, pa = a >= prm->alpha_min;
  int tq = near_rel(q, prm->q_cut, margin), ta = near_rel(a, prm->alpha_min, margin);
  if ((tq && (pa || ta)) || (ta && (pq || tq))) {
    *marg |= MARG_CAND;
    if (flip) {
      if (tq) pq = !pq;
      if (ta) pa = !pa;
    }
  }
  return pq && pa;
}

static float alpha32(const orc_rec *r, float o, int32_t u, int32_t v, const orc_params *prm) {
  float dx = (float)u - r->mx, dy = (float)v - r->my;
  float q = (r->qa * dx) * dx;
  q = fmaf((2.0f * r->qb) * dx, dy, q);
  q = fmaf(r->qc * dy, dy, q);
  float a = o * expf(-0.5f * q);
  return a > prm->alpha_max ? prm->alpha_max : a;
}

/* Candidate lists for every pixel of the view (CSR, sorted by depth then id). */
typedef struct {
  int64_t *off;   /* [P+1] */
  ent *e;
  uint8_t *marg;  /* [P] */
  int64_t superset_violations;
} lists_t;

static void lists_free(lists_t *L) { free(L->off); free(L->e); free(L->marg); }

static int lists_build(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                       const scene_t *s, float margin, lists_t *L) {
  int32_t W = v->cam.width, H = v->cam.height;
  int64_t P = (int64_t)W * H;
  L->off = (int64_t *)calloc((size_t)P + 1, sizeof(int64_t));
  L->marg = (uint8_t *)calloc((size_t)(P > 0 ? P : 1), 1);
  L->superset_violations = 0;
  L->e = NULL;
  if (!L->off || !L->marg) return -1;
  for (int pass = 0; pass < 2; pass++) {
    int64_t *fill = NULL;
    if (pass == 1) {
      for (int64_t p = 0; p < P; p++) L->off[p + 1] += L->off[p];
      L->e = (ent *)malloc(sizeof(ent) * (size_t)(L->off[P] > 0 ? L->off[P] : 1));
      fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(P > 0 ? P : 1));
      if (!L->e || !fill) { free(fill); return -1; }
      for (int64_t p = 0; p < P; p++) fill[p] = L->off[p];
    }
    /* (threads claim list slots with atomics; each pixel's list is sorted by
     * its unique (depth, id) keys below, so the order of claims is immaterial) */
    int64_t viol = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : viol)
#endif
    for (int32_t g = 0; g < s->N; g++) {
      const orc_rec *r = &s->rec[g];
      if (!r->count) continue;
      float o = opa32(v, kfs, g);
      /* scan the box mu +- (R + 2): pixels beyond mu +- R must fail q <= Q_CUT */
      int32_t x0 = (int32_t)floorf(r->mx - r->ext) - 2, x1 = (int32_t)ceilf(r->mx + r->ext) + 2;
      int32_t y0 = (int32_t)floorf(r->my - r->ext) - 2, y1 = (int32_t)ceilf(r->my + r->ext) + 2;
      if (x0 < 0) x0 = 0;
      if (y0 < 0) y0 = 0;
      if (x1 > W - 1) x1 = W - 1;
      if (y1 > H - 1) y1 = H - 1;
      for (int32_t y = y0; y <= y1; y++)
        for (int32_t x = x0; x <= x1; x++) {
          uint8_t cl = 0, mg = 0;
          int ok = test32(r, o, x, y, prm, margin, 0, &cl, &mg);
          int64_t p = (int64_t)y * W + x;
          if (pass == 0) {
            L->marg[p] |= mg;
            if (ok) {
#ifdef _OPENMP
#pragma omp atomic
#endif
              L->off[p + 1]++;
              if (fabsf((float)x - r->mx) > r->ext || fabsf((float)y - r->my) > r->ext) viol++;
            }
          } else if (ok) {
            int64_t slot;
#ifdef _OPENMP
#pragma omp atomic capture
#endif
            slot = fill[p]++;
            ent *e = &L->e[slot];
            e->zb = fbits(r->pz);
            e->id = g;
            e->clamped = cl;
          }
        }
    }
    if (pass == 0) L->superset_violations = viol;
    free(fill);
  }
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1024)
#endif
  for (int64_t p = 0; p < P; p++)
    qsort(L->e + L->off[p], (size_t)(L->off[p + 1] - L->off[p]), sizeof(ent), cmp_ent);
  return 0;
}

/* Candidate list of one pixel by brute force over every Gaussian. */
static int64_t pixel_list(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                          const scene_t *s, float margin, int32_t x, int32_t y, ent *out,
                          uint8_t *marg) {
  int64_t n = 0;
  for (int32_t g = 0; g < s->N; g++) {
    const orc_rec *r = &s->rec[g];
    if (!r->count) continue;
    uint8_t cl = 0;
    if (test32(r, opa32(v, kfs, g), x, y, prm, margin, 0, &cl, marg)) {
      out[n].zb = fbits(r->pz);
      out[n].id = g;
      out[n].clamped = cl;
      n++;
    }
  }
  qsort(out, (size_t)n, sizeof(ent), cmp_ent);
  return n;
}

/* Front-to-back compositing of one pixel.  FP32 transmittance decides when
 * to stop; colour, depth and transmittance values are accumulated in FP64.
 * Returns the number of contributors.  With nd != NULL the near-tie stop
 * decisions are numbered from *nd on (which is advanced) and the one
 * numbered `flip` is taken the other way (flip < 0: none). */
static int32_t composite(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                         const scene_t *s, float margin, int32_t x, int32_t y, const ent *e,
                         int64_t n, double *C, double *D, double *T_out, uint8_t *marg,
                         int32_t flip, int32_t *nd) {
  float T32 = 1.0f;
  double T = 1.0;
  /* Relative uncertainty of T32 against an evaluation whose exp differs by
   * at most `margin` (relative): an alpha error of margin*alpha becomes a
   * relative error margin*alpha/(1-alpha) of (1 - alpha), plus one rounding
   * per product.  A stop decision closer to t_min than that is marginal. */
  double u = 0.0;
  C[0] = C[1] = C[2] = 0.0;
  *D = 0.0;
  int32_t k = 0;
  for (int64_t i = 0; i < n; i++) {
    int32_t g = e[i].id;
    const orc_rec *r = &s->rec[g];
    float a32 = alpha32(r, opa32(v, kfs, g), x, y, prm);
    float Tn = T32 * (1.0f - a32);
    double un = u + (double)margin * a32 / (1.0 - a32) + (margin > 0.f ? 1.2e-7 : 0.0);
    int stop = Tn < prm->t_min;
    if (fabs((double)Tn - prm->t_min) <= un * prm->t_min) {
      *marg |= MARG_STOP;
      if (nd) {
        if (*nd == flip) stop = !stop;
        (*nd)++;
      }
    }
    if (stop) break;
    double w[2];
    double q = q_at(&s->geo[g], x, y, w);
    double a = e[i].clamped ? (double)prm->alpha_max : s->opa[g] * exp(-0.5 * q);
    for (int c = 0; c < 3; c++) C[c] += s->col[(size_t)c * s->N + g] * a * T;
    *D += s->geo[g].z * a * T;
    T *= (1.0 - a);
    T32 = Tn;
    u = un;
    k++;
  }
  for (int c = 0; c < 3; c++) C[c] += T * prm->bg[c];
  *T_out = T;
  return k;
}

int orc_render_fwd(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                   const orc_values *val, float margin, int32_t n_px, const int32_t *px_idx,
                   double *rgb, double *depth, double *sil, double *t_final,
                   int32_t *n_contrib, uint8_t *marginal) {
  scene_t s;
  if (scene_build(v, kfs, prm, val, &s)) return -1;
  int32_t W = v->cam.width;
  int64_t P = n_px < 0 ? (int64_t)W * v->cam.height : n_px;
  int rc = 0;
  if (n_px < 0) {
    lists_t L;
    if (lists_build(v, kfs, prm, &s, margin, &L)) { lists_free(&L); scene_free(&s); return -1; }
    rc = L.superset_violations ? 1 : 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256)
#endif
    for (int64_t p = 0; p < P; p++) {
      double C[3], D, T;
      uint8_t mg = L.marg[p];
      int32_t k = composite(v, kfs, prm, &s, margin, (int32_t)(p % W), (int32_t)(p / W),
                            L.e + L.off[p], L.off[p + 1] - L.off[p], C, &D, &T, &mg, -1, NULL);
      for (int c = 0; c < 3; c++) rgb[c * P + p] = C[c];
      depth[p] = D;
      sil[p] = 1.0 - T;
      if (t_final) t_final[p] = T;
      if (n_contrib) n_contrib[p] = k;
      if (marginal) marginal[p] = mg;
    }
    lists_free(&L);
  } else {
    ent *buf = (ent *)malloc(sizeof(ent) * (size_t)(s.N > 0 ? s.N : 1));
    for (int64_t i = 0; i < P; i++) {
      int32_t p = px_idx[i];
      int32_t x = p % W, y = p / W;
      uint8_t mg = 0;
      int64_t n = pixel_list(v, kfs, prm, &s, margin, x, y, buf, &mg);
      double C[3], D, T;
      int32_t k = composite(v, kfs, prm, &s, margin, x, y, buf, n, C, &D, &T, &mg, -1, NULL);
      for (int c = 0; c < 3; c++) rgb[c * P + i] = C[c];
      depth[i] = D;
      sil[i] = 1.0 - T;
      if (t_final) t_final[i] = T;
      if (n_contrib) n_contrib[i] = k;
      if (marginal) marginal[i] = mg;
    }
    free(buf);
  }
  scene_free(&s);
  return rc;
}

/* The other outcomes of a pixel's near-tie decisions.  A decision within
 * `margin` of its threshold (a candidate test, or a stop) may legitimately
 * go either way in an evaluation whose exp differs by that much; the pixel's
 * near-tie decisions are numbered as they are met -- candidate tests in
 * slice order, then stop decisions front to back -- and variant j is the
 * pixel with decision j taken the other way and every later decision taken
 * by the FP32 tests.  Only the Gaussians whose scan box (mu +- (R + 2))
 * holds the pixel are tested: beyond it q exceeds Q_CUT by a wide margin. */
int orc_render_alt(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                   const orc_values *val, float margin, int32_t n_px, const int32_t *px_idx,
                   int32_t max_alt, double *rgb, double *depth, double *sil, int32_t *n_dec) {
  scene_t s;
  if (scene_build(v, kfs, prm, val, &s)) return -1;
  int32_t W = v->cam.width, H = v->cam.height;
  int64_t P = (int64_t)W * H;
  /* request index of every pixel (-1: not requested) */
  int32_t *req = (int32_t *)malloc(sizeof(int32_t) * (size_t)(P > 0 ? P : 1));
  int64_t *off = (int64_t *)calloc((size_t)n_px + 1, sizeof(int64_t));
  if (!req || !off) { free(req); free(off); scene_free(&s); return -1; }
  for (int64_t p = 0; p < P; p++) req[p] = -1;
  for (int32_t i = 0; i < n_px; i++) req[px_idx[i]] = i;
  int32_t *near = NULL;
  int64_t *fill = NULL;
  /* two passes over the Gaussians in slice order: count, then fill, so each
   * pixel's Gaussians are listed in ascending local id */
  for (int pass = 0; pass < 2; pass++) {
    if (pass == 1) {
      for (int32_t i = 0; i < n_px; i++) off[i + 1] += off[i];
      near = (int32_t *)malloc(sizeof(int32_t) * (size_t)(off[n_px] > 0 ? off[n_px] : 1));
      fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_px > 0 ? n_px : 1));
      if (!near || !fill) { free(near); free(fill); free(req); free(off); scene_free(&s); return -1; }
      for (int32_t i = 0; i < n_px; i++) fill[i] = off[i];
    }
    for (int32_t g = 0; g < s.N; g++) {
      const orc_rec *r = &s.rec[g];
      if (!r->count) continue;
      int32_t x0 = (int32_t)floorf(r->mx - r->ext) - 2, x1 = (int32_t)ceilf(r->mx + r->ext) + 2;
      int32_t y0 = (int32_t)floorf(r->my - r->ext) - 2, y1 = (int32_t)ceilf(r->my + r->ext) + 2;
      if (x0 < 0) x0 = 0;
      if (y0 < 0) y0 = 0;
      if (x1 > W - 1) x1 = W - 1;
      if (y1 > H - 1) y1 = H - 1;
      for (int32_t y = y0; y <= y1; y++)
        for (int32_t x = x0; x <= x1; x++) {
          int32_t i = req[(int64_t)y * W + x];
          if (i < 0) continue;
          if (pass == 0) off[i + 1]++;
          else near[fill[i]++] = g;
        }
    }
  }
  free(fill);
  ent *buf = (ent *)malloc(sizeof(ent) * (size_t)(s.N > 0 ? s.N : 1));
  if (!buf) { free(near); free(req); free(off); scene_free(&s); return -1; }
  for (int32_t i = 0; i < n_px; i++) {
    int32_t x = px_idx[i] % W, y = px_idx[i] / W;
    int32_t total = 0;
    for (int32_t flip = -1; flip < (total < max_alt ? total : max_alt); flip++) {
      int32_t nd = 0;
      int64_t n = 0;
      for (int64_t j = off[i]; j < off[i + 1]; j++) {
        int32_t g = near[j];
        const orc_rec *r = &s.rec[g];
        uint8_t cl = 0, mg = 0;
        float o = opa32(v, kfs, g);
        int ok = test32(r, o, x, y, prm, margin, 0, &cl, &mg);
        if (mg & MARG_CAND) {
          if (nd == flip) ok = test32(r, o, x, y, prm, margin, 1, &cl, &mg);
          nd++;
        }
        if (ok) {
          buf[n].zb = fbits(r->pz);
          buf[n].id = g;
          buf[n].clamped = cl;
          n++;
        }
      }
      qsort(buf, (size_t)n, sizeof(ent), cmp_ent);
      double C[3], D, T;
      uint8_t mg = 0;
      composite(v, kfs, prm, &s, margin, x, y, buf, n, C, &D, &T, &mg, flip, &nd);
      if (flip < 0) {
        total = nd;
        n_dec[i] = nd;
        continue;
      }
      size_t o = (size_t)i * (size_t)max_alt + (size_t)flip;
      for (int c = 0; c < 3; c++) rgb[3 * o + c] = C[c];
      depth[o] = D;
      sil[o] = 1.0 - T;
    }
  }
  free(buf); free(near); free(req); free(off);
  scene_free(&s);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* backward: derivative of C = sum c_i a_i T_i + bg T_N, D = sum z_i a_i T_i, */
/* S = 1 - T_N, with T_i = prod_{j<i} (1 - a_j), contributor sets fixed.     */
/* ------------------------------------------------------------------------ */

/* Per-thread partial sums of the backward: the pixels of a contiguous range
 * of rows add their terms here; the ranges are reduced in row order. */
typedef struct {
  double *g_color, *g_opac, *g_rad, *g_p, *mag, *mag_p;
} bwd_acc;

static int bwd_acc_init(bwd_acc *b, int32_t N, int want_mag) {
  size_t n1 = (size_t)(N > 0 ? N : 1);
  memset(b, 0, sizeof(*b));
  b->g_color = (double *)calloc(3 * n1, sizeof(double));
  b->g_opac = (double *)calloc(n1, sizeof(double));
  b->g_rad = (double *)calloc(n1, sizeof(double));
  b->g_p = (double *)calloc(3 * n1, sizeof(double));
  if (want_mag) {
    b->mag = (double *)calloc(5 * n1, sizeof(double));
    b->mag_p = (double *)calloc(3 * n1, sizeof(double));
  }
  return b->g_color && b->g_opac && b->g_rad && b->g_p && (!want_mag || (b->mag && b->mag_p)) ? 0 : -1;
}

static void bwd_acc_free(bwd_acc *b) {
  free(b->g_color); free(b->g_opac); free(b->g_rad); free(b->g_p); free(b->mag); free(b->mag_p);
}

/* The backward terms of the pixels [p0, p1). */
static void bwd_pixels(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                       const scene_t *sp, const lists_t *Lp, int64_t p0, int64_t p1, int64_t maxn,
                       const double *g_rgb, const double *g_depth, const double *g_sil,
                       bwd_acc *acc) {
  const scene_t s = *sp;
  const lists_t L = *Lp;
  int32_t N = s.N, W = v->cam.width;
  int64_t P = (int64_t)W * v->cam.height;
  double *g_color = acc->g_color, *g_opac = acc->g_opac, *g_rad = acc->g_rad, *g_p = acc->g_p;
  double *g_mag = acc->mag, *mag_p = acc->mag_p;
  double *a = (double *)malloc(sizeof(double) * (size_t)(maxn + 1));
  double *G = (double *)malloc(sizeof(double) * (size_t)(maxn + 1));
  double *T = (double *)malloc(sizeof(double) * (size_t)(maxn + 2));
  double *qw = (double *)malloc(sizeof(double) * 2 * (size_t)(maxn + 1));
  for (int64_t p = p0; p < p1; p++) {
    int32_t x = (int32_t)(p % W), y = (int32_t)(p / W);
    const ent *e = L.e + L.off[p];
    int64_t n = L.off[p + 1] - L.off[p];
    /* contributor prefix by the FP32 transmittance rule */
    float T32 = 1.0f;
    int64_t k = 0;
    for (; k < n; k++) {
      float a32 = alpha32(&s.rec[e[k].id], opa32(v, kfs, e[k].id), x, y, prm);
      float Tn = T32 * (1.0f - a32);
      if (Tn < prm->t_min) break;
      T32 = Tn;
    }
    T[0] = 1.0;
    for (int64_t i = 0; i < k; i++) {
      int32_t g = e[i].id;
      double q = q_at(&s.geo[g], x, y, &qw[2 * i]);
      G[i] = exp(-0.5 * q);
      a[i] = e[i].clamped ? (double)prm->alpha_max : s.opa[g] * G[i];
      T[i + 1] = T[i] * (1.0 - a[i]);
    }
    double TN = T[k];
    double gC[3] = {g_rgb[p], g_rgb[P + p], g_rgb[2 * P + p]};
    double gD = g_depth ? g_depth[p] : 0.0, gS = g_sil ? g_sil[p] : 0.0;
    for (int64_t i = 0; i < k; i++) {
      int32_t g = e[i].id;
      double z = s.geo[g].z;
      /* contributions of everything behind i, summed directly */
      double behindC[3] = {prm->bg[0] * TN, prm->bg[1] * TN, prm->bg[2] * TN}, behindD = 0.0;
      for (int64_t j = i + 1; j < k; j++) {
        int32_t h = e[j].id;
        for (int c = 0; c < 3; c++) behindC[c] += s.col[(size_t)c * N + h] * a[j] * T[j];
        behindD += s.geo[h].z * a[j] * T[j];
      }
      double inv = 1.0 / (1.0 - a[i]);
      double dL_da = 0.0;
      for (int c = 0; c < 3; c++)
        dL_da += gC[c] * (s.col[(size_t)c * N + g] * T[i] - behindC[c] * inv);
      dL_da += gD * (z * T[i] - behindD * inv);
      dL_da += gS * (TN * inv);
      for (int c = 0; c < 3; c++) g_color[(size_t)c * N + g] += a[i] * T[i] * gC[c];
      double dL_dz = a[i] * T[i] * gD;
      double dL_dq = 0.0;
      if (!e[i].clamped) {
        g_opac[g] += G[i] * dL_da;
        dL_dq = dL_da * s.opa[g] * G[i] * (-0.5);
      }
      double dq_dr, dq_dp[3];
      dq_of(&s.geo[g], &qw[2 * i], &dq_dr, dq_dp);
      g_rad[g] += dL_dq * dq_dr;
      for (int m = 0; m < 3; m++) g_p[3 * g + m] += dL_dq * dq_dp[m];
      g_p[3 * g + 2] += dL_dz;
      if (g_mag) {
        /* the same terms with every summand replaced by its absolute value:
         * the scale against which a rounded evaluation of the sums is judged */
        double m_da = 0.0;
        for (int c = 0; c < 3; c++)
          m_da += fabs(gC[c]) * (fabs(s.col[(size_t)c * N + g]) * T[i] + fabs(behindC[c]) * inv);
        m_da += fabs(gD) * (fabs(z) * T[i] + fabs(behindD) * inv);
        m_da += fabs(gS) * (TN * inv);
        for (int c = 0; c < 3; c++) g_mag[(size_t)c * N + g] += fabs(a[i] * T[i] * gC[c]);
        double m_dq = 0.0;
        if (!e[i].clamped) {
          g_mag[3 * (size_t)N + g] += G[i] * m_da;
          m_dq = m_da * s.opa[g] * G[i] * 0.5;
        }
        g_mag[4 * (size_t)N + g] += m_dq * fabs(dq_dr);
        for (int m = 0; m < 3; m++) mag_p[3 * g + m] += m_dq * fabs(dq_dp[m]);
        mag_p[3 * g + 2] += fabs(dL_dz);
      }
    }
  }
  free(a); free(G); free(T); free(qw);
}

int orc_render_bwd(const orc_view *v, const orc_kf *kfs, const orc_params *prm,
                   const orc_values *val, const double *g_rgb, const double *g_depth,
                   const double *g_sil, double *g_color, double *g_opac, double *g_rad,
                   double *g_twist, double *g_mag, double *g_kdepth, double *g_kpose,
                   double *g_kmag) {
  scene_t s;
  if (scene_build(v, kfs, prm, val, &s)) return -1;
  lists_t L;
  if (lists_build(v, kfs, prm, &s, 0.f, &L)) { lists_free(&L); scene_free(&s); return -1; }
  int32_t N = s.N, W = v->cam.width, H = v->cam.height;
  int64_t P = (int64_t)W * H;
  int64_t maxn = 0;
  for (int64_t p = 0; p < P; p++)
    if (L.off[p + 1] - L.off[p] > maxn) maxn = L.off[p + 1] - L.off[p];
  /* rows split into one contiguous range per thread (one range without
   * OpenMP); every range sums into its own buffers */
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
  if (nt > H) nt = H > 0 ? H : 1;
#endif
  bwd_acc *acc = (bwd_acc *)calloc((size_t)nt, sizeof(bwd_acc));
  int bad = acc == NULL;
  for (int t = 0; t < nt && !bad; t++) bad |= bwd_acc_init(&acc[t], N, g_mag != NULL);
  if (bad) {
    if (acc) for (int t = 0; t < nt; t++) bwd_acc_free(&acc[t]);
    free(acc); lists_free(&L); scene_free(&s);
    return -1;
  }
#ifdef _OPENMP
#pragma omp parallel for num_threads(nt) schedule(static, 1)
#endif
  for (int t = 0; t < nt; t++) {
    int64_t r0 = (int64_t)H * t / nt, r1 = (int64_t)H * (t + 1) / nt;
    bwd_pixels(v, kfs, prm, &s, &L, r0 * W, r1 * W, maxn, g_rgb, g_depth, g_sil, &acc[t]);
  }
  /* reduction in row order */
  memset(g_color, 0, sizeof(double) * 3 * (size_t)N);
  memset(g_opac, 0, sizeof(double) * (size_t)N);
  memset(g_rad, 0, sizeof(double) * (size_t)N);
  double *g_p = (double *)calloc((size_t)(N > 0 ? N : 1) * 3, sizeof(double));
  double *mag_p = NULL;
  if (g_mag) {
    memset(g_mag, 0, sizeof(double) * (5 * (size_t)N + 6));
    mag_p = (double *)calloc((size_t)(N > 0 ? N : 1) * 3, sizeof(double));
  }
  for (int t = 0; t < nt; t++) {
    for (size_t i = 0; i < 3 * (size_t)N; i++) { g_color[i] += acc[t].g_color[i]; g_p[i] += acc[t].g_p[i]; }
    for (size_t i = 0; i < (size_t)N; i++) { g_opac[i] += acc[t].g_opac[i]; g_rad[i] += acc[t].g_rad[i]; }
    if (g_mag) {
      for (size_t i = 0; i < 5 * (size_t)N; i++) g_mag[i] += acc[t].mag[i];
      for (size_t i = 0; i < 3 * (size_t)N; i++) mag_p[i] += acc[t].mag_p[i];
    }
    bwd_acc_free(&acc[t]);
  }
  free(acc);
  /* twist (rho, phi) of the left perturbation: dp/drho = I, dp/dphi = -[p]x */
  for (int m = 0; m < 6; m++) g_twist[m] = 0.0;
  for (int32_t g = 0; g < N; g++) {
    const double *pp = s.geo[g].p, *gp = &g_p[3 * g];
    g_twist[0] += gp[0];
    g_twist[1] += gp[1];
    g_twist[2] += gp[2];
    g_twist[3] += pp[1] * gp[2] - pp[2] * gp[1];
    g_twist[4] += pp[2] * gp[0] - pp[0] * gp[2];
    g_twist[5] += pp[0] * gp[1] - pp[1] * gp[0];
    if (g_mag) {
      const double *mp = &mag_p[3 * g];
      double *mt = g_mag + 5 * (size_t)N;
      mt[0] += mp[0];
      mt[1] += mp[1];
      mt[2] += mp[2];
      mt[3] += fabs(pp[1]) * mp[2] + fabs(pp[2]) * mp[1];
      mt[4] += fabs(pp[2]) * mp[0] + fabs(pp[0]) * mp[2];
      mt[5] += fabs(pp[0]) * mp[1] + fabs(pp[1]) * mp[0];
    }
  }
  /* the keyframe side of the centres: X = d n in the keyframe camera, n the
   * pixel's ray (z = 1), p = R X + t with (R, t) = T_v T_k^-1.  With
   * h = R^T dL/dp:  dL/dd = h . n;  a left twist of T_k moves X to
   * exp(-twist^) X, so dL/drho_k = -sum h and dL/dphi_k = -sum X x h. */
  if (g_kdepth || g_kpose) {
    int32_t id = 0;
    for (int32_t sidx = 0; sidx < v->kf_count; sidx++) {
      const orc_kf *k = &kfs[v->kf_first + sidx];
      double M[12], G6[6] = {0, 0, 0, 0, 0, 0}, A6[6] = {0, 0, 0, 0, 0, 0};
      slice_M(v, kfs, val, sidx, M);
      for (int32_t i = 0; i < k->n; i++, id++) {
        const double *gp = &g_p[3 * id];
        double h[3], ha[3];
        for (int c = 0; c < 3; c++) h[c] = M[c] * gp[0] + M[4 + c] * gp[1] + M[8 + c] * gp[2];
        int32_t u = (int32_t)(k->pix[i] % (uint32_t)k->cam.width);
        int32_t w = (int32_t)(k->pix[i] / (uint32_t)k->cam.width);
        double n[3] = {(u - (double)k->cam.cx) / k->cam.fx, (w - (double)k->cam.cy) / k->cam.fy, 1.0};
        double d = (val && val->depth) ? val->depth[id] : k->depth[i];
        if (g_kdepth) g_kdepth[id] = h[0] * n[0] + h[1] * n[1] + h[2] * n[2];
        double X[3] = {d * n[0], d * n[1], d * n[2]};
        G6[0] -= h[0];
        G6[1] -= h[1];
        G6[2] -= h[2];
        G6[3] -= X[1] * h[2] - X[2] * h[1];
        G6[4] -= X[2] * h[0] - X[0] * h[2];
        G6[5] -= X[0] * h[1] - X[1] * h[0];
        if (g_kmag && mag_p) {
          /* the same with every summand in absolute value */
          const double *mp = &mag_p[3 * id];
          for (int c = 0; c < 3; c++)
            ha[c] = fabs(M[c]) * mp[0] + fabs(M[4 + c]) * mp[1] + fabs(M[8 + c]) * mp[2];
          g_kmag[id] = ha[0] * fabs(n[0]) + ha[1] * fabs(n[1]) + ha[2];
          A6[0] += ha[0];
          A6[1] += ha[1];
          A6[2] += ha[2];
          A6[3] += fabs(X[1]) * ha[2] + fabs(X[2]) * ha[1];
          A6[4] += fabs(X[2]) * ha[0] + fabs(X[0]) * ha[2];
          A6[5] += fabs(X[0]) * ha[1] + fabs(X[1]) * ha[0];
        }
      }
      if (g_kpose)
        for (int c = 0; c < 6; c++) g_kpose[6 * sidx + c] = G6[c];
      if (g_kmag && mag_p)
        for (int c = 0; c < 6; c++) g_kmag[(size_t)N + 6 * sidx + c] = A6[c];
    }
  }
  free(mag_p);
  free(g_p);
  lists_free(&L);
  scene_free(&s);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* losses                                                                   */
/* ------------------------------------------------------------------------ */

static double sgn(double x) { return (double)((x > 0) - (x < 0)); }

/* Eq. 1: alpha * sum W |V - V'| + beta * sum W |D - D'|, with
 * W = vis & (D > 0) & (S' > sil_thr) held fixed; gradients w.r.t. V', D'. */
double orc_track_loss(int32_t P, const double *rgb, const double *depth, const double *sil,
                      const float *obs_rgb, const float *obs_depth, const uint8_t *vis,
                      double alpha, double beta, double sil_thr,
                      double *g_rgb, double *g_depth) {
  double L = 0.0;
  for (int32_t p = 0; p < P; p++) {
    int w = (!vis || vis[p]) && obs_depth[p] > 0.f && sil[p] > sil_thr;
    for (int c = 0; c < 3; c++) {
      double r = (double)obs_rgb[(int64_t)c * P + p] - rgb[(int64_t)c * P + p];
      if (w) L += alpha * fabs(r);
      if (g_rgb) g_rgb[(int64_t)c * P + p] = w ? -alpha * sgn(r) : 0.0;
    }
    double rd = (double)obs_depth[p] - depth[p];
    if (w) L += beta * fabs(rd);
    if (g_depth) g_depth[p] = w ? -beta * sgn(rd) : 0.0;
  }
  return L;
}

/* SSIM with an 11x11 Gaussian window (sigma 1.5), zero padding, constants
 * C1 = 0.01^2, C2 = 0.03^2 (Wang et al.).  Returns the mean over pixels; if
 * g_x != NULL writes d mean / d x.  Direct 2-D window, no separation. */
double orc_ssim(int32_t H, int32_t W, const double *x, const double *y, double *g_x) {
  const int R = 5;
  const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
  double g1[11], s = 0;
  for (int i = -R; i <= R; i++) { g1[i + R] = exp(-(double)(i * i) / (2 * 1.5 * 1.5)); s += g1[i + R]; }
  double w[11][11];
  for (int i = 0; i < 11; i++)
    for (int j = 0; j < 11; j++) w[i][j] = g1[i] * g1[j] / (s * s);
  int64_t P = (int64_t)H * W;
  double *mx = (double *)malloc(sizeof(double) * (size_t)P);
  double *my = (double *)malloc(sizeof(double) * (size_t)P);
  double *dS_dmx = (double *)malloc(sizeof(double) * (size_t)P);
  double *dS_dvx = (double *)malloc(sizeof(double) * (size_t)P);
  double *dS_dcxy = (double *)malloc(sizeof(double) * (size_t)P);
  double total = 0.0;
  for (int32_t r = 0; r < H; r++)
    for (int32_t c = 0; c < W; c++) {
      double ux = 0, uy = 0, exx = 0, eyy = 0, exy = 0;
      for (int i = -R; i <= R; i++)
        for (int j = -R; j <= R; j++) {
          int32_t rr = r + i, cc = c + j;
          if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
          double wt = w[i + R][j + R], a = x[(int64_t)rr * W + cc], b = y[(int64_t)rr * W + cc];
          ux += wt * a; uy += wt * b; exx += wt * a * a; eyy += wt * b * b; exy += wt * a * b;
        }
      double vx = exx - ux * ux, vy = eyy - uy * uy, cxy = exy - ux * uy;
      double A1 = 2 * ux * uy + C1, A2 = 2 * cxy + C2;
      double B1 = ux * ux + uy * uy + C1, B2 = vx + vy + C2;
      double S = (A1 * A2) / (B1 * B2);
      total += S;
      int64_t p = (int64_t)r * W + c;
      mx[p] = ux; my[p] = uy;
      dS_dmx[p] = 2 * uy * A2 / (B1 * B2) - S * 2 * ux / B1;
      dS_dvx[p] = -S / B2;
      dS_dcxy[p] = 2 * A1 / (B1 * B2);
    }
  if (g_x) {
    /* dS(q)/dx(p) = w(q-p) [dS/dmu_x + 2 dS/dvar_x (x(p) - mu_x(q)) + dS/dcov (y(p) - mu_y(q))] */
    for (int64_t p = 0; p < P; p++) g_x[p] = 0.0;
    for (int32_t r = 0; r < H; r++)
      for (int32_t c = 0; c < W; c++) {
        int64_t q = (int64_t)r * W + c;
        for (int i = -R; i <= R; i++)
          for (int j = -R; j <= R; j++) {
            int32_t rr = r + i, cc = c + j;
            if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
            int64_t p = (int64_t)rr * W + cc;
            g_x[p] += w[i + R][j + R] *
                      (dS_dmx[q] + 2 * dS_dvx[q] * (x[p] - mx[q]) + dS_dcxy[q] * (y[p] - my[q]));
          }
      }
    for (int64_t p = 0; p < P; p++) g_x[p] /= (double)P;
  }
  free(mx); free(my); free(dS_dmx); free(dS_dvx); free(dS_dcxy);
  return total / (double)P;
}

/* Eq. 2: rho mean|V - V'| + tau (1 - SSIM(V, V')) + sigma mean(U |D - D'|),
 * U = (D > 0); SSIM averaged over the three channels. */
double orc_map_loss(int32_t H, int32_t W, const double *rgb, const double *depth,
                    const float *obs_rgb, const float *obs_depth,
                    double rho, double tau, double sigma, double *g_rgb, double *g_depth) {
  int64_t P = (int64_t)H * W;
  double l1 = 0.0, ld = 0.0, ss = 0.0;
  double *obs = (double *)malloc(sizeof(double) * (size_t)P);
  double *gs = (double *)malloc(sizeof(double) * (size_t)P);
  for (int c = 0; c < 3; c++) {
    for (int64_t p = 0; p < P; p++) obs[p] = obs_rgb[c * P + p];
    ss += orc_ssim(H, W, rgb + c * P, obs, g_rgb ? gs : NULL) / 3.0;
    for (int64_t p = 0; p < P; p++) {
      double r = obs[p] - rgb[c * P + p];
      l1 += fabs(r);
      if (g_rgb) g_rgb[c * P + p] = -rho * sgn(r) / (3.0 * P) - tau * gs[p] / 3.0;
    }
  }
  for (int64_t p = 0; p < P; p++) {
    int u = obs_depth[p] > 0.f;
    double r = (double)obs_depth[p] - depth[p];
    if (u) ld += fabs(r);
    if (g_depth) g_depth[p] = u ? -sigma * sgn(r) / (double)P : 0.0;
  }
  free(obs); free(gs);
  return rho * l1 / (3.0 * P) + tau * (1.0 - ss) + sigma * ld / (double)P;
}

/* ------------------------------------------------------------------------ */
/* optimiser pieces                                                         */
/* ------------------------------------------------------------------------ */

/* exp of a twist xi = (rho, phi) in se(3): R = exp([phi]x), t = V rho. */
void orc_se3_exp(const double *xi, double *T) {
  const double *rho = xi, *phi = xi + 3;
  double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2], th = sqrt(th2);
  double A, B, Cc;
  if (th < 1e-5) {
    A = 1 - th2 / 6;
    B = 0.5 - th2 / 24;
    Cc = 1.0 / 6 - th2 / 120;
  } else {
    A = sin(th) / th;
    B = (1 - cos(th)) / th2;
    Cc = (th - sin(th)) / (th2 * th);
  }
  double K[3][3] = {{0, -phi[2], phi[1]}, {phi[2], 0, -phi[0]}, {-phi[1], phi[0], 0}};
  double K2[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      K2[i][j] = 0;
      for (int k = 0; k < 3; k++) K2[i][j] += K[i][k] * K[k][j];
    }
  for (int i = 0; i < 3; i++) {
    double t = 0;
    for (int j = 0; j < 3; j++) {
      double I = i == j ? 1.0 : 0.0;
      T[4 * i + j] = I + A * K[i][j] + B * K2[i][j];
      t += (I + B * K[i][j] + Cc * K2[i][j]) * rho[j];
    }
    T[4 * i + 3] = t;
  }
}

void orc_adam(int64_t n, double *param, const double *grad, double *m, double *v,
              int64_t t, double lr, double b1, double b2, double eps) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int64_t i = 0; i < n; i++) {
    m[i] = b1 * m[i] + (1 - b1) * grad[i];
    v[i] = b2 * v[i] + (1 - b2) * grad[i] * grad[i];
    param[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}
