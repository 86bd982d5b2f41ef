/* Driver for the sanitizer build of the CPU oracle (test infrastructure).
 * Reads a keyframe (depth [H*W] f32, rgb [3*H*W] f32, pose [12] f32, camera
 * fx fy cx cy) and a view pose from the directory given as argv[1] and runs
 * every oracle entry point on it: ingestion, FP32 preprocessing, tile lists,
 * forward (full image and pixel mode), backward with gradient magnitudes,
 * Eq. 1, Eq. 2 with SSIM, the SE(3) exponential and Adam.  Built with
 * -fsanitize=address,undefined; any report fails the test. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

static void *load(const char *dir, const char *name, size_t bytes) {
  char path[4096];
  snprintf(path, sizeof(path), "%s/%s", dir, name);
  FILE *f = fopen(path, "rb");
  if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
  void *p = malloc(bytes);
  if (fread(p, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
  fclose(f);
  return p;
}

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  const char *dir = argv[1];
  int32_t *dims = (int32_t *)load(dir, "dims.bin", 8);
  int32_t H = dims[0], W = dims[1];
  int64_t P = (int64_t)H * W;
  float *depth = (float *)load(dir, "depth.bin", 4 * (size_t)P);
  float *rgb = (float *)load(dir, "rgb.bin", 12 * (size_t)P);
  float *kpose = (float *)load(dir, "kpose.bin", 48);
  float *vpose = (float *)load(dir, "vpose.bin", 48);
  float *intr = (float *)load(dir, "intr.bin", 16);
  orc_cam cam = {intr[0], intr[1], intr[2], intr[3], W, H};
  int32_t n = orc_ingest_count(depth, NULL, H, W, 1);
  uint32_t *pix = malloc(4 * (size_t)n);
  float *dep = malloc(4 * (size_t)n), *col = malloc(12 * (size_t)n);
  float *opa = malloc(4 * (size_t)n), *rad = malloc(4 * (size_t)n);
  if (orc_ingest_fill(depth, rgb, NULL, H, W, 1, cam.fx, 0.9f, n, pix, dep, col, opa, rad) != n) return 3;
  orc_kf kf = {n, pix, dep, col, opa, rad, kpose, cam};
  orc_view view = {cam, vpose, 0, 1};
  orc_params prm = {1.0f / 255.0f, 0.99f, 1e-4f, 11.0826f, 0.01f, 0.3f, {0.1f, 0.2f, 0.3f}, 16};
  float M[12];
  orc_relpose32(vpose, kpose, M);
  orc_rec *rec = malloc(sizeof(orc_rec) * (size_t)n);
  if (orc_preprocess32(&view, &kf, &prm, rec) != n) return 4;
  int32_t nt = ((W + 15) / 16) * ((H + 15) / 16);
  uint32_t *ranges = malloc(8 * (size_t)nt);
  int64_t K = orc_tile_lists(&view, &kf, &prm, NULL, NULL, ranges, 0);
  uint64_t *keys = malloc(8 * (size_t)(K + 1));
  uint32_t *vals = malloc(4 * (size_t)(K + 1));
  if (orc_tile_lists(&view, &kf, &prm, keys, vals, ranges, K) != K) return 5;
  double *img = malloc(sizeof(double) * 3 * (size_t)P), *dimg = malloc(sizeof(double) * (size_t)P);
  double *sil = malloc(sizeof(double) * (size_t)P), *tf = malloc(sizeof(double) * (size_t)P);
  int32_t *nc = malloc(4 * (size_t)P);
  uint8_t *mg = malloc((size_t)P);
  if (orc_render_fwd(&view, &kf, &prm, NULL, 2e-6f, -1, NULL, img, dimg, sil, tf, nc, mg) < 0) return 6;
  int32_t some[3] = {0, (int32_t)(P / 2), (int32_t)(P - 1)};
  double prgb[9], pd[3], ps[3], pt[3];
  int32_t pn[3];
  uint8_t pm[3];
  if (orc_render_fwd(&view, &kf, &prm, NULL, 2e-6f, 3, some, prgb, pd, ps, pt, pn, pm) < 0) return 7;
  /* near-tie alternatives of three pixels under a wide margin */
  double argb[3 * 3 * 4], adep[3 * 4], asil[3 * 4];
  int32_t andec[3];
  if (orc_render_alt(&view, &kf, &prm, NULL, 1e-2f, 3, some, 4, argb, adep, asil, andec) < 0) return 10;
  double *g_rgb = malloc(sizeof(double) * 3 * (size_t)P), *g_d = malloc(sizeof(double) * (size_t)P);
  double L1 = orc_track_loss((int32_t)P, img, dimg, sil, rgb, depth, NULL, 0.5, 1.0, 0.5, g_rgb, g_d);
  double *gc = malloc(sizeof(double) * 3 * (size_t)n), *go = malloc(sizeof(double) * (size_t)n);
  double *gr = malloc(sizeof(double) * (size_t)n), *mag = malloc(sizeof(double) * (5 * (size_t)n + 6));
  double tw[6];
  double *gkd = malloc(sizeof(double) * (size_t)n), gkp[6];
  if (orc_render_bwd(&view, &kf, &prm, NULL, g_rgb, g_d, sil, gc, go, gr, tw, mag, gkd, gkp, NULL) < 0) return 8;
  orc_values val = {NULL, NULL, NULL, {1e-3, -2e-3, 1e-3, 1e-3, 2e-3, -1e-3}, 1};
  if (orc_render_fwd(&view, &kf, &prm, &val, 0.f, -1, NULL, img, dimg, sil, tf, nc, mg) < 0) return 9;
  double L2 = orc_map_loss(H, W, img, dimg, rgb, depth, 0.8, 0.2, 1.0, g_rgb, g_d);
  double xi[6] = {0.1, -0.2, 0.3, 0.01, 0.02, -0.03}, T[12];
  orc_se3_exp(xi, T);
  double par[4] = {1, 2, 3, 4}, gg[4] = {0.1, -0.2, 0.3, 0}, m[4] = {0}, v[4] = {0};
  orc_adam(4, par, gg, m, v, 1, 0.01, 0.9, 0.999, 1e-8);
  printf("ok n=%d K=%lld L1=%.6g L2=%.6g tw0=%.6g\n", n, (long long)K, L1, L2, tw[0]);
  free(pix); free(dep); free(col); free(opa); free(rad); free(rec); free(ranges); free(keys);
  free(vals); free(img); free(dimg); free(sil); free(tf); free(nc); free(mg); free(g_rgb); free(g_d);
  free(gc); free(go); free(gr); free(mag); free(gkd); free(depth); free(rgb); free(kpose); free(vpose);
  free(intr); free(dims);
  return 0;
}
