// Losses and optimiser steps around the splat.
//
//  (Eq. 1 itself, alpha sum W |V - V'| + beta sum W |D - D'| with
//  W = vis & (D > 0) & (S' > sil_thr) held fixed, is evaluated per pixel by
//  the tracking backward, which also keeps each tile's loss)
//  twist_reduce per view, the tiles' twist partials summed in a fixed order
//  track_update twist reduce + Adam on the twist (lr_trans on rho, lr_rot on
//               phi; App. A) + pose <- exp(step^) pose
//  map_l1       Eq. 2 (Sec. 3.4) L1 terms: rho mean|V - V'|,
//               sigma mean(U |D - D'|) with U = (D > 0); gradients
//  ssim_a/b     tau (1 - SSIM(V, V')): 11x11 Gaussian window (sigma 1.5),
//               zero padding, C1 = 0.01^2, C2 = 0.03^2; separable passes
//               through LDS; the backward filters the per-pixel partials
//               with the same (symmetric) window
//  gather       per learnable keyframe Gaussian, the (record, tile) slots of
//               every view that renders it, summed in a fixed order; then
//               either added to the caller's gradient planes or used for
//               one Adam step on (c, logit o, log r) (App. A learning rates).
//               With geometry the slots also hold dL/dp: turned into the
//               keyframe's frame it gives dL/d(depth) along the pixel's ray
//               (supplementary, movable Gaussians) and, summed per
//               keyframe, the gradient of its pose twist (Sec. 3.5 bundle
//               adjustment), with Adam steps on both in map_step
#include "vtgs_internal.h"

namespace vtgs {

namespace {

constexpr int kNT = 256;
// Adam's decay rates as FP32 constants, with 1 - beta written out (1 - 0.999f
// would be 1.3e-5 away from 0.001), and its bias corrections 1 - beta^t
// through expm1 / log1p, accurate to a few ulp also for small t.
constexpr float kB1 = 0.9f, kB2 = 0.999f, kEps = 1e-8f;
constexpr float kOmB1 = 0.1f, kOmB2 = 0.001f;  // 1 - beta1, 1 - beta2

__device__ __forceinline__ float bias_corr(float one_minus_beta, float t) {
  return -expm1f(t * log1pf(-one_minus_beta));
}

__device__ __forceinline__ float sgnf(float x) { return (float)((x > 0.f) - (x < 0.f)); }

__device__ __forceinline__ float block_sum(float x, float *lds) {
  const float s = wave_sum(x);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) lds[w] = s;
  __syncthreads();
  float t = 0.f;
  for (int i = 0; i < (int)(blockDim.x / kWave); i++) t += lds[i];
  __syncthreads();
  return t;
}

// Sum of the view's tile partials (6 twist floats and the tile's Eq. 1 loss,
// at a stride of 8) in a fixed order.
__device__ __forceinline__ void reduce_view(const Ws &ws, int v, float *g6, float *loss,
                                           float *lds) {
  const DevView &vw = ws.views[v];
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float l = 0.f;
  for (int i = threadIdx.x; i < vw.n_tiles; i += blockDim.x) {
    const float *tp = ws.twist_part + 8 * (int64_t)(vw.tile_base + i);
    for (int c = 0; c < 6; c++) acc[c] += tp[c];
    l += tp[6];
  }
  for (int c = 0; c < 6; c++) g6[c] = block_sum(acc[c], lds);
  if (loss) *loss = block_sum(l, lds);
}

__global__ __launch_bounds__(kNT) void k_twist_reduce(Ws ws, float *g_twist) {
  __shared__ float lds[kNT / kWave];
  float g[6];
  reduce_view(ws, blockIdx.x, g, nullptr, lds);
  if (threadIdx.x == 0)
    for (int c = 0; c < 6; c++) g_twist[6 * blockIdx.x + c] = g[c];
}

// exp of a twist (rho, phi): R = I + A K + B K^2, t = (I + B K + C K^2) rho.
__device__ void se3_exp(const float *xi, float *E) {
  const float *rho = xi, *phi = xi + 3;
  const float th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  const float th = sqrtf(th2);
  float A, B, C;
  if (th < 1e-3f) {
    A = 1.f - th2 / 6.f;
    B = 0.5f - th2 / 24.f;
    C = 1.f / 6.f - th2 / 120.f;
  } else {
    A = sinf(th) / th;
    B = (1.f - cosf(th)) / th2;
    C = (th - sinf(th)) / (th2 * th);
  }
  const float K[3][3] = {{0.f, -phi[2], phi[1]}, {phi[2], 0.f, -phi[0]}, {-phi[1], phi[0], 0.f}};
  float K2[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) K2[i][j] = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
  for (int i = 0; i < 3; i++) {
    float t = 0.f;
    for (int j = 0; j < 3; j++) {
      const float I = i == j ? 1.f : 0.f;
      E[4 * i + j] = I + A * K[i][j] + B * K2[i][j];
      t += (I + B * K[i][j] + C * K2[i][j]) * rho[j];
    }
    E[4 * i + 3] = t;
  }
}

constexpr int kUpdNT = 1024;

__global__ __launch_bounds__(kUpdNT) void k_track_update(Ws ws, vtgs_track_cfg cfg, float *loss) {
  // the view's tile partials (6 twist sums + loss, stride 8): per thread,
  // then per wave (DPP), then the 16 waves in order -- one barrier
  __shared__ float part[kUpdNT / kWave][7];
  const int v = blockIdx.x;
  const DevView &vw0 = ws.views[v];
  // the pose, its Adam state and the iteration count, read before the sums
  // so that their latency overlaps the reduction (thread 0 uses them)
  float T[12], S[13];
  int iter = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 12; i++) T[i] = vw0.pose[i];
#pragma unroll
    for (int i = 0; i < 13; i++) S[i] = vw0.pose_adam[i];
    iter = *ws.iter;
  }
  float acc[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int i = threadIdx.x; i < vw0.n_tiles; i += kUpdNT) {
    const float *tp = ws.twist_part + 8 * (int64_t)(vw0.tile_base + i);
#pragma unroll
    for (int c = 0; c < 7; c++) acc[c] += tp[c];
  }
#pragma unroll
  for (int c = 0; c < 7; c++) {
    const float sw = wave_sum(acc[c]);
    if (lane_id() == 0) part[threadIdx.x / kWave][c] = sw;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  float g[6], L = 0.f;
  for (int c = 0; c < 6; c++) g[c] = 0.f;
  for (int w = 0; w < kUpdNT / kWave; w++) {
    for (int c = 0; c < 6; c++) g[c] += part[w][c];
    L += part[w][6];
  }
  const DevView &vw = ws.views[v];
  if (loss) loss[(int64_t)iter * ws.n_views + v] = L;
  bool finite = __builtin_isfinite(L);
  for (int c = 0; c < 6; c++) finite &= __builtin_isfinite(g[c]);
  if (!finite) { atomicOr(ws.flags, kFlagNonfinite); return; }
  float *st = vw.pose_adam;
  const float t = S[12] + 1.f;
  st[12] = t;
  const float c1 = bias_corr(kOmB1, t), c2 = bias_corr(kOmB2, t);
  float xi[6];
  for (int i = 0; i < 6; i++) {
    const float m = kB1 * S[i] + kOmB1 * g[i];
    const float s = kB2 * S[6 + i] + kOmB2 * g[i] * g[i];
    st[i] = m;
    st[6 + i] = s;
    const float lr = i < 3 ? cfg.lr_trans : cfg.lr_rot;
    xi[i] = -lr * (m / c1) / (sqrtf(s / c2) + kEps);
  }
  float E[12], N[12];
  se3_exp(xi, E);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 4; j++) {
      float s = E[4 * i + 0] * T[j] + E[4 * i + 1] * T[4 + j] + E[4 * i + 2] * T[8 + j];
      if (j == 3) s += E[4 * i + 3];
      N[4 * i + j] = s;
    }
  for (int i = 0; i < 12; i++) vw.pose[i] = N[i];
}

// ---- Eq. 2 ----------------------------------------------------------------

__global__ __launch_bounds__(kNT) void k_map_l1(Ws ws, vtgs_map_cfg cfg) {
  __shared__ float lds[kNT / kWave];
  const int v = blockIdx.y;
  const DevView &vw = ws.views[v];
  const int64_t Pv = (int64_t)vw.width * vw.height;
  const int64_t lp = (int64_t)blockIdx.x * kNT + threadIdx.x;
  const int64_t P = ws.P;
  float l1 = 0.f, ld = 0.f;
  if (lp < Pv) {
    const int64_t p = vw.pix_off + lp;
    const float inv3 = 1.0f / (3.0f * (float)Pv), inv1 = 1.0f / (float)Pv;
    for (int c = 0; c < 3; c++) {
      const float r = vw.obs_rgb[c * Pv + lp] - ws.img[c * P + p];
      l1 += fabsf(r);
      ws.gimg[c * P + p] = -cfg.rho * sgnf(r) * inv3;
    }
    const float od = vw.obs_depth[lp];
    const float rd = od - ws.img[3 * P + p];
    const bool U = od > 0.f;
    if (U) ld += fabsf(rd);
    ws.gimg[3 * P + p] = U ? -cfg.sigma * sgnf(rd) * inv1 : 0.f;
  }
  const float s1 = block_sum(l1, lds);
  const float s2 = block_sum(ld, lds);
  if (threadIdx.x == 0) {
    float *o = ws.loss_part + 4 * ((int64_t)v * ws.loss_blocks + blockIdx.x);
    o[0] = s1;
    o[1] = s2;
  }
}

constexpr int kS = 16, kR = 5, kH = kS + 2 * kR;  // SSIM output tile, window radius

__device__ __forceinline__ double gwin(int k) {
  // normalised 11-tap Gaussian, sigma 1.5: exp(-i^2 / 4.5) / sum, i = -5..5
  constexpr double w[11] = {1.02838008447911008e-03, 7.59875813523918503e-03,
                            3.60007721284308288e-02, 1.09360689509700015e-01,
                            2.13005537711253690e-01, 2.66011724861794363e-01,
                            2.13005537711253690e-01, 1.09360689509700015e-01,
                            3.60007721284308288e-02, 7.59875813523918503e-03,
                            1.02838008447911008e-03};
  return w[k];
}

// The SSIM moments, the map and its partials are evaluated in FP64: the
// variances are differences of second moments and squared means of similar
// size, which FP32 would leave with ~1e-5 relative error, and the gradient
// combines the filtered partials with cancellation.
__global__ __launch_bounds__(kNT) void k_ssim_a(Ws ws, int gx, int gy) {
  __shared__ float xs[kH][kH], ys[kH][kH];
  __shared__ double hs[5][kH][kS];
  __shared__ float lds[kNT / kWave];
  const int v = blockIdx.z / 3, c = blockIdx.z % 3;
  const DevView &vw = ws.views[v];
  const int W = vw.width, H = vw.height;
  const int x0 = blockIdx.x * kS, y0 = blockIdx.y * kS;
  if (x0 >= W || y0 >= H) {
    if (threadIdx.x == 0) ws.ssim_part[((int64_t)blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x] = 0.f;
    return;
  }
  const int64_t P = ws.P, Pv = (int64_t)W * H;
  const float *X = ws.img + c * P + vw.pix_off;
  const float *Y = vw.obs_rgb + c * Pv;
  for (int i = threadIdx.x; i < kH * kH; i += kNT) {
    const int yy = y0 - kR + i / kH, xx = x0 - kR + i % kH;
    const bool in = xx >= 0 && xx < W && yy >= 0 && yy < H;
    xs[i / kH][i % kH] = in ? X[(int64_t)yy * W + xx] : 0.f;
    ys[i / kH][i % kH] = in ? Y[(int64_t)yy * W + xx] : 0.f;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kH * kS; i += kNT) {
    const int r = i / kS, cc = i % kS;
    double a = 0.0, b = 0.0, aa = 0.0, bb = 0.0, ab = 0.0;
    for (int k = 0; k < 2 * kR + 1; k++) {
      const double w = gwin(k), xv = xs[r][cc + k], yv = ys[r][cc + k];
      a = fma(w, xv, a); b = fma(w, yv, b);
      aa = fma(w, xv * xv, aa); bb = fma(w, yv * yv, bb); ab = fma(w, xv * yv, ab);
    }
    hs[0][r][cc] = a; hs[1][r][cc] = b; hs[2][r][cc] = aa; hs[3][r][cc] = bb; hs[4][r][cc] = ab;
  }
  __syncthreads();
  const int lx = threadIdx.x % kS, ly = threadIdx.x / kS;
  const int xx = x0 + lx, yy = y0 + ly;
  float S = 0.f;
  if (xx < W && yy < H) {
    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < 2 * kR + 1; k++) {
      const double w = gwin(k);
      for (int q = 0; q < 5; q++) m[q] = fma(w, hs[q][ly + k][lx], m[q]);
    }
    const double C1 = 1e-4, C2 = 9e-4;
    const double mx = m[0], my = m[1];
    const double vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
    const double A1 = 2.0 * mx * my + C1, A2 = 2.0 * cxy + C2;
    const double B1 = mx * mx + my * my + C1, B2 = vx + vy + C2;
    const double inv = 1.0 / (B1 * B2);
    const double Sd = A1 * A2 * inv;
    S = (float)Sd;
    const double Smu = 2.0 * my * A2 * inv - 2.0 * mx * Sd / B1;
    const double Ssig = -Sd / B2;
    const double Scov = 2.0 * A1 * inv;
    const int64_t p = (int64_t)c * P + vw.pix_off + (int64_t)yy * W + xx;
    ws.ssim_map[p] = Smu - 2.0 * mx * Ssig - my * Scov;
    ws.ssim_map[3 * P + p] = Ssig;
    ws.ssim_map[6 * P + p] = Scov;
  }
  const float s = block_sum(S, lds);
  if (threadIdx.x == 0) ws.ssim_part[((int64_t)blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x] = s;
}

// dSSIM_mean/dx(p) = (1/P) [ (w*A)(p) + 2 x(p) (w*B)(p) + y(p) (w*Cov)(p) ]
__global__ __launch_bounds__(kNT) void k_ssim_b(Ws ws, vtgs_map_cfg cfg) {
  __shared__ double ms[3][kH][kH];
  __shared__ double hs[3][kH][kS];
  const int v = blockIdx.z / 3, c = blockIdx.z % 3;
  const DevView &vw = ws.views[v];
  const int W = vw.width, H = vw.height;
  const int x0 = blockIdx.x * kS, y0 = blockIdx.y * kS;
  if (x0 >= W || y0 >= H) return;
  const int64_t P = ws.P, Pv = (int64_t)W * H;
  for (int i = threadIdx.x; i < kH * kH; i += kNT) {
    const int yy = y0 - kR + i / kH, xx = x0 - kR + i % kH;
    const bool in = xx >= 0 && xx < W && yy >= 0 && yy < H;
    const int64_t p = (int64_t)c * P + vw.pix_off + (int64_t)yy * W + xx;
    for (int q = 0; q < 3; q++) ms[q][i / kH][i % kH] = in ? ws.ssim_map[q * 3 * P + p] : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kH * kS; i += kNT) {
    const int r = i / kS, cc = i % kS;
    double a[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 2 * kR + 1; k++) {
      const double w = gwin(k);
      for (int q = 0; q < 3; q++) a[q] = fma(w, ms[q][r][cc + k], a[q]);
    }
    for (int q = 0; q < 3; q++) hs[q][r][cc] = a[q];
  }
  __syncthreads();
  const int lx = threadIdx.x % kS, ly = threadIdx.x / kS;
  const int xx = x0 + lx, yy = y0 + ly;
  if (xx >= W || yy >= H) return;
  double f[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 2 * kR + 1; k++) {
    const double w = gwin(k);
    for (int q = 0; q < 3; q++) f[q] = fma(w, hs[q][ly + k][lx], f[q]);
  }
  const int64_t lp = (int64_t)yy * W + xx;
  const int64_t p = vw.pix_off + lp;
  const double x = ws.img[c * P + p], y = vw.obs_rgb[c * Pv + lp];
  const double g = (f[0] + 2.0 * x * f[1] + y * f[2]) / (double)Pv;
  ws.gimg[c * P + p] = (float)((double)ws.gimg[c * P + p] - (double)cfg.tau * g / 3.0);
}

__global__ __launch_bounds__(kNT) void k_map_loss_reduce(Ws ws, vtgs_map_cfg cfg, int gx, int gy,
                                                         float *loss) {
  __shared__ float lds[kNT / kWave];
  const int v = blockIdx.x;
  const DevView &vw = ws.views[v];
  const int64_t Pv = (int64_t)vw.width * vw.height;
  const int nb = (int)((Pv + kNT - 1) / kNT);
  float a = 0.f, b = 0.f, s = 0.f;
  for (int i = threadIdx.x; i < nb; i += kNT) {
    const float *o = ws.loss_part + 4 * ((int64_t)v * ws.loss_blocks + i);
    a += o[0];
    b += o[1];
  }
  for (int i = threadIdx.x; i < 3 * gx * gy; i += kNT) s += ws.ssim_part[(int64_t)v * 3 * gx * gy + i];
  a = block_sum(a, lds);
  b = block_sum(b, lds);
  s = block_sum(s, lds);
  if (threadIdx.x == 0) {
    const float L = cfg.rho * a / (3.f * (float)Pv) + cfg.tau * (1.f - s / (3.f * (float)Pv)) +
                    cfg.sigma * b / (float)Pv;
    if (!__builtin_isfinite(L)) atomicOr(ws.flags, kFlagNonfinite);
    if (loss) loss[v] = L;
  }
}

// Sum of a keyframe Gaussian's slots over the views rendering it, in a
// fixed order: g = (dL/dc, dL/do, dL/dr) and, with geometry, h = dL/dX, the
// gradient of its centre in the keyframe's camera frame (each view's dL/dp
// turned back by that view's rotation, p = R X + t).
__device__ __forceinline__ void gather_slots(const Ws &ws, int kf, int i, float *g, float *h) {
  for (int c = 0; c < 5; c++) g[c] = 0.f;
  h[0] = h[1] = h[2] = 0.f;
  const int SW = ws.slot_w;
  for (int u = ws.kf_use_off[kf]; u < ws.kf_use_off[kf + 1]; u++) {
    const DevKFUse U = ws.kf_use[u];
    const int rec = U.rec_start + i;
    const uint32_t a = ws.rec_off[rec];
    const uint32_t b = (uint64_t)ws.rec_off[rec + 1] < (uint64_t)ws.cap ? ws.rec_off[rec + 1]
                                                                        : (uint32_t)ws.cap;
    float gp[3] = {0.f, 0.f, 0.f};
    for (uint32_t s = a; s < b; s++) {
      const float *sl = ws.slots + SW * (int64_t)s;
      for (int c = 0; c < 5; c++) g[c] += sl[c];
      if (SW == 8)
        for (int c = 0; c < 3; c++) gp[c] += sl[5 + c];
    }
    if (SW == 8) {
      const float *M = ws.segs[U.seg].M;
      for (int c = 0; c < 3; c++) h[c] += fmaf(M[c], gp[0], fmaf(M[4 + c], gp[1], M[8 + c] * gp[2]));
    }
  }
}

// The keyframe side of a Gaussian's centre gradient h: X = d n with n its
// pixel's ray (z = 1); dL/dd = h . n, and a left twist of the keyframe pose
// moves X to exp(-twist^) X, so the twist gradient gets (-h, -X x h).
__device__ __forceinline__ float centre_terms(const DevKF &K, int i, const float *h, float *tw) {
  const uint32_t pix = K.pix[i];
  const float u = (float)(pix % (uint32_t)K.width), v = (float)(pix / (uint32_t)K.width);
  const float n0 = (u - K.cx) / K.fx, n1 = (v - K.cy) / K.fy;
  const float d = K.depth[i];
  const float X0 = d * n0, X1 = d * n1, X2 = d;
  tw[0] = -h[0];
  tw[1] = -h[1];
  tw[2] = -h[2];
  tw[3] = -(X1 * h[2] - X2 * h[1]);
  tw[4] = -(X2 * h[0] - X0 * h[2]);
  tw[5] = -(X0 * h[1] - X1 * h[0]);
  return fmaf(h[0], n0, fmaf(h[1], n1, h[2]));
}

// Six sums over the block (wave sums, then the waves in order), written as
// this block's partial of keyframe kf's pose twist.
__device__ __forceinline__ void store_pose_partial(const Ws &ws, int kf, const float *tw,
                                                   float (*lds)[6]) {
  const int w = threadIdx.x / kWave;
  for (int c = 0; c < 6; c++) {
    const float s = wave_sum(tw[c]);
    if (lane_id() == 0) lds[w][c] = s;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    float s = 0.f;
    for (int ww = 0; ww < kNT / kWave; ww++) s += lds[ww][threadIdx.x];
    ws.kpose_part[((int64_t)kf * ws.gblocks + blockIdx.x) * 8 + threadIdx.x] = s;
  }
}

__global__ __launch_bounds__(kNT) void k_gather_accumulate(Ws ws) {
  __shared__ float lds[kNT / kWave][6];
  const int kf = blockIdx.y;
  const DevKF &K = ws.kfs[kf];
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (!K.learnable) return;  // uniform over the block
  const bool on = i < K.n;
  float g[5], h[3], tw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (on) {
    gather_slots(ws, kf, i, g, h);
    if (K.g_color)
      for (int c = 0; c < 3; c++) K.g_color[(int64_t)c * K.n + i] += g[c];
    if (K.g_opacity) K.g_opacity[i] += g[3];
    if (K.g_radius) K.g_radius[i] += g[4];
    if (ws.slot_w == 8 && K.geo) {
      const float gd = centre_terms(K, i, h, tw);
      if (K.g_depth) K.g_depth[i] += gd;
    }
  }
  if (ws.slot_w == 8 && K.geo) store_pose_partial(ws, kf, tw, lds);
}

// Per keyframe with geometry: the blocks' pose partials summed in order,
// added into g_pose.
__global__ __launch_bounds__(kWave) void k_kpose_accumulate(Ws ws) {
  const int kf = blockIdx.x;
  const DevKF &K = ws.kfs[kf];
  if (!K.learnable || !K.geo || !K.g_pose || threadIdx.x >= 6) return;
  float s = 0.f;
  for (int b = 0; b < ws.gblocks; b++) s += ws.kpose_part[((int64_t)kf * ws.gblocks + b) * 8 + threadIdx.x];
  K.g_pose[threadIdx.x] += s;
}

__global__ __launch_bounds__(kNT) void k_map_adam(Ws ws, vtgs_map_cfg cfg, const int32_t *step) {
  __shared__ float lds[kNT / kWave][6];
  const int kf = blockIdx.y;
  const DevKF &K = ws.kfs[kf];
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (!K.learnable || !K.adam) return;  // uniform over the block
  const bool geo = ws.slot_w == 8 && K.geo;
  float tw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const float t = (float)(*step);
  const float c1 = bias_corr(kOmB1, t), c2 = bias_corr(kOmB2, t);
  if (i < K.n) {
    float g[5], h[3];
    gather_slots(ws, kf, i, g, h);
    const int64_t n = K.n;
    const float o = K.opacity[i], r = K.radius[i];
    // parameters: colour as is, logit of opacity, log of radius
    float x[5] = {K.color[i], K.color[n + i], K.color[2 * n + i], logf(o / (1.f - o)), logf(r)};
    const float gx[5] = {g[0], g[1], g[2], g[3] * o * (1.f - o), g[4] * r};
    const float lr[5] = {cfg.lr_color, cfg.lr_color, cfg.lr_color, cfg.lr_opacity, cfg.lr_radius};
    float *M = K.adam, *V = K.adam + 5 * n;
    for (int c = 0; c < 5; c++) {
      const float m = kB1 * M[c * n + i] + kOmB1 * gx[c];
      const float s = kB2 * V[c * n + i] + kOmB2 * gx[c] * gx[c];
      M[c * n + i] = m;
      V[c * n + i] = s;
      x[c] -= lr[c] * (m / c1) / (sqrtf(s / c2) + kEps);
    }
    K.color[i] = x[0];
    K.color[n + i] = x[1];
    K.color[2 * n + i] = x[2];
    K.opacity[i] = 1.f / (1.f + expf(-x[3]));
    K.radius[i] = expf(x[4]);
    if (geo) {
      // the pose terms use the depth before its own step
      const float gd = centre_terms(K, i, h, tw);
      if (K.depth_adam) {
        float *DM = K.depth_adam, *DV = K.depth_adam + n;
        const float m = kB1 * DM[i] + kOmB1 * gd;
        const float s = kB2 * DV[i] + kOmB2 * gd * gd;
        DM[i] = m;
        DV[i] = s;
        K.depth[i] -= cfg.lr_depth * (m / c1) / (sqrtf(s / c2) + kEps);
      }
    }
  }
  if (geo) store_pose_partial(ws, kf, tw, lds);
}

// Adam on the left twist of a keyframe pose (lr_trans on rho, lr_rot on
// phi; step count in pose_adam[12]) from its blocks' partials, then
// pose <- exp(step^) pose: bundle adjustment inside the mapping step.
__global__ __launch_bounds__(kWave) void k_kpose_update(Ws ws, vtgs_map_cfg cfg) {
  const int kf = blockIdx.x;
  const DevKF &K = ws.kfs[kf];
  if (!K.learnable || !K.geo || !K.pose_adam || threadIdx.x != 0) return;
  float g[6];
  for (int c = 0; c < 6; c++) {
    float s = 0.f;
    for (int b = 0; b < ws.gblocks; b++) s += ws.kpose_part[((int64_t)kf * ws.gblocks + b) * 8 + c];
    g[c] = s;
  }
  bool finite = true;
  for (int c = 0; c < 6; c++) finite &= __builtin_isfinite(g[c]);
  if (!finite) { atomicOr(ws.flags, kFlagNonfinite); return; }
  float *st = K.pose_adam;
  const float t = st[12] + 1.f;
  st[12] = t;
  const float c1 = bias_corr(kOmB1, t), c2 = bias_corr(kOmB2, t);
  float xi[6];
  for (int c = 0; c < 6; c++) {
    const float m = kB1 * st[c] + kOmB1 * g[c];
    const float s = kB2 * st[6 + c] + kOmB2 * g[c] * g[c];
    st[c] = m;
    st[6 + c] = s;
    const float lr = c < 3 ? cfg.lr_trans : cfg.lr_rot;
    xi[c] = -lr * (m / c1) / (sqrtf(s / c2) + kEps);
  }
  float E[12], T[12], N[12];
  for (int c = 0; c < 12; c++) T[c] = K.pose[c];
  se3_exp(xi, E);
  for (int r = 0; r < 3; r++)
    for (int j = 0; j < 4; j++) {
      float s = E[4 * r + 0] * T[j] + E[4 * r + 1] * T[4 + j] + E[4 * r + 2] * T[8 + j];
      if (j == 3) s += E[4 * r + 3];
      N[4 * r + j] = s;
    }
  for (int c = 0; c < 12; c++) K.pose[c] = N[c];
}

__global__ void k_step_inc(int32_t *step) { *step += 1; }

}  // namespace


hipError_t launch_twist_reduce(const Ws &ws, float *g_twist, hipStream_t st) {
  hipLaunchKernelGGL(k_twist_reduce, dim3(ws.n_views), dim3(kNT), 0, st, ws, g_twist);
  return hipGetLastError();
}

hipError_t launch_track_update(const Ws &ws, const vtgs_track_cfg &cfg, float *loss,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_track_update, dim3(ws.n_views), dim3(kUpdNT), 0, st, ws, cfg, loss);
  return hipGetLastError();
}

void ssim_grid(const Ws &ws, int *gx, int *gy) {
  *gx = ws.ssim_gx;
  *gy = ws.ssim_gy;
}

hipError_t launch_map_loss(const Ws &ws, const vtgs_map_cfg &cfg, hipStream_t st) {
  int gx, gy;
  ssim_grid(ws, &gx, &gy);
  hipLaunchKernelGGL(k_map_l1, dim3(ws.loss_blocks, ws.n_views), dim3(kNT), 0, st, ws, cfg);
  hipLaunchKernelGGL(k_ssim_a, dim3(gx, gy, 3 * ws.n_views), dim3(kNT), 0, st, ws, gx, gy);
  hipLaunchKernelGGL(k_ssim_b, dim3(gx, gy, 3 * ws.n_views), dim3(kNT), 0, st, ws, cfg);
  return hipGetLastError();
}

hipError_t launch_gather(const Ws &ws, int max_n, hipStream_t st) {
  if (max_n <= 0 || ws.n_kf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_accumulate, dim3((max_n + kNT - 1) / kNT, ws.n_kf), dim3(kNT), 0, st,
                     ws);
  if (ws.slot_w == 8)
    hipLaunchKernelGGL(k_kpose_accumulate, dim3(ws.n_kf), dim3(kWave), 0, st, ws);
  return hipGetLastError();
}

hipError_t launch_map_update(const Ws &ws, const vtgs_map_cfg &cfg, int32_t *step, float *loss,
                               int max_n, hipStream_t st) {
  int gx, gy;
  ssim_grid(ws, &gx, &gy);
  hipLaunchKernelGGL(k_map_loss_reduce, dim3(ws.n_views), dim3(kNT), 0, st, ws, cfg, gx, gy, loss);
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(1), 0, st, step);
  if (max_n > 0 && ws.n_kf > 0) {
    hipLaunchKernelGGL(k_map_adam, dim3((max_n + kNT - 1) / kNT, ws.n_kf), dim3(kNT), 0, st, ws,
                       cfg, (const int32_t *)step);
    if (ws.slot_w == 8)
      hipLaunchKernelGGL(k_kpose_update, dim3(ws.n_kf), dim3(kWave), 0, st, ws, cfg);
  }
  return hipGetLastError();
}

}  // namespace vtgs
