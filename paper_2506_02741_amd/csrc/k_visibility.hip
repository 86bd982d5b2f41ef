// Visibility of a frame's depth points in other views [Sec. 3.3, visibility
// check]: the point of source pixel (u, v) with depth d > 0 is visible in a
// target view when its depth there, p_z > z_near, lies within rel_tol (1 %)
// of the target's depth map bilinearly interpolated at its projection (the
// four neighbours inside the map and valid).  One thread per source pixel
// walks the targets of the launch; the union over targets goes to a mask
// (Eq. 1's W against a section: its head, middle and last frames) and each
// target's count of visible points (the overlap selection) is added with one
// integer atomic per wave.  The decisions are FP32 in a pinned order (this
// file is compiled without FMA contraction), so they are bit-exact.
#include "vtgs_internal.h"
#include "geom32.h"

namespace vtgs {

namespace {

constexpr int kVisNT = 256;

__global__ __launch_bounds__(kVisNT) void k_visibility(const float *src_depth, VisCam sc,
                                                       const float *src_pose, VisTargets tg,
                                                       float tol, float znear, uint8_t *mask,
                                                       int32_t *counts, int first) {
  __shared__ float Ms[kVisMaxTargets][12];
  if (threadIdx.x < (unsigned)tg.n) relative_pose(tg.pose[threadIdx.x], src_pose, Ms[threadIdx.x]);
  __syncthreads();
  const int64_t P = (int64_t)sc.width * sc.height;
  const int64_t p = (int64_t)blockIdx.x * kVisNT + threadIdx.x;
  const bool in = p < P;
  const float d = in ? src_depth[p] : 0.f;
  const int u = in ? (int)(p % sc.width) : 0, v = in ? (int)(p / sc.width) : 0;
  uint32_t any = 0u;
  for (int t = 0; t < tg.n; t++) {
    bool vis = false;
    if (d > 0.f) {
      float px, py, pz;
      backproject_move(Ms[t], sc.fx, sc.fy, sc.cx, sc.cy, u, v, d, px, py, pz);
      if (pz > znear) {
        const float mx = tg.fx[t] * (px / pz) + tg.cx[t];
        const float my = tg.fy[t] * (py / pz) + tg.cy[t];
        const int W = tg.width[t], H = tg.height[t];
        // decided on the float coordinates before any conversion to int
        if (mx >= 0.f && my >= 0.f && mx < (float)(W - 1) && my < (float)(H - 1)) {
          const float fx0 = floorf(mx), fy0 = floorf(my);
          const int x0 = (int)fx0, y0 = (int)fy0;
          const float *D = tg.depth[t];
          const float d00 = D[(int64_t)y0 * W + x0], d01 = D[(int64_t)y0 * W + x0 + 1];
          const float d10 = D[(int64_t)(y0 + 1) * W + x0], d11 = D[(int64_t)(y0 + 1) * W + x0 + 1];
          if (d00 > 0.f && d01 > 0.f && d10 > 0.f && d11 > 0.f) {
            const float ax = mx - fx0, ay = my - fy0;
            const float top = d00 + ax * (d01 - d00);
            const float bot = d10 + ax * (d11 - d10);
            const float Dt = top + ay * (bot - top);
            vis = fabsf(pz - Dt) <= tol * Dt;
          }
        }
      }
    }
    any |= vis ? 1u : 0u;
    if (counts) {
      const unsigned long long b = ballot64(vis);
      if (lane_id() == 0 && b) atomicAdd(&counts[t], (int32_t)__popcll(b));
    }
  }
  if (in && mask) mask[p] = (uint8_t)(first ? any : (mask[p] | any));
}

}  // namespace

hipError_t launch_visibility(const float *src_depth, const VisCam &sc, const float *src_pose,
                             const VisTargets &tg, float tol, float znear, uint8_t *mask,
                             int32_t *counts, int first, hipStream_t st) {
  const int64_t P = (int64_t)sc.width * sc.height;
  if (P <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_visibility, dim3((unsigned)((P + kVisNT - 1) / kVisNT)), dim3(kVisNT), 0, st,
                     src_depth, sc, src_pose, tg, tol, znear, mask, counts, first);
  return hipGetLastError();
}

}  // namespace vtgs
