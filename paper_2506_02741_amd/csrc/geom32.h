// FP32 camera geometry shared by the kernels whose decisions follow a
// pinned IEEE operation order (binning, visibility): include it only from
// sources compiled without FMA contraction (-ffp-contract=off), so that
// every line below is the same sequence of rounded operations everywhere.
#pragma once

#include "vtgs_internal.h"

namespace vtgs {

// M = Tv * Tk^-1 = [Rv Rk^T | tv - (Rv Rk^T) tk], fixed summation order.
// Relative pose M = T_v T_k^-1 (3x4, world->camera poses with orthonormal
// rotations, so T_k^-1 = [R_k^T | -R_k^T t_k]) in a fixed FP32 order.
__device__ __forceinline__ void relative_pose(const float *Tv, const float *Tk, float *M) {
  float tv[12], tk[12];
#pragma unroll
  for (int i = 0; i < 12; i++) { tv[i] = Tv[i]; tk[i] = Tk[i]; }
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
      M[4 * i + j] = (tv[4 * i + 0] * tk[4 * j + 0] + tv[4 * i + 1] * tk[4 * j + 1]) +
                     tv[4 * i + 2] * tk[4 * j + 2];
#pragma unroll
  for (int i = 0; i < 3; i++)
    M[4 * i + 3] = tv[4 * i + 3] -
                   ((M[4 * i + 0] * tk[3] + M[4 * i + 1] * tk[7]) + M[4 * i + 2] * tk[11]);
}

// A keyframe pixel (u, v) with z-depth d, back-projected through the
// pinhole (fx, fy, cx, cy) and moved by M into another camera's frame.
__device__ __forceinline__ void backproject_move(const float *M, float fx, float fy, float cx,
                                                 float cy, int u, int v, float d, float &px,
                                                 float &py, float &pz) {
  const float xk = (((float)u - cx) / fx) * d;
  const float yk = (((float)v - cy) / fy) * d;
  const float zk = d;
  px = ((M[0] * xk + M[1] * yk) + M[2] * zk) + M[3];
  py = ((M[4] * xk + M[5] * yk) + M[6] * zk) + M[7];
  pz = ((M[8] * xk + M[9] * yk) + M[10] * zk) + M[11];
}

}  // namespace vtgs
