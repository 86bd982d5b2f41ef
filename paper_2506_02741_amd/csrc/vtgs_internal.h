// Internal declarations of the gfx950 view-tied splatting library: device
// descriptors, the workspace view every kernel receives, wave64 helpers and
// the launchers each kernel source file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vtgs.h"

namespace vtgs {

constexpr int kWave = 64;

// Keyframe descriptor in device memory.
struct DevKF {
  const uint32_t *pix;
  float *depth;
  float *color;      // [3][n]
  float *opacity;
  float *radius;
  float *pose;       // [12]
  float fx, fy, cx, cy;
  int32_t width, height, n, learnable;
  float *g_color, *g_opacity, *g_radius;
  float *adam;       // [10][n]
  // geometry (learnable keyframes only): depth and pose gradients, Adam states
  float *g_depth, *g_pose, *depth_adam, *pose_adam;
  int32_t geo, pad;  // geo: the backward carries dLoss/d(centre) for it
};

// View descriptor: its records are [rec_base, rec_base + n_rec) and its
// tiles [tile_base, tile_base + tiles_x * tiles_y) of the plan.
struct DevView {
  float fx, fy, cx, cy;
  int32_t width, height, tiles_x, tiles_y;
  float *pose;
  int32_t kf_first, kf_count;
  int32_t rec_base, n_rec;
  int32_t tile_base, n_tiles;
  int64_t pix_off;
  const float *obs_rgb;
  const float *obs_depth;
  const uint8_t *vis;
  float *pose_adam;
  int32_t seg_first, seg_count;
};

// One (view, keyframe) pair: records [rec_start, rec_start + n) are the
// keyframe's Gaussians seen from the view.  M = view pose * keyframe pose^-1,
// written by every preprocessing pass (by the thread of the segment's first
// record) and read by the gradient gathers that turn dL/dp back into the
// keyframe's frame.
struct DevSeg {
  float M[12];
  int32_t view, kf, rec_start, n;
};

// Per keyframe: the views (records) that render it, for gradient gathers.
struct DevKFUse {
  int32_t rec_start;  // record index of the keyframe's Gaussian 0 in that view
  int32_t view;
  int32_t seg;        // the (view, keyframe) segment
};

enum : uint32_t { kFlagCapacity = 1u, kFlagNonfinite = 2u };

// Everything a kernel needs, passed by value.
struct Ws {
  // header
  uint32_t *flags;
  unsigned long long *n_pairs;
  uint32_t *iter;              // tracking iteration counter (bumped by preprocess)
  uint32_t *n_long;            // tiles with lists longer than the short-list sort takes
  uint32_t *long_next;         // cursor of the long-list sort over long_tiles
  uint32_t *long_tiles;        // [n_tiles] those tiles (written by the tile scan)
  uint32_t *tile_order;        // [n_tiles] compositing order, longest lists first (NULL: tile order)
  // descriptors
  const DevKF *kfs;
  const DevView *views;
  DevSeg *segs;
  const int32_t *kf_use_off;   // [n_kf + 1]
  const DevKFUse *kf_use;      // per keyframe, the views rendering it
  int32_t n_kf, n_views, n_segs, n_rec, n_tiles, max_view_tiles;
  int32_t max_view_px, pad0;
  int64_t P;                   // total pixels
  int64_t cap;                 // pair capacity
  // per record
  float4 *recA;                // [n_rec][3]: (mx,my,qa,qb) (qc,o,z,R) (c0,c1,c2,r)
  float4 *recB;                // [n_rec]: (px, py, learnable, 0)
  uint2 *rect;                 // [n_rec]: tx0|ty0<<16, tx1|ty1<<16 (tx0 > tx1: culled)
  uint32_t *rec_cnt;           // [n_rec] tiles per record
  uint32_t *zbits;             // [n_rec] FP32 bits of the centre depth (the sort key's high word)
  uint32_t *rec_off;           // [n_rec + 1] exclusive scan of rec_cnt
  uint32_t *scan_part;         // [scan blocks + 1]
  // per tile
  uint32_t *tile_count;        // [n_tiles] pairs of record groups with a shared tile box
  uint32_t *tile_count_ns;     // [n_tiles] pairs of the other groups
  uint32_t *tile_fill;         // [n_tiles] next free list position of the other groups
  uint32_t *wave_off;          // [n_rec rounded up to 64] per 64-record group, lane j: the
                               // group's first position in its box tile j (relative)
  uint2 *ranges;               // [n_tiles] (start, end)
  // pairs
  unsigned long long *keys;    // [cap] (depth bits << 32) | view-local id
  unsigned long long *keys_tmp;// [cap]
  unsigned long long *lane_bits;// [(cap/64 + n_tiles + 2) * lane_bits_per_chunk(tile)]
  uint32_t *ids;               // [cap] sorted view-local ids
  float *slots;                // [cap][slot_w] per (record, tile) gradient partials:
                               // dL/dc (3), dL/do, dL/dr (, dL/dp in the view frame (3))
  float *kpose_part;           // [n_kf][gblocks][8] keyframe pose twist partials
  int32_t slot_w, gblocks;     // 5, or 8 with geometry; gather blocks per keyframe
  // per pixel
  float *t_final;              // [P]
  uint32_t *last;              // [P] contributors end (relative to tile start)
  float *img;                  // [5][P] internal rgb(3), depth, sil
  float *gimg;                 // [5][P] internal upstream gradients
  float *twist_part;           // [n_tiles][8]: six twist sums, the Eq. 1 loss, one unused
  float *loss_part;            // [n_views][loss_blocks][4]
  double *ssim_map;            // [3 kinds][3 ch][P], FP64
  float *ssim_part;            // [n_views][3][loss_blocks]
  int32_t loss_blocks, ssim_gx, ssim_gy, pad1;
  // render parameters
  float amin, amax, tmin, qcut, znear, lowpass;
  float bg[3];
  int32_t tile, batch;
};

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ unsigned long long lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Sum over the 64 lanes, result in every lane.  Rows of 16 are reduced with
// DPP row rotations; the four row sums are combined through readlane.
__device__ __forceinline__ float wave_sum(float x) {
  // row_ror:8, 4, 2, 1 (dpp_ctrl 0x128, 0x124, 0x122, 0x121)
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x122, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x121, 0xf, 0xf, false));
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
  return (r0 + r1) + (r2 + r3);
}

// Row sums (16 lanes) in every lane of the row: row_ror 8, 4, 2, 1.
__device__ __forceinline__ float row_sum(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x122, 0xf, 0xf, false));
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x121, 0xf, 0xf, false));
  return x;
}

// Wave minimum / maximum of an int (all 64 lanes active), returned as a
// uniform value: row_ror 8, 4, 2, 1 within rows, then the four row results.
__device__ __forceinline__ int wave_min_i(int x) {
  x = min(x, __builtin_amdgcn_update_dpp(x, x, 0x128, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(x, x, 0x124, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(x, x, 0x122, 0xf, 0xf, false));
  x = min(x, __builtin_amdgcn_update_dpp(x, x, 0x121, 0xf, 0xf, false));
  return min(min(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
             min(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}
__device__ __forceinline__ int wave_max_i(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x128, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x124, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x122, 0xf, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x121, 0xf, 0xf, false));
  return max(max(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
             max(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}

// Exclusive scan of one uint32 per thread over a block of NT threads.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds_waves,
                                                         uint32_t *total) {
  const int l = lane_id(), w = threadIdx.x / kWave;
  uint32_t x = v;
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(x, o);
    if (l >= o) x += y;
  }
  if (l == kWave - 1) lds_waves[w] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int i = 0; i < NT / kWave; i++) {
    const uint32_t s = lds_waves[i];
    if (i < w) base += s;
    tot += s;
  }
  __syncthreads();
  if (total) *total = tot;
  return base + x - v;
}

__device__ __forceinline__ int find_view_by_record(const Ws &ws, int r) {
  int lo = 0, hi = ws.n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ws.views[mid].rec_base <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The tile a compositing block takes: the scan's longest-first order when
// the plan has one, else the block's own index.
__device__ __forceinline__ int tile_of_block(const Ws &ws) {
  return ws.tile_order ? (int)ws.tile_order[blockIdx.x] : (int)blockIdx.x;
}

__device__ __forceinline__ int find_view_by_tile(const Ws &ws, int t) {
  int lo = 0, hi = ws.n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ws.views[mid].tile_base <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// launchers (each kernel source file implements its own)
// ---------------------------------------------------------------------------
// u64 words of lane bits per 64-entry chunk of a tile list: one per lane
// and pixel of every wave of the tile's block (tile 8: 1 wave of 64 pixels;
// 16: 4 waves; 32: 4 waves with 4 pixels per lane).
inline int lane_bits_per_chunk(int tile) { return tile == 8 ? 64 : tile == 16 ? 256 : 1024; }

hipError_t launch_ingest_count(const float *depth, const uint8_t *mask, int H, int W, int s,
                               uint32_t *scratch, int32_t *count, hipStream_t st);
hipError_t launch_ingest_fill(const float *depth, const float *rgb, const uint8_t *mask, int H,
                              int W, int s, float fx, float o_init, const uint32_t *scratch,
                              int n, uint32_t *pix, float *dep, float *col, float *opa,
                              float *rad, hipStream_t st);
int64_t ingest_scratch_words(int H, int W, int s);
hipError_t launch_uncovered(const float *sil, const float *depth, int64_t n, float thr,
                            uint8_t *mask, hipStream_t st);

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t st);
hipError_t launch_preprocess(const Ws &ws, hipStream_t st);
hipError_t launch_scan_tiles(const Ws &ws, hipStream_t st);
hipError_t launch_fill_keys(const Ws &ws, hipStream_t st);
hipError_t launch_sort_tiles(const Ws &ws, hipStream_t st);
hipError_t launch_scan_records(const Ws &ws, hipStream_t st);
hipError_t launch_composite_fwd(const Ws &ws, float *rgb, float *depth, float *sil,
                                hipStream_t st);
// mode bit 0: twist partials per tile, bit 1: per-(record, tile) slots,
// bit 2 (with bit 1): the slots also carry dL/dp (the plan's slot_w is 8)
// mode 1: twist, 2: slots, 3: both, 6 / 7: slots with geometry.  track (mode 1 only, else NULL): the
// upstream gradient is Eq. 1's, evaluated per pixel from the internal images
// and the views' observations (g_* ignored), and each tile's loss is kept.
hipError_t launch_composite_bwd(const Ws &ws, const float *g_rgb, const float *g_depth,
                                const float *g_sil, int mode, hipStream_t st,
                                const vtgs_track_cfg *track = nullptr);
hipError_t launch_twist_reduce(const Ws &ws, float *g_twist, hipStream_t st);
// max_n: largest Gaussian count of a learnable keyframe.  Adds the slots'
// sums (and the depth gradients) into the keyframes' gradient buffers and,
// with geometry, the keyframe pose twists into g_pose.
hipError_t launch_gather(const Ws &ws, int max_n, hipStream_t st);
hipError_t launch_track_update(const Ws &ws, const vtgs_track_cfg &cfg, float *loss,
                               hipStream_t st);
hipError_t launch_map_loss(const Ws &ws, const vtgs_map_cfg &cfg, hipStream_t st);
hipError_t launch_map_update(const Ws &ws, const vtgs_map_cfg &cfg, int32_t *step, float *loss,
                             int max_n, hipStream_t st);
int64_t rec_scan_blocks(int64_t n_rec);

// visibility: targets of one launch, passed by value
constexpr int kVisMaxTargets = 16;
struct VisCam {
  float fx, fy, cx, cy;
  int32_t width, height;
};
struct VisTargets {
  const float *depth[kVisMaxTargets];
  const float *pose[kVisMaxTargets];
  float fx[kVisMaxTargets], fy[kVisMaxTargets], cx[kVisMaxTargets], cy[kVisMaxTargets];
  int32_t width[kVisMaxTargets], height[kVisMaxTargets];
  int32_t n;
};
// first != 0: the mask is written, else OR-ed into; counts are added to
hipError_t launch_visibility(const float *src_depth, const VisCam &sc, const float *src_pose,
                             const VisTargets &tg, float tol, float znear, uint8_t *mask,
                             int32_t *counts, int first, hipStream_t st);
hipError_t launch_debug_copy(const Ws &ws, float *records, int32_t *rect, hipStream_t st);

}  // namespace vtgs
