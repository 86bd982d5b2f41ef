// Preprocessing and tile binning of view-tied Gaussians.
//
//  setup      M_vk = T_v T_k^-1 for every (view, keyframe) pair
//  preprocess per (view, Gaussian): back-project the tied depth pixel with
//             the keyframe pose (Sec. 3.2), move it to the view camera,
//             project, Sigma_2D = r^2 J J^T + lowpass*I, conic, extent
//             R = ceil(sqrt(q_cut * lambda_max)), tile rectangle; then count
//             the Gaussian in each tile it covers (wave-aggregated atomics,
//             whose old values are the wave's positions in those tiles)
//  scan_tiles exclusive scan of the tile counts -> per-tile [start, end)
//  fill_keys  write (depth bits << 32 | view-local id) into the tile slots
//  sort_tiles sort each tile's keys (ascending depth, ties by id) in LDS and
//             emit the id list the compositing kernels walk
//  scan_recs  exclusive scan of tiles per record (gradient slot offsets)
//
// Every floating-point operation that decides a tile or a record is
// written in a fixed order and compiled without contraction, so the tile
// lists are bit-identical to an IEEE single-precision evaluation of the same
// expressions.
#include "vtgs_internal.h"
#include "geom32.h"

#pragma clang fp contract(off)

namespace vtgs {

namespace {

constexpr int kNT = 256;

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_f32(float *p, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__device__ __forceinline__ int find_seg(const Ws &ws, int r) {
  int lo = 0, hi = ws.n_segs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ws.segs[mid].rec_start <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ void unpack_rect(uint2 rc, int &x0, int &y0, int &x1, int &y1) {
  x0 = rc.x & 0xffff; y0 = rc.x >> 16; x1 = rc.y & 0xffff; y1 = rc.y >> 16;
}

constexpr int kBoxMax = 24;  // tiles of a shared box

// Tiles covered by a wave's rectangles (a group of 64 consecutive records).
// When the whole wave belongs to one view and its rectangles fit in a
// bounding box of at most kBoxMax tiles, box tile j (row-major) is owned by
// lane j: the lanes count their tiles in LDS counters, and lane j issues the
// global atomic of tile j, so one instruction serves the whole box.
// Otherwise (mixed views or a large box) each lane adds to its own tiles'
// counters alone.
struct WaveBox {
  int bx0, by0, nx, area;
  int src;  // a lane with a rectangle (when shared): its view is the box's
  bool shared;
};

__device__ __forceinline__ WaveBox wave_box(bool has, int view, int x0, int y0, int x1, int y1) {
  WaveBox b;
  const int vmin = wave_min_i(has ? view : 0x7fffffff);
  const int vmax = wave_max_i(has ? view : -1);
  b.bx0 = wave_min_i(has ? x0 : 0x7fffffff);
  b.by0 = wave_min_i(has ? y0 : 0x7fffffff);
  const int bx1 = wave_max_i(has ? x1 : -1), by1 = wave_max_i(has ? y1 : -1);
  b.nx = bx1 - b.bx0 + 1;
  const long area = vmax < 0 ? 0 : (long)b.nx * (long)(by1 - b.by0 + 1);
  b.shared = vmax >= 0 && vmin == vmax && area <= kBoxMax;
  b.area = b.shared ? (int)area : 0;
  b.src = (int)__builtin_ctzll(ballot64(has) | (1ull << 63));
  return b;
}

// An empty statement the compiler must take as reading and writing all
// memory: LDS accesses keep their program order across it, and the LDS
// executes a wave's accesses in that order.
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

// Lane j's box tile (row-major in the box) as a tile index of the box's
// view (tiles_x btx, first tile btb); lanes past the box get a tile of the
// box's first row, unused.
__device__ __forceinline__ int box_tile_of_lane(const WaveBox &b, int btx, int btb) {
  const int j = lane_id(), nx = max(b.nx, 1);
  const int q = j / nx;
  return btb + (b.by0 + q) * btx + (b.bx0 + (j - q * nx));
}

// Lane j of a shared box: the number of the wave's rectangles covering box
// tile j (0 past the box).  Every lane adds one to the counter of each box
// tile its rectangle covers, in the wave's own LDS row `cnt` (kBoxMax).
__device__ __forceinline__ uint32_t box_counts(const WaveBox &b, bool has, int x0, int y0, int x1,
                                               int y1, uint32_t *cnt) {
  const int j = lane_id();
  if (j < kBoxMax) cnt[j] = 0u;
  lds_order();
  if (has) {
    for (int ty = y0; ty <= y1; ty++)
      for (int tx = x0; tx <= x1; tx++) atomicAdd(&cnt[(ty - b.by0) * b.nx + (tx - b.bx0)], 1u);
  }
  lds_order();
  const uint32_t mine = j < b.area ? cnt[j] : 0u;
  lds_order();
  return mine;
}

// A load through a descriptor's pointer, which addresses global memory:
// read as such (the compiler cannot tell, and would issue a flat load).
template <class T>
__device__ __forceinline__ T gload(const T *p, int64_t i) {
  return ((const __attribute__((address_space(1))) T *)p)[i];
}

constexpr int kSegLds = 1024;  // segment starts the preprocess keeps in LDS
constexpr int kViewLds = 256;  // view descriptors the key fill keeps in LDS

__global__ __launch_bounds__(kNT) void k_preprocess(Ws ws) {
  const int r = blockIdx.x * kNT + threadIdx.x;
  // the segments' first records, read by the block at once, then searched
  // in LDS (plans with more segments search them in global memory, plans
  // with one take it without a search)
  __shared__ int seg_start[kSegLds];
  __shared__ uint32_t box_cnt[kNT / kWave][kBoxMax];
  const bool seg_lds = ws.n_segs > 1 && ws.n_segs <= kSegLds;
  if (seg_lds) {
    for (int k = threadIdx.x; k < ws.n_segs; k += kNT) seg_start[k] = ws.segs[k].rec_start;
    __syncthreads();
  }
  // one more pass of the pipeline: the tracking update writes its loss at
  // this index, so a captured iteration needs no per-iteration argument
  if (r == 0) *ws.iter += 1u;
  const bool active = r < ws.n_rec;
  bool has = false;
  int view = 0, x0 = 1, y0 = 0, x1 = 0, y1 = 0, tiles_x = 1, tile_base = 0;
  if (active) {
    int seg = 0;
    if (seg_lds) {
      int lo = 0, hi = ws.n_segs - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_start[mid] <= r) lo = mid; else hi = mid - 1;
      }
      seg = lo;
    } else {
      seg = find_seg(ws, r);
    }
    const DevSeg &sg = ws.segs[seg];
    const DevKF &kf = ws.kfs[sg.kf];
    const DevView &vw = ws.views[sg.view];
    // the descriptor fields used below, read up front (not inside branches)
    const float kfx = kf.fx, kfy = kf.fy, kcx = kf.cx, kcy = kf.cy;
    const float vfx = vw.fx, vfy = vw.fy, vcx = vw.cx, vcy = vw.cy;
    const int kwidth = kf.width, vtiles_y = vw.tiles_y, kn = kf.n, klearn = kf.learnable;
    const uint32_t *kpix = kf.pix;
    const float *kdepth = kf.depth, *kradius = kf.radius, *kopa = kf.opacity, *kcolor = kf.color;
    const float *vpose = vw.pose, *kpose = kf.pose;
    view = sg.view;
    tiles_x = vw.tiles_x;
    tile_base = vw.tile_base;
    const int i = r - sg.rec_start;
    // the two poses and every per-Gaussian load issued together, before the
    // arithmetic (and before any store, which the compiler could not move
    // them past)
    const uint32_t pix = gload(kpix, i);
    const float d = gload(kdepth, i);
    const float rad = gload(kradius, i);
    const float o = gload(kopa, i);
    const float c0 = gload(kcolor, i), c1 = gload(kcolor, (int64_t)kn + i),
                c2 = gload(kcolor, 2 * (int64_t)kn + i);
    float tv[12], tk[12];
#pragma unroll
    for (int c = 0; c < 12; c++) { tv[c] = gload(vpose, c); tk[c] = gload(kpose, c); }
    float M[12];
    relative_pose(tv, tk, M);
    const float learn = klearn ? 1.f : 0.f;
    const int u = (int)(pix % (uint32_t)kwidth), v = (int)(pix / (uint32_t)kwidth);
    // back-projection of the tied depth pixel (keyframe camera), into the view
    float px, py, pz;
    backproject_move(M, kfx, kfy, kcx, kcy, u, v, d, px, py, pz);
    float mx = 0.f, my = 0.f, qa = 0.f, qb = 0.f, qc = 0.f, R = 0.f;
    if (pz > ws.znear) {
      mx = vfx * (px / pz) + vcx;
      my = vfy * (py / pz) + vcy;
      const float a = vfx / pz, b = vfy / pz;
      const float zz = pz * pz;
      const float jx = -(vfx * px) / zz, jy = -(vfy * py) / zz;
      const float r2 = rad * rad;
      const float s11 = r2 * (a * a + jx * jx) + ws.lowpass;
      const float s12 = r2 * (jx * jy);
      const float s22 = r2 * (b * b + jy * jy) + ws.lowpass;
      const float det = s11 * s22 - s12 * s12;
      if (det > 0.f) {
        const float mid = 0.5f * (s11 + s22);
        const float lmax = mid + sqrtf(fmaxf(0.f, mid * mid - det));
        R = ceilf(sqrtf(ws.qcut * lmax));
        if (__builtin_isfinite(mx) && __builtin_isfinite(my) && __builtin_isfinite(R)) {
          qa = s22 / det; qb = -s12 / det; qc = s11 / det;
          const float invB = 1.0f / (float)ws.tile;
          const float fx0 = fmaxf(floorf((mx - R) * invB), 0.f);
          const float fy0 = fmaxf(floorf((my - R) * invB), 0.f);
          const float fx1 = fminf(floorf((mx + R) * invB), (float)(tiles_x - 1));
          const float fy1 = fminf(floorf((my + R) * invB), (float)(vtiles_y - 1));
          if (!(fx0 > fx1 || fy0 > fy1)) {
            x0 = (int)fx0; y0 = (int)fy0; x1 = (int)fx1; y1 = (int)fy1;
            has = true;
          }
        }
      }
    }
    float4 *A = ws.recA + 3 * (int64_t)r;
    A[0] = make_float4(mx, my, qa, qb);
    A[1] = make_float4(qc, o, pz, R);
    A[2] = make_float4(c0, c1, c2, rad);
    ws.recB[r] = make_float4(px, py, learn, 0.f);
    if (!has) { x0 = 1; y0 = 0; x1 = 0; y1 = 0; }
    ws.rect[r] = make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16));
    ws.rec_cnt[r] = has ? (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1)) : 0u;
    // the depth again on its own, so that the key fill reads 4 B per record
    ws.zbits[r] = __float_as_uint(pz);
    // the segment's relative pose, kept for the gradient gathers
    if (i == 0) {
#pragma unroll
      for (int c = 0; c < 12; c++) ws.segs[seg].M[c] = M[c];
    }
  }
  const WaveBox box = wave_box(has, view, x0, y0, x1, y1);
  if (box.shared) {
    // the lanes count their tiles in the wave's LDS row, then lane j adds
    // box tile j's count with one atomic instruction for the whole box.
    // Lane j need not hold a record of the box's view (or any record), so
    // the tile index takes that view's geometry from a lane that does.
    const int btx = __builtin_amdgcn_readlane(tiles_x, box.src);
    const int btb = __builtin_amdgcn_readlane(tile_base, box.src);
    const int mt = box_tile_of_lane(box, btx, btb);
    const uint32_t mine = box_counts(box, has, x0, y0, x1, y1, box_cnt[threadIdx.x / kWave]);
    // the atomic's old value is the group's first position in box tile j:
    // kept for the key fill, which then claims nothing for this group
    if (mine) ws.wave_off[(r & ~(kWave - 1)) + lane_id()] = atomicAdd(ws.tile_count + mt, mine);
  } else if (has) {
    // the other groups' pairs take the positions after them, claimed by
    // the key fill
    uint32_t *cnt = ws.tile_count_ns + tile_base;
    for (int ty = y0; ty <= y1; ty++)
      for (int tx = x0; tx <= x1; tx++) atomicAdd(cnt + ty * tiles_x + tx, 1u);
  }
}

constexpr int kSmallSort = 768;  // longer tile lists go to the long-list sort

// One block: tile counts -> ranges (clamped to the pair capacity), total
// pairs, capacity flag; lists longer than kSmallSort are queued for the
// long-list sort (queue and its cursor reset here); clears the counters for
// the next pass.
constexpr int kScanNT = 1024, kScanPer = 8;
constexpr int kOrderBuckets = 64;
// Bucket of a list of n entries in the longest-first order: 0 for the
// longest, two per octave (bit length and the next bit), 63 for empty.
__device__ __forceinline__ int order_bucket(uint32_t n) {
  if (n == 0u) return kOrderBuckets - 1;
  const int bl = 32 - __clz((int)n);                              // 1 .. 32
  const int sb = bl >= 2 ? (int)((n >> (bl - 2)) & 1u) : 0;
  return kOrderBuckets - 2 - min(2 * bl + sb - 2, kOrderBuckets - 2);
}
__global__ __launch_bounds__(kScanNT) void k_scan_tiles(Ws ws) {
  __shared__ uint32_t lw[kScanNT / kWave];
  __shared__ unsigned long long carry_s;
  __shared__ uint32_t nlong_s;
  if (threadIdx.x == 0) { carry_s = 0; nlong_s = 0; }
  __syncthreads();
  for (int base = 0; base < ws.n_tiles; base += kScanNT * kScanPer) {
    const int i0 = base + threadIdx.x * kScanPer;
    uint32_t v[kScanPer], vs[kScanPer], sum = 0;
    for (int k = 0; k < kScanPer; k++) {
      vs[k] = (i0 + k < ws.n_tiles) ? ws.tile_count[i0 + k] : 0u;
      v[k] = vs[k] + ((i0 + k < ws.n_tiles) ? ws.tile_count_ns[i0 + k] : 0u);
      sum += v[k];
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<kScanNT>(sum, lw, &tot);
    const unsigned long long c = carry_s;
    unsigned long long pos = c + ex;
    for (int k = 0; k < kScanPer; k++) {
      const int i = i0 + k;
      if (i < ws.n_tiles) {
        const unsigned long long s = pos < (unsigned long long)ws.cap ? pos : ws.cap;
        const unsigned long long e = pos + v[k] < (unsigned long long)ws.cap ? pos + v[k] : ws.cap;
        ws.ranges[i] = make_uint2((uint32_t)s, (uint32_t)e);
        if (e - s > (unsigned long long)kSmallSort) ws.long_tiles[atomicAdd(&nlong_s, 1u)] = i;
        ws.tile_count[i] = 0;
        ws.tile_count_ns[i] = 0;
        ws.tile_fill[i] = vs[k];
      }
      pos += v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) carry_s = c + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *ws.n_pairs = carry_s;
    if (carry_s > (unsigned long long)ws.cap) atomicOr(ws.flags, kFlagCapacity);
    *ws.n_long = nlong_s;
    *ws.long_next = 0u;
  }
  if (ws.tile_order) {
    // longest lists first: tiles bucketed by list length (two buckets per
    // octave, longest first, empty lists last), so that the compositing
    // grid, dispatched in block order, starts its heaviest tiles first and
    // ends on light ones; the order within a bucket is whatever the atomics
    // give (each tile's results do not depend on it)
    __shared__ uint32_t bk[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) bk[threadIdx.x] = 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < ws.n_tiles; i += kScanNT)
      atomicAdd(&bk[order_bucket(ws.ranges[i].y - ws.ranges[i].x)], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t run = 0u;
      for (int b = 0; b < kOrderBuckets; b++) {
        const uint32_t c = bk[b];
        bk[b] = run;
        run += c;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ws.n_tiles; i += kScanNT)
      ws.tile_order[atomicAdd(&bk[order_bucket(ws.ranges[i].y - ws.ranges[i].x)], 1u)] = (uint32_t)i;
  }
}

// Keys into tile slots.  A thread takes RPT records, r = (block * RPT + k) *
// kNT + thread, so that each k is a group of 64 consecutive records, the
// preprocess's wave; the loads of all k are issued first, then every
// group's slot bases, then the key stores, so that a wave waits on one
// round trip per phase rather than one per group (large plans; the tracking
// frame, with ~5 waves per SIMD, takes one record per thread).  A group whose
// rectangles share a tile box recomputes the preprocess's box and takes the
// positions its atomics returned; the other groups claim positions after
// all of those with atomics here.  Either way a tile's keys land in no fixed
// order; the sort that follows fixes it.
template <int RPT>
__global__ __launch_bounds__(kNT) void k_fill_keys(Ws ws) {
  // the views' first records, tiles per row and first tiles, read by the
  // block at once beside its records' loads and then searched in LDS
  // (plans with more views search the descriptors in global memory, plans
  // with one read its descriptor without a search)
  __shared__ int3 vtab[kViewLds];
  __shared__ uint32_t fill_cnt[kNT / kWave][kBoxMax], fill_base[kNT / kWave][kBoxMax],
      fill_lim[kNT / kWave][kBoxMax];
  const bool view_lds = ws.n_views > 1 && ws.n_views <= kViewLds;
  bool has[RPT];
  int x0[RPT], y0[RPT], x1[RPT], y1[RPT], tiles_x[RPT], tile_base[RPT], view[RPT];
  unsigned long long key[RPT];
  uint32_t zb[RPT];
  uint2 rc[RPT];
#pragma unroll
  for (int k = 0; k < RPT; k++) {
    const int r = (blockIdx.x * RPT + k) * kNT + threadIdx.x;
    const int rr = min(r, ws.n_rec - 1);
    rc[k] = ws.rect[rr];
    zb[k] = ws.zbits[rr];
  }
  if (view_lds) {
    for (int v = threadIdx.x; v < ws.n_views; v += kNT)
      vtab[v] = make_int3(ws.views[v].rec_base, ws.views[v].tiles_x, ws.views[v].tile_base);
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < RPT; k++) {
    const int r = (blockIdx.x * RPT + k) * kNT + threadIdx.x;
    const bool active = r < ws.n_rec;
    unpack_rect(rc[k], x0[k], y0[k], x1[k], y1[k]);
    has[k] = active && x0[k] <= x1[k];
    if (!has[k]) { x0[k] = 1; y0[k] = 0; x1[k] = 0; y1[k] = 0; }
    int rec_base;
    if (view_lds) {
      int lo = 0, hi = ws.n_views - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (vtab[mid].x <= r) lo = mid; else hi = mid - 1;
      }
      view[k] = active ? lo : 0;
      const int3 e = vtab[view[k]];
      rec_base = e.x; tiles_x[k] = e.y; tile_base[k] = e.z;
    } else {
      view[k] = active ? find_view_by_record(ws, r) : 0;
      const DevView &vw = ws.views[view[k]];
      rec_base = vw.rec_base; tiles_x[k] = vw.tiles_x; tile_base[k] = vw.tile_base;
    }
    key[k] = ((unsigned long long)zb[k] << 32) | (uint32_t)(r - rec_base);
  }
  // lane j of a group with a shared box: box tile j's first position and
  // end
  WaveBox box[RPT];
  uint32_t base[RPT], lim[RPT];
#pragma unroll
  for (int k = 0; k < RPT; k++) {
    box[k] = wave_box(has[k], view[k], x0[k], y0[k], x1[k], y1[k]);
    base[k] = 0u; lim[k] = 0u;
    if (!box[k].shared) continue;
    const int btx = __builtin_amdgcn_readlane(tiles_x[k], box[k].src);
    const int btb = __builtin_amdgcn_readlane(tile_base[k], box[k].src);
    if (lane_id() < box[k].area) {
      // the group's first position in box tile j, claimed by the
      // preprocess (unused, and never written, where no rectangle of the
      // group covers the tile)
      const uint2 rg = ws.ranges[box_tile_of_lane(box[k], btx, btb)];
      const int g0 = (blockIdx.x * RPT + k) * kNT + (threadIdx.x & ~(kWave - 1));
      base[k] = rg.x + ws.wave_off[g0 + lane_id()];
      lim[k] = rg.y;
    }
  }
  // stores: lane j parks box tile j's first position and end in the wave's
  // LDS row; every lane then takes a rank in each box tile its rectangle
  // covers from that tile's LDS counter (in whatever order the lanes come:
  // the sort fixes it).  Groups without a shared box claim and store pair
  // by pair.
  uint32_t *cnt = fill_cnt[threadIdx.x / kWave], *bs = fill_base[threadIdx.x / kWave],
           *ls = fill_lim[threadIdx.x / kWave];
#pragma unroll
  for (int k = 0; k < RPT; k++) {
    if (box[k].shared) {
      const int j = lane_id();
      if (j < kBoxMax) { cnt[j] = 0u; bs[j] = base[k]; ls[j] = lim[k]; }
      lds_order();
      if (has[k]) {
        for (int ty = y0[k]; ty <= y1[k]; ty++)
          for (int tx = x0[k]; tx <= x1[k]; tx++) {
            const int jj = (ty - box[k].by0) * box[k].nx + (tx - box[k].bx0);
            const uint32_t pos = bs[jj] + atomicAdd(&cnt[jj], 1u);
            if (pos < ls[jj]) ws.keys[pos] = key[k];
          }
      }
      lds_order();
    } else if (has[k]) {
      for (int ty = y0[k]; ty <= y1[k]; ty++)
        for (int tx = x0[k]; tx <= x1[k]; tx++) {
          const int t = tile_base[k] + ty * tiles_x[k] + tx;
          const uint32_t pos = ws.ranges[t].x + atomicAdd(ws.tile_fill + t, 1u);
          if (pos < ws.ranges[t].y) ws.keys[pos] = key[k];
        }
    }
  }
}

constexpr int kSortCap = 8192;

// Wave-wide inclusive prefix sum of a u32 (DPP row_shr 1, 2, 4, 8 within
// rows, then row_bcast:15 and row_bcast:31 across rows).  Packed 16-bit
// fields scan independently while no field total exceeds 0xffff.
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
  return x;
}

// 8-bit field d (0..15) of the pair (lo: fields 0-7, hi: fields 8-15).
__device__ __forceinline__ uint32_t field8(unsigned long long lo, unsigned long long hi, int d) {
  const unsigned long long v = d < 8 ? lo : hi;
  return (uint32_t)(v >> (8 * (d & 7))) & 0xffu;
}

// LDS slot of list position i: one spare slot after every 16, so that the
// lanes reading positions t*E .. t*E+E-1 spread over the banks.
__device__ __forceinline__ int lds_pos(int i) { return i + (i >> 4); }

// Wave OR / AND of a uint32 (all 64 lanes active), uniform result.
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t x) {
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xf, 0xf, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xf, 0xf, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x122, 0xf, 0xf, false);
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x121, 0xf, 0xf, false);
  return ((uint32_t)__builtin_amdgcn_readlane((int)x, 0) | (uint32_t)__builtin_amdgcn_readlane((int)x, 16)) |
         ((uint32_t)__builtin_amdgcn_readlane((int)x, 32) | (uint32_t)__builtin_amdgcn_readlane((int)x, 48));
}
__device__ __forceinline__ uint32_t wave_and_u32(uint32_t x) {
  x &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x128, 0xf, 0xf, false);
  x &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x124, 0xf, 0xf, false);
  x &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x122, 0xf, 0xf, false);
  x &= (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x121, 0xf, 0xf, false);
  return ((uint32_t)__builtin_amdgcn_readlane((int)x, 0) & (uint32_t)__builtin_amdgcn_readlane((int)x, 16)) &
         ((uint32_t)__builtin_amdgcn_readlane((int)x, 32) & (uint32_t)__builtin_amdgcn_readlane((int)x, 48));
}

// Padding keys (~0) must end after every real key, but the depth passes
// take only the depth nibbles in which the real keys differ: a real key
// whose varying depth nibbles are all 15 (or any key, when the depth does
// not vary) would tie with the padding on every depth pass and could keep
// a place before it.  For such a list the top nibble is sorted as well; it
// is below 8 in every real key (a finite positive depth), so it puts the
// padding last.
__device__ __forceinline__ unsigned long long nibbles_of(unsigned long long diff) {
  unsigned long long nib = 0ull;
#pragma unroll
  for (int sh = 0; sh < 64; sh += 4) nib |= ((diff >> sh) & 15ull) != 0ull ? 15ull << sh : 0ull;
  return nib;
}
constexpr unsigned long long kTopNibble = 15ull << 60;

// Stable LSD radix passes, 4-bit digits, over the nibbles set in `digits`,
// of the NT * E keys of a block.  Thread t holds keys t*E .. t*E+E-1 in
// registers ("blocked" order).  Per pass each thread counts its keys per
// digit (4-bit fields of one u64 for E <= 15, else 8-bit fields of two), a
// DPP wave scan of the counts (as 16-bit fields) and the wave totals in LDS
// give each thread its start in every digit bucket (with E <= 15 parked in
// `starts` so that each key fetches its own), and the keys are scattered
// through `buf` (at lds_pos) in thread-then-register order, which keeps each
// pass stable.  On return buf and the registers hold the keys in the new
// order.
template <int NT, int E>
__device__ void radix_passes(unsigned long long (&k)[E], unsigned long long digits,
                             unsigned long long *buf, uint32_t (*wsum)[8], uint32_t *starts) {
  constexpr int NW = NT / kWave;
  constexpr bool k4 = E <= 15;
  const int t = threadIdx.x, l = lane_id(), w = t / kWave;
  for (int sh = 0; sh < 64; sh += 4) {
    if (((digits >> sh) & 15ull) == 0ull) continue;
    int dg[E];
    unsigned long long clo = 0ull, chi = 0ull;
#pragma unroll
    for (int e = 0; e < E; e++) {
      const int d = (int)((k[e] >> sh) & 15ull);
      dg[e] = d;
      if (k4) {
        clo += 1ull << (4 * d);
      } else {
        const unsigned long long one = 1ull << (8 * (d & 7));
        clo += d < 8 ? one : 0ull;
        chi += d < 8 ? 0ull : one;
      }
    }
    // counts as 16-bit fields: c[q] holds digits 2q and 2q + 1
    uint32_t c[8], inc[8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
      if (k4) {
        const uint32_t v = q < 4 ? (uint32_t)clo : (uint32_t)(clo >> 32);
        const int o = 8 * (q & 3);
        c[q] = ((v >> o) & 15u) | (((v >> (o + 4)) & 15u) << 16);
      } else {
        c[q] = field8(clo, chi, 2 * q) | (field8(clo, chi, 2 * q + 1) << 16);
      }
      inc[q] = wave_incl_scan_u32(c[q]);
    }
    if (l == kWave - 1) {
#pragma unroll
      for (int q = 0; q < 8; q++) wsum[w][q] = inc[q];
    }
    __syncthreads();
    uint32_t start[8];
    uint32_t run = 0u;
#pragma unroll
    for (int q = 0; q < 8; q++) {
      uint32_t pre = 0u, tot = 0u;
#pragma unroll
      for (int i = 0; i < NW; i++) {
        const uint32_t v = wsum[i][q];
        pre += i < w ? v : 0u;
        tot += v;
      }
      const uint32_t a = tot & 0xffffu;
      start[q] = inc[q] - c[q] + pre + (run | ((run + a) << 16));
      run += a + (tot >> 16);
      if (k4) starts[q * NT + t] = start[q];
    }
    unsigned long long slo = 0ull, shi = 0ull;
#pragma unroll
    for (int e = 0; e < E; e++) {
      const int d = dg[e];
      uint32_t v, seen;
      if (k4) {
        v = starts[(d >> 1) * NT + t];
        seen = (uint32_t)((slo >> (4 * d)) & 15ull);
        slo += 1ull << (4 * d);
      } else {
        v = start[0];
#pragma unroll
        for (int q = 1; q < 8; q++) v = (d >> 1) == q ? start[q] : v;
        seen = field8(slo, shi, d);
        const unsigned long long one = 1ull << (8 * (d & 7));
        slo += d < 8 ? one : 0ull;
        shi += d < 8 ? 0ull : one;
      }
      const uint32_t pos = ((v >> (16 * (d & 1))) & 0xffffu) + seen;
      buf[lds_pos((int)min(pos, (uint32_t)(NT * E - 1)))] = k[e];  // a permutation
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; e++) k[e] = buf[lds_pos(t * E + e)];
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < E; e++) buf[lds_pos(t * E + e)] = k[e];
  __syncthreads();
}

// Sort of the NT * E keys (depth bits << 32 | id) of a block; the first n
// are the tile's, the rest ~0ull (maximal, and last, so they stay last; no
// real key is ~0ull, its depth bits being below the infinity bits).  Depth
// first: radix passes over the depth nibbles that vary.  Keys of equal depth
// then form runs ordered by their earlier positions; each run is put in id
// order by one thread (insertion sort), unless some run is longer than 64,
// in which case every varying nibble (id included) is sorted by radix
// instead.  Either way buf (at lds_pos) ends in ascending (depth, id) order.
template <int NT, int E>
__device__ void block_sort_u64(unsigned long long (&k)[E], int n, unsigned long long *buf,
                               uint32_t (*wsum)[8], unsigned long long *red, uint32_t *starts) {
  constexpr int NW = NT / kWave;
  const int t = threadIdx.x, l = lane_id(), w = t / kWave;
  uint32_t olo = 0u, ohi = 0u, alo = ~0u, ahi = ~0u;
#pragma unroll
  for (int e = 0; e < E; e++) {
    const bool in = k[e] != ~0ull;
    olo |= in ? (uint32_t)k[e] : 0u;
    ohi |= in ? (uint32_t)(k[e] >> 32) : 0u;
    alo &= in ? (uint32_t)k[e] : ~0u;
    ahi &= in ? (uint32_t)(k[e] >> 32) : ~0u;
  }
  const unsigned long long orw = ((unsigned long long)wave_or_u32(ohi) << 32) | wave_or_u32(olo);
  const unsigned long long andw = ((unsigned long long)wave_and_u32(ahi) << 32) | wave_and_u32(alo);
  if (l == 0) { red[2 * w] = orw; red[2 * w + 1] = andw; }
  __syncthreads();
  unsigned long long orv = 0ull, andv = ~0ull;
#pragma unroll
  for (int i = 0; i < NW; i++) { orv |= red[2 * i]; andv &= red[2 * i + 1]; }
  const unsigned long long nib = nibbles_of((orv ^ andv) & 0xFFFFFFFF00000000ull);
  bool pad_tie = false;
#pragma unroll
  for (int e = 0; e < E; e++) pad_tie |= k[e] != ~0ull && (k[e] & nib) == nib;
  const unsigned long long diff = (orv ^ andv) | (__syncthreads_or(pad_tie) ? kTopNibble : 0ull);
  radix_passes<NT, E>(k, diff & 0xFFFFFFFF00000000ull, buf, wsum, starts);
  // runs of equal depth among the first n keys, found from their first key
  bool long_run = false;
#pragma unroll
  for (int e = 0; e < E; e++) {
    const int i = t * E + e;
    if (i + 1 >= n) continue;
    const uint32_t z = (uint32_t)(buf[lds_pos(i)] >> 32);
    if ((uint32_t)(buf[lds_pos(i + 1)] >> 32) != z ||
        (i > 0 && (uint32_t)(buf[lds_pos(i - 1)] >> 32) == z)) continue;
    int len = 2;
    while (i + len < n && len <= 64 && (uint32_t)(buf[lds_pos(i + len)] >> 32) == z) len++;
    long_run = long_run || len > 64;
  }
  if (__syncthreads_or(long_run)) {
    radix_passes<NT, E>(k, diff & 0x00000000FFFFFFFFull, buf, wsum, starts);
    radix_passes<NT, E>(k, diff & 0xFFFFFFFF00000000ull, buf, wsum, starts);
    return;
  }
  // insertion sort of every run by id (the runs are disjoint)
#pragma unroll
  for (int e = 0; e < E; e++) {
    const int i = t * E + e;
    if (i + 1 >= n) continue;
    const uint32_t z = (uint32_t)(buf[lds_pos(i)] >> 32);
    if ((uint32_t)(buf[lds_pos(i + 1)] >> 32) != z ||
        (i > 0 && (uint32_t)(buf[lds_pos(i - 1)] >> 32) == z)) continue;
    int len = 2;
    while (i + len < n && (uint32_t)(buf[lds_pos(i + len)] >> 32) == z) len++;
    for (int a = i + 1; a < i + len; a++) {
      const unsigned long long v = buf[lds_pos(a)];
      int b = a - 1;
      while (b >= i && buf[lds_pos(b)] > v) { buf[lds_pos(b + 1)] = buf[lds_pos(b)]; b--; }
      buf[lds_pos(b + 1)] = v;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// One-wave tile sort (lists of up to 15 keys per lane)
// ---------------------------------------------------------------------------
// Stable LSD radix passes, 4-bit digits, over the nibbles set in `digits`,
// of the 64 * E keys of a one-wave block, lane t holding keys t*E ..
// t*E+E-1.  Per pass each lane counts its keys per digit in the 4-bit fields
// of one u64 (E <= 15), a DPP scan of the counts (as 16-bit fields) and the
// wave totals give the lane's start in every digit bucket, which the lane
// parks in LDS so that each key fetches its own; the keys are scattered in
// lane-then-register order, which keeps each pass stable.  On return the
// registers and buf (at lds_pos) hold the keys in the new order.
template <int E>
__device__ __forceinline__ void wave_radix_passes(unsigned long long (&k)[E], unsigned long long digits,
                                  unsigned long long *buf, uint32_t *starts) {
  static_assert(E <= 15, "4-bit digit counters");
  const int l = lane_id();
  for (int sh = 0; sh < 64; sh += 4) {
    if (((digits >> sh) & 15ull) == 0ull) continue;
    int dg[E];
    unsigned long long cnt = 0ull;
#pragma unroll
    for (int e = 0; e < E; e++) {
      const int d = (int)((k[e] >> sh) & 15ull);
      dg[e] = d;
      cnt += 1ull << (4 * d);
    }
    const uint32_t clo = (uint32_t)cnt, chi = (uint32_t)(cnt >> 32);
    uint32_t run = 0u;
#pragma unroll
    for (int q = 0; q < 8; q++) {
      // digits 2q and 2q + 1 as 16-bit fields, scanned over the wave
      const uint32_t v = q < 4 ? clo : chi;
      const int o = 8 * (q & 3);
      const uint32_t c = ((v >> o) & 15u) | (((v >> (o + 4)) & 15u) << 16);
      const uint32_t inc = wave_incl_scan_u32(c);
      const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
      const uint32_t a = tot & 0xffffu;
      starts[q * kWave + l] = inc - c + (run | ((run + a) << 16));
      run += a + (tot >> 16);
    }
    unsigned long long seen = 0ull;
#pragma unroll
    for (int e = 0; e < E; e++) {
      const int d = dg[e];
      const uint32_t w = starts[(d >> 1) * kWave + l];
      const uint32_t pos =
          ((w >> (16 * (d & 1))) & 0xffffu) + (uint32_t)((seen >> (4 * d)) & 15ull);
      seen += 1ull << (4 * d);
      buf[lds_pos((int)min(pos, (uint32_t)(kWave * E - 1)))] = k[e];  // a permutation
    }
    // one wave: its LDS accesses complete in program order, so no barrier
    lds_order();
#pragma unroll
    for (int e = 0; e < E; e++) k[e] = buf[lds_pos(l * E + e)];
    lds_order();
  }
}

// Sort of one tile's n <= 64 * E keys (depth bits << 32 | id, unique) by a
// one-wave block, written to dst in ascending key order as D (u32: the ids,
// u64: the keys).  The keys are
// loaded coalesced (any starting arrangement sorts to the same result, the
// keys being unique).  Depth first, over the depth nibbles that vary; equal
// depths (rare) are then put in id order as in the block sort.
template <int E, typename D>
__device__ __forceinline__ void wave_sort_tile(const unsigned long long *src, D *dst, int n,
                               unsigned long long *buf, uint32_t *starts) {
  const int l = lane_id();
  unsigned long long k[E];
  uint32_t olo = 0u, ohi = 0u, alo = ~0u, ahi = ~0u;
  // every load first (clamped index), then the padding: no wait per load
#pragma unroll
  for (int e = 0; e < E; e++) k[e] = src[min(l + kWave * e, n - 1)];
#pragma unroll
  for (int e = 0; e < E; e++) {
    const bool in = l + kWave * e < n;
    k[e] = in ? k[e] : ~0ull;
    olo |= in ? (uint32_t)k[e] : 0u;
    ohi |= in ? (uint32_t)(k[e] >> 32) : 0u;
    alo &= in ? (uint32_t)k[e] : ~0u;
    ahi &= in ? (uint32_t)(k[e] >> 32) : ~0u;
  }
  const unsigned long long diff0 =
      ((unsigned long long)(wave_or_u32(ohi) ^ wave_and_u32(ahi)) << 32) |
      (wave_or_u32(olo) ^ wave_and_u32(alo));
  const unsigned long long nib = nibbles_of(diff0 & 0xFFFFFFFF00000000ull);
  bool pad_tie = false;
#pragma unroll
  for (int e = 0; e < E; e++) pad_tie |= l + kWave * e < n && (k[e] & nib) == nib;
  const unsigned long long diff = diff0 | (ballot64(pad_tie) != 0ull ? kTopNibble : 0ull);
  if ((diff0 >> 32) == 0ull) {
    // one depth for the whole tile: the order is the id order, then the
    // top depth nibble (below 8 in every real key) puts the padding last
    wave_radix_passes<E>(k, (diff0 & 0xFFFFFFFFull) | kTopNibble, buf, starts);
  } else {
    wave_radix_passes<E>(k, diff & 0xFFFFFFFF00000000ull, buf, starts);
    // equal depths at consecutive positions?
    const uint32_t nxt = (uint32_t)__shfl_down((int)(uint32_t)(k[0] >> 32), 1);
    bool tie = false;
#pragma unroll
    for (int e = 0; e + 1 < E; e++)
      tie |= l * E + e + 1 < n && (uint32_t)(k[e] >> 32) == (uint32_t)(k[e + 1] >> 32);
    tie |= l + 1 < kWave && l * E + E < n && (uint32_t)(k[E - 1] >> 32) == nxt;
    if (ballot64(tie) != 0ull) {
      // runs of equal depth, put in id order by odd-even transposition
      // between neighbours of equal depth (runs are short: a round per key
      // of the longest run); past 64 rounds, every varying nibble (id, then
      // depth) is sorted by radix instead.  Padding keys (~0) tie with no
      // real key, a real depth being below the infinity bits.
      bool more = true;
      for (int round = 0; more && round < 64; round++) {
        bool sw = false;
#pragma unroll
        for (int ph = 0; ph < 2; ph++) {
#pragma unroll
          for (int e = ph; e + 1 < E; e += 2) {
            const bool x = (uint32_t)(k[e] >> 32) == (uint32_t)(k[e + 1] >> 32) && k[e] > k[e + 1];
            const unsigned long long lo = x ? k[e + 1] : k[e], hi = x ? k[e] : k[e + 1];
            k[e] = lo; k[e + 1] = hi;
            sw |= x;
          }
          if (ph == 1) {  // across lanes: (last of lane l, first of lane l + 1)
            const unsigned long long nx =
                ((unsigned long long)(uint32_t)__shfl_down((int)(uint32_t)(k[0] >> 32), 1) << 32) |
                (uint32_t)__shfl_down((int)(uint32_t)k[0], 1);
            const unsigned long long pv =
                ((unsigned long long)(uint32_t)__shfl_up((int)(uint32_t)(k[E - 1] >> 32), 1) << 32) |
                (uint32_t)__shfl_up((int)(uint32_t)k[E - 1], 1);
            const bool xd = l + 1 < kWave && (uint32_t)(k[E - 1] >> 32) == (uint32_t)(nx >> 32) &&
                            k[E - 1] > nx;
            const bool xu = l > 0 && (uint32_t)(pv >> 32) == (uint32_t)(k[0] >> 32) && pv > k[0];
            k[E - 1] = xd ? nx : k[E - 1];
            k[0] = xu ? pv : k[0];
            sw |= xd | xu;
          }
        }
        more = ballot64(sw) != 0ull;
      }
      if (more) {
        wave_radix_passes<E>(k, diff & 0x00000000FFFFFFFFull, buf, starts);
        wave_radix_passes<E>(k, diff & 0xFFFFFFFF00000000ull, buf, starts);
      } else {
#pragma unroll
        for (int e = 0; e < E; e++) buf[lds_pos(l * E + e)] = k[e];
        lds_order();
      }
    }
  }
  for (int i = l; i < n; i += kWave) dst[i] = (D)buf[lds_pos(i)];
}

// One round of a merge sort over n keys held as sorted runs of `width`
// keys in `in`: each pair of neighbouring runs is merged into `out` (an odd
// run at the end is copied), written as D (u64: the keys, u32: the ids).
// Every thread takes an equal share of each merged pair's output, finds
// where its share starts by a binary search along the merge path, and
// merges its share serially.  Keys are unique and below ~0, so ~0 serves
// as the end of either run.
template <int NT, typename D>
__device__ void merge_round(const unsigned long long *in, D *out, int n, int width) {
  for (int lo = 0; lo < n; lo += 2 * width) {
    const int mid = min(lo + width, n), hi = min(lo + 2 * width, n);
    const unsigned long long *A = in + lo, *B = in + mid;
    const int la = mid - lo, lb = hi - mid, m = hi - lo;
    const int d0 = (int)((int64_t)m * threadIdx.x / NT);
    const int d1 = (int)((int64_t)m * (threadIdx.x + 1) / NT);
    // the first d0 outputs are A[0, i) and B[0, d0 - i)
    int a = max(0, d0 - lb), b = min(d0, la);
    while (a < b) {
      const int md = (a + b) >> 1;
      if (A[md] < B[d0 - md - 1]) a = md + 1;
      else b = md;
    }
    int i = a, j = d0 - a;
    unsigned long long va = i < la ? A[i] : ~0ull, vb = j < lb ? B[j] : ~0ull;
    for (int d = d0; d < d1; d++) {
      const bool ta = va < vb;
      out[lo + d] = (D)(ta ? va : vb);
      if (ta) { i++; va = i < la ? A[i] : ~0ull; }
      else { j++; vb = j < lb ? B[j] : ~0ull; }
    }
  }
}

// Sort of one tile's n keys with EE keys per thread (n <= NT * EE), written
// to dst in ascending key order as D (u32: the ids, u64: the keys).
template <int NT, int EE, typename D>
__device__ __forceinline__ void sort_tile_regs(const unsigned long long *src, D *dst, int n,
                                               unsigned long long *buf, uint32_t (*wsum)[8],
                                               unsigned long long *red, uint32_t *starts) {
  unsigned long long k[EE];
  // coalesced loads (any starting arrangement sorts to the same result, the
  // keys being unique), every load first (clamped index), then the padding
#pragma unroll
  for (int e = 0; e < EE; e++) k[e] = src[min((int)threadIdx.x + NT * e, n - 1)];
#pragma unroll
  for (int e = 0; e < EE; e++) k[e] = (int)threadIdx.x + NT * e < n ? k[e] : ~0ull;
  block_sort_u64<NT, EE>(k, n, buf, wsum, red, starts);
  for (int i = threadIdx.x; i < n; i += NT) dst[i] = (D)buf[lds_pos(i)];
}

// Register tiers of the tile sort: keys per thread for a one-wave block
// (4 and 12) and for the 512-thread long-list block (6, 10 and 16); up to
// 15 keys per thread count digits in 4-bit fields and fetch their bucket
// starts from LDS.
template <int NT, int E>
struct SortTiers {
  static constexpr int E1 = NT == kWave ? E / 3 : E / 4 + E / 8;
  static constexpr int E2 = NT == kWave ? E : E / 2 + E / 8;
};

// One block per tile: keys (depth bits << 32 | id) are unique within a tile,
// so ascending key order is the (depth, id) order.  Each variant handles the
// tiles whose length lies in (lo_n, hi_n]; a list is held in registers with
// the fewest keys per thread of the tiers that fit it, and longer than
// NT * E -> global memory.
template <int NT, int E>
__global__ __launch_bounds__(NT) void k_sort_tiles(Ws ws, int lo_n, int hi_n, int queued) {
  constexpr int CAP = NT * E;
  constexpr int E1 = SortTiers<NT, E>::E1, E2 = SortTiers<NT, E>::E2;
  constexpr bool kWaveSort = NT == kWave && E <= 15;
  // the keys (padded) and, for up to 15 keys per thread, the threads' bucket
  // starts: separate arrays, so that the compiler sees they never alias
  __shared__ unsigned long long buf[CAP + CAP / 16];
  __shared__ uint32_t starts[8 * NT];
  __shared__ uint32_t wsum[NT / kWave][8];
  __shared__ unsigned long long red[2 * (NT / kWave)];
  // short lists: tile = block; long lists: blocks take queued tiles in turn
  __shared__ int next_s;
  if (queued && *ws.n_long == 0u) return;  // (one load when nothing is queued)
  for (int round = 0;; round++) {
  int tile;
  if (!queued) {
    if (round > 0) break;
    tile = blockIdx.x;
  } else {
    if (threadIdx.x == 0) {
      const uint32_t q = atomicAdd(ws.long_next, 1u);
      next_s = q < *ws.n_long ? (int)ws.long_tiles[q] : -1;
    }
    __syncthreads();
    tile = next_s;
    __syncthreads();
    if (tile < 0) break;
  }
  // ranges are clamped to the capacity, and every position of a clamped
  // range was written by the fill, so sorting stays in bounds on overflow
  const uint2 rg = ws.ranges[tile];
  const int n = (int)(rg.y - rg.x);
  if (n <= lo_n || n > hi_n || n <= 0) continue;
  const unsigned long long *src = ws.keys + rg.x;
  uint32_t *dst = ws.ids + rg.x;
  if (n == 1) {
    if (threadIdx.x == 0) dst[0] = (uint32_t)src[0];
    continue;
  }
  // a list (or run) of c <= CAP keys sorted in LDS, written to d
  auto sort_run = [&](const unsigned long long *s_, auto *d_, int c) {
    if constexpr (kWaveSort) {
      if (c <= NT * E1) wave_sort_tile<E1>(s_, d_, c, buf, starts);
      else wave_sort_tile<E>(s_, d_, c, buf, starts);
    } else {
      if (c <= NT * E1) sort_tile_regs<NT, E1>(s_, d_, c, buf, wsum, red, starts);
      else if (c <= NT * E2) sort_tile_regs<NT, E2>(s_, d_, c, buf, wsum, red, starts);
      else sort_tile_regs<NT, E>(s_, d_, c, buf, wsum, red, starts);
    }
  };
  if (n <= CAP) {
    sort_run(src, dst, n);
  } else {
    // longer than the LDS holds: runs of CAP keys sorted in LDS into
    // keys_tmp, then merged pairwise, back and forth between keys_tmp and
    // the tile's own key range (free once its runs are sorted); the last
    // round writes the ids
    unsigned long long *runs = ws.keys_tmp + rg.x, *spare = ws.keys + rg.x;
    for (int lo = 0; lo < n; lo += CAP) {
      sort_run(src + lo, runs + lo, min(CAP, n - lo));
      __syncthreads();  // buf is reused by the next run
    }
    const unsigned long long *in = runs;
    unsigned long long *out = spare;
    int width = CAP;
    for (; 2 * width < n; width *= 2) {
      merge_round<NT>(in, out, n, width);
      __syncthreads();
      unsigned long long *nxt = const_cast<unsigned long long *>(in);
      in = out;
      out = nxt;
    }
    merge_round<NT>(in, dst, n, width);
  }
  __syncthreads();  // buf is reused by the block's next tile
  }
}

// Device-wide exclusive scan of rec_cnt -> rec_off (3 phases).
constexpr int kRecPer = 8, kRecBlock = kNT * kRecPer;
__global__ __launch_bounds__(kNT) void k_rec_scan_a(Ws ws) {
  __shared__ uint32_t lw[kNT / kWave];
  const int64_t i0 = (int64_t)blockIdx.x * kRecBlock + threadIdx.x * kRecPer;
  uint32_t s = 0;
  for (int k = 0; k < kRecPer; k++)
    if (i0 + k < ws.n_rec) s += ws.rec_cnt[i0 + k];
  uint32_t tot;
  block_exclusive_scan<kNT>(s, lw, &tot);
  if (threadIdx.x == 0) ws.scan_part[blockIdx.x] = tot;
}
__global__ __launch_bounds__(1024) void k_rec_scan_b(Ws ws, int nb) {
  __shared__ uint32_t lw[1024 / kWave];
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < nb ? ws.scan_part[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<1024>(v, lw, &tot);
    if (i < nb) ws.scan_part[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) ws.rec_off[ws.n_rec] = carry;
}
__global__ __launch_bounds__(kNT) void k_rec_scan_c(Ws ws) {
  __shared__ uint32_t lw[kNT / kWave];
  const int64_t i0 = (int64_t)blockIdx.x * kRecBlock + threadIdx.x * kRecPer;
  uint32_t v[kRecPer], s = 0;
  for (int k = 0; k < kRecPer; k++) {
    v[k] = (i0 + k < ws.n_rec) ? ws.rec_cnt[i0 + k] : 0u;
    s += v[k];
  }
  uint32_t pos = ws.scan_part[blockIdx.x] + block_exclusive_scan<kNT>(s, lw, nullptr);
  for (int k = 0; k < kRecPer; k++) {
    if (i0 + k < ws.n_rec) ws.rec_off[i0 + k] = pos;
    pos += v[k];
  }
}

__global__ void k_debug_copy(Ws ws, float *records, int32_t *rect) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ws.n_rec) return;
  if (records) {
    const float4 a = ws.recA[3 * (int64_t)r], b = ws.recA[3 * (int64_t)r + 1],
                 c = ws.recA[3 * (int64_t)r + 2];
    float *o = records + 12 * (int64_t)r;
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
    o[8] = c.x; o[9] = c.y; o[10] = c.z; o[11] = c.w;
  }
  if (rect) {
    int x0, y0, x1, y1;
    unpack_rect(ws.rect[r], x0, y0, x1, y1);
    int32_t *o = rect + 4 * (int64_t)r;
    o[0] = x0; o[1] = y0; o[2] = x1; o[3] = y1;
  }
}

inline unsigned blocks_for(int64_t n, int nt) { return (unsigned)((n + nt - 1) / nt); }

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, kNT)), dim3(kNT), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(n, kNT)), dim3(kNT), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_preprocess(const Ws &ws, hipStream_t st) {
  // at least one block: it bumps the pass counter
  const int64_t nb = ws.n_rec > 0 ? blocks_for(ws.n_rec, kNT) : 1;
  hipLaunchKernelGGL(k_preprocess, dim3(nb), dim3(kNT), 0, st, ws);
  return hipGetLastError();
}


hipError_t launch_scan_tiles(const Ws &ws, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kScanNT), 0, st, ws);
  return hipGetLastError();
}

hipError_t launch_fill_keys(const Ws &ws, hipStream_t st) {
  if (ws.n_rec == 0) return hipSuccess;
  // four records per thread once the grid holds several waves per SIMD
  // at that rate (1,024 SIMDs)
  if (ws.n_rec >= (1 << 20)) {
    hipLaunchKernelGGL(k_fill_keys<4>, dim3(blocks_for(ws.n_rec, 4 * kNT)), dim3(kNT), 0, st, ws);
  } else {
    hipLaunchKernelGGL(k_fill_keys<1>, dim3(blocks_for(ws.n_rec, kNT)), dim3(kNT), 0, st, ws);
  }
  return hipGetLastError();
}

hipError_t launch_sort_tiles(const Ws &ws, hipStream_t st) {
  // Where the records' expected pairs per tile (a Gaussian of extent ~4-5 px
  // covers about (1 + 10 / B)^2 tiles of side B) make long lists the rule,
  // lists of up to 768 go to one wave per tile (4 or 12 keys per lane) and
  // the longer ones, queued by the scan, to 512-thread blocks taken in turn
  // (6, 10 or 16 keys per thread; 8192 keys in LDS, longer lists merged from
  // runs), a CU's worth of them.  Otherwise the one-wave blocks sort every
  // list, a long one (the odd one) as runs of 768 merged in rounds, and no
  // second kernel is launched.
  const double per = (1.0 + 10.0 / ws.tile) * (1.0 + 10.0 / ws.tile);
  const bool many = per * (double)ws.n_rec > 1024.0 * (double)ws.n_tiles;
  hipLaunchKernelGGL((k_sort_tiles<kWave, kSmallSort / kWave>), dim3(ws.n_tiles), dim3(kWave), 0,
                     st, ws, 0, many ? kSmallSort : 0x7fffffff, 0);
  if (many) {
    hipLaunchKernelGGL((k_sort_tiles<512, kSortCap / 512>), dim3(std::min(ws.n_tiles, 512)), dim3(512),
                       0, st, ws, kSmallSort, 0x7fffffff, 1);
  }
  return hipGetLastError();
}

hipError_t launch_scan_records(const Ws &ws, hipStream_t st) {
  const int nb = (int)blocks_for(ws.n_rec, kRecBlock);
  if (nb == 0) return launch_fill_u32(ws.rec_off, 0u, 1, st);
  hipLaunchKernelGGL(k_rec_scan_a, dim3(nb), dim3(kNT), 0, st, ws);
  hipLaunchKernelGGL(k_rec_scan_b, dim3(1), dim3(1024), 0, st, ws, nb);
  hipLaunchKernelGGL(k_rec_scan_c, dim3(nb), dim3(kNT), 0, st, ws);
  return hipGetLastError();
}

int64_t rec_scan_blocks(int64_t n_rec) { return (n_rec + kRecBlock - 1) / kRecBlock; }

hipError_t launch_debug_copy(const Ws &ws, float *records, int32_t *rect, hipStream_t st) {
  if (ws.n_rec == 0) return hipSuccess;
  hipLaunchKernelGGL(k_debug_copy, dim3(blocks_for(ws.n_rec, kNT)), dim3(kNT), 0, st, ws,
                     records, rect);
  return hipGetLastError();
}

}  // namespace vtgs
