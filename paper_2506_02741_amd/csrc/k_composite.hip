// Tile compositing of view-tied Gaussians: forward (RGB, depth, silhouette)
// and its reverse-mode replay.
//
// One workgroup per (view, tile).  Each wave owns a square block of the
// tile (8x8 pixels, or 16x16 for 32-pixel tiles with four pixels per lane).
// The tile's depth-sorted list is walked in batches staged through LDS;
// while staging, the block marks for every wave which entries may reach
// the wave's pixels -- extent box touching its block and block inside the
// entry's cull circle (one 64-bit mask per wave and 64 entries) -- and each
// wave then visits only the set bits of its masks with scalar bit scans,
// four entries per step, recording for each lane which entries reach its
// pixel (q <= q_cut, the exact test).  The lanes then composite their own entries of a
// group of chunks (up to 256 entries) as one stream each, so a wave takes as
// many steps as its busiest lane has entries in the whole group.
//
// Forward, per pixel, front to back [splat of Sec. 3.3]:
//   q = d^T Q d with d = pixel - mu; skip q > q_cut
//   alpha = min(alpha_max, o exp(-q/2)); skip alpha < alpha_min
//   stop before T (1 - alpha) < t_min
//   C += c alpha T, D += z alpha T, T *= (1 - alpha)
//   out: C + T bg, D, 1 - T; keep T_final and the list position past the
//   last contributor for the backward.
//
// Backward replays the same list from the last contributor towards the
// front, recovering T_i = T_{i+1} / (1 - alpha_i).  What lies behind
// contributor i, normalised, is B_i = alpha_b x_b + (1 - alpha_b) B_b with
// b the next contributor behind it and x = (c, z, 1), and B = (bg, 0, 0) at
// the back; only g . (x_i - B_i) enters the gradient, carried per pixel by
// the difference recurrence
//   g.(x_i - B_i) = g.(x_i - x_b) + (1 - alpha_b) g.(x_b - B_b)
// (x_b = (bg, 0, 0) and the second term 0 at the back).  Neighbouring
// colours and depths are close, so their differences are exact or nearly,
// and the result keeps its relative accuracy where x_i and B_i agree (a
// surface seen through Gaussians of its own colour), which a running
// g . B subtracted from g . x_i would lose to cancellation.  Per
// contributing pair:
//   dL/dalpha = T [g_C.(c - B_C) + g_D (z - B_D) + g_S (1 - B_S)] = T g.(x - B)
//   dL/dc = alpha T g_C, dL/dz = alpha T g_D,
//   if o G <= alpha_max: dL/do = G dL/dalpha, dL/dq = -o G dL/dalpha / 2
// and q's dependence on the camera-frame centre p and the radius r
// (mu = proj(p), Sigma = r^2 J J^T + s I, w = Sigma^-1 d, t = J^T w):
//   dq/dr = -2 r |t|^2
//   dq/dp = (-2 t0 + k t0 t2, -2 t1 + k t1 t2, -2 t2 + k (t0^2 + t1^2 + 2 t2^2)),
//   k = 2 r^2 / p_z.
// Mode "twist": dL/dp is chained straight to the view's left twist
// (rho += dL/dp, phi += p x dL/dp) in registers, summed per tile.
// Mode "slots": each lane adds its (dL/dc, dL/do, dL/dr) -- and with
// geometry its dL/dp -- for an entry into its wave's own LDS accumulators
// (LDS atomics, in the wave's program order); after a batch the four waves'
// sums go to the pair's (record, tile) slot, and a gather pass sums a
// record's slots.  Neither mode uses global
// atomics and no two waves share an accumulator, so both are deterministic.
#include <type_traits>

#include "vtgs_internal.h"

namespace vtgs {

namespace {

constexpr float kNegHalfLog2e = -0.72134752044448170368f;  // -log2(e) / 2

// Eq. 1 evaluated inside the tracking backward (on = 0: upstream gradients
// come from the caller's arrays).
struct TrackArgs {
  float alpha, beta, sil_thr;
  int on;
};

__device__ __forceinline__ float sgn(float x) { return (float)((x > 0.f) - (x < 0.f)); }

template <int TILE>
struct Shape {
  static constexpr int NT = TILE == 8 ? 64 : 256;
  static constexpr int PPT = TILE * TILE / NT;  // pixels per lane
  static constexpr int WB = TILE == 32 ? 16 : 8;  // side of a wave's block
};

// Pixel k of this lane, relative to the tile origin.
template <int TILE>
__device__ __forceinline__ void lane_pixel(int k, int &x, int &y) {
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  if (TILE == 8) { x = l % 8; y = l / 8; return; }
  const int qx = (w % 2) * Shape<TILE>::WB, qy = (w / 2) * Shape<TILE>::WB;
  x = qx + l % 8 + 8 * (k % 2);
  y = qy + l / 8 + 8 * (k / 2);
}

// Origin of wave ww's pixel block relative to the tile origin.
template <int TILE>
__device__ __forceinline__ void block_of(int ww, int &x0, int &y0) {
  if (TILE == 8) { x0 = 0; y0 = 0; return; }
  x0 = (ww % 2) * Shape<TILE>::WB;
  y0 = (ww / 2) * Shape<TILE>::WB;
}

// Squared radius of a circle around mu that holds every offset d with
// d^T Q d <= q_cut: |d|^2 <= q_cut / lambda_min(Q) = q_cut lambda_max / det,
// widened by 2 % so that the FP32 value of q can never pass the cut outside
// it.  A conic that is not positive definite gets no circle (box test only).
__device__ __forceinline__ float cull_r2(float qa, float qb, float qc, float qcut) {
  // (hardware square root and reciprocal, ~1 ulp: far inside the 2 %)
  const float h = 0.5f * (qa - qc);
  const float lmax = 0.5f * (qa + qc) + __builtin_amdgcn_sqrtf(fmaf(h, h, qb * qb));
  const float det = fmaf(qa, qc, -qb * qb);
  return det > 0.f ? 1.0201f * qcut * lmax * __builtin_amdgcn_rcpf(det) : 3.0e38f;
}

// Wave masks of a staged batch: bit (i % 64) of masks[ww][i / 64] is set
// when entry i is present and reaches wave ww's pixel block: its extent box
// mu +- R touches the block and the block lies within the cull circle.
// Called by every lane (the ballot is wave-wide); the lanes of a wave stage
// 64 consecutive entries, so i / 64 is uniform.
template <int TILE, int NCH>
__device__ __forceinline__ void stage_masks(unsigned long long (*masks)[NCH], int i, bool have,
                                            const float4 &e0, float qc, float R, float qcut,
                                            float ox, float oy) {
  constexpr int NW = Shape<TILE>::NT / kWave, WB = Shape<TILE>::WB;
  const float r2 = cull_r2(e0.z, e0.w, qc, qcut);
#pragma unroll
  for (int ww = 0; ww < NW; ww++) {
    int x0, y0;
    block_of<TILE>(ww, x0, y0);
    const float bx0 = ox + (float)x0, by0 = oy + (float)y0;
    const float bx1 = bx0 + (float)(WB - 1), by1 = by0 + (float)(WB - 1);
    const bool miss = (e0.x + R < bx0) | (e0.x - R > bx1) | (e0.y + R < by0) | (e0.y - R > by1);
    // distance from mu to the nearest pixel centre of the block
    const float gx = fmaxf(fmaxf(bx0 - e0.x, e0.x - bx1), 0.f);
    const float gy = fmaxf(fmaxf(by0 - e0.y, e0.y - by1), 0.f);
    const bool far = fmaf(gx, gx, gy * gy) > r2;
    const unsigned long long m = ballot64(have && !miss && !far);
    if (lane_id() == 0) masks[ww][i / kWave] = m;
  }
}

__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// First u64 of the lane bits of chunk c of the batch at list offset `boff`
// (a multiple of 64) of tile t, wave w of nw, ppt pixels per lane.  Chunks
// of consecutive tiles never share an index (the tile number is added to
// the list position / 64), and the index stays below cap / 64 + n_tiles + 1.
__device__ __forceinline__ int64_t chunk_word(int start, int boff, int c, int t, int w, int nw,
                                              int ppt) {
  const int64_t cid = (int64_t)(start >> 6) + (boff >> 6) + c + t;
  return ((cid * nw + w) * ppt) * kWave;
}

// q = d^T Q d (d = pixel - mu) in a fixed order, from a staged entry whose
// off-diagonal term is already doubled (e0.w = 2 qb, exact in FP32).
__device__ __forceinline__ float quad2(const float4 &e0, float qc, float px, float py) {
  const float dx = px - e0.x, dy = py - e0.y;
  float q = (e0.z * dx) * dx;
  q = fmaf(e0.w * dx, dy, q);
  q = fmaf(qc * dy, dy, q);
  return q;
}

// Chunks of 64 entries whose lane bits one phase-2 pass walks as a single
// stream per lane (a lane then steps once per entry that reaches its pixel,
// not once per entry of the busiest lane of every chunk).  Four pixels per
// lane keep one chunk per pass to bound the LDS word lists.
template <int TILE, int BATCH>
struct Group {
  static constexpr int NCB = BATCH / kWave;  // chunks of a full batch
  static constexpr int G = Shape<TILE>::PPT > 1 ? 1 : (NCB < 4 ? NCB : 4);
  static constexpr int NS = 2 * G + 2;       // LDS word slots per pixel
};

// Word list of one pixel-lane: the nonzero 32-entry halves of its bits in
// slots 0.., a zero word after the last; `seq` holds each slot's half index
// within the group, four bits per slot, the current slot's in bits 0-3.
template <int NS, int NR>
__device__ __forceinline__ void push_word(uint32_t (*words)[NR][kWave], int row, uint32_t word,
                                          uint32_t half, uint32_t &ns, uint32_t &seq) {
  if (word != 0u) {
    words[ns][row][lane_id()] = word;
    seq |= half << (4u * ns);
    ns++;
  }
}

// Lowest set bit of a word, 31 for a zero word (an index that stays inside
// the group, read and then ignored).
__device__ __forceinline__ int low_bit(uint32_t v) { return __builtin_ctz(v | 0x80000000u); }

// Gather the record of entry `id` of the view.  No branch around the loads
// (so that nothing waits for them before their use): an id out of range,
// which a consistent list never holds, reads record 0 and clears `ok`, and
// the staging then leaves the entry out of every wave's mask.
__device__ __forceinline__ void fetch_record(const Ws &ws, int n_rec, int rec_base, uint32_t id,
                                             float4 &e0, float4 &e1, float4 &e2, bool &ok) {
  ok = id < (uint32_t)n_rec;
  const float4 *A = ws.recA + 3 * ((int64_t)rec_base + (ok ? id : 0u));
  e0 = A[0]; e1 = A[1]; e2 = A[2];
}

template <int TILE, int BATCH>
__global__ __launch_bounds__(Shape<TILE>::NT) void k_fwd(Ws ws, float *out_rgb, float *out_depth,
                                                         float *out_sil) {
  constexpr int NT = Shape<TILE>::NT, PPT = Shape<TILE>::PPT;
  constexpr int NW = NT / kWave;
  constexpr int PER = (BATCH + NT - 1) / NT;  // list entries each thread stages per batch
  constexpr int NCH = PER * NT / kWave;       // 64-entry chunks of a staged batch
  constexpr int G = Group<TILE, BATCH>::G, NS = Group<TILE, BATCH>::NS, NR = NW * PPT;
  __shared__ float4 e0s[BATCH], e1s[BATCH], e2s[BATCH];
  __shared__ unsigned long long masks[NW][NCH];
  __shared__ uint32_t words[NS][NR][kWave];
  const int t = tile_of_block(ws);
  const DevView &vw = ws.views[find_view_by_tile(ws, t)];
  const int lt = t - vw.tile_base;
  const int ox = (lt % vw.tiles_x) * TILE, oy = (lt / vw.tiles_x) * TILE;
  const uint2 rg = ws.ranges[t];
  const int start = (int)rg.x, end = (int)rg.y;
  const int w = threadIdx.x / kWave;

  float px[PPT], py[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT];
  uint32_t last[PPT];
  bool done[PPT], valid[PPT];
#pragma unroll
  for (int k = 0; k < PPT; k++) {
    int x, y;
    lane_pixel<TILE>(k, x, y);
    px[k] = (float)(ox + x);
    py[k] = (float)(oy + y);
    valid[k] = (ox + x) < vw.width && (oy + y) < vw.height;
    done[k] = !valid[k];
    T[k] = 1.f; C0[k] = C1[k] = C2[k] = D[k] = 0.f; last[k] = 0;
  }
  const float amin = ws.amin, amax = ws.amax, tmin = ws.tmin, qcut = ws.qcut;

  auto wave_done = [&]() {
    bool all = true;
#pragma unroll
    for (int k = 0; k < PPT; k++) all &= done[k];
    return ballot64(!all) == 0ull;
  };

  // the next batch's records are gathered into registers while the current
  // batch is composited, and the ids of the batch after it one batch ahead
  // (list positions are clamped to the list; the extra loads go unused)
  float4 p0[PER], p1[PER], p2[PER];
  bool pok[PER];
  uint32_t pid[PER];
  const int n_rec = vw.n_rec, rec_base = vw.rec_base;
  if (end > start) {
#pragma unroll
    for (int k = 0; k < PER; k++) pid[k] = ws.ids[min(start + (int)threadIdx.x + k * NT, end - 1)];
#pragma unroll
    for (int k = 0; k < PER; k++) fetch_record(ws, n_rec, rec_base, pid[k], p0[k], p1[k], p2[k], pok[k]);
#pragma unroll
    for (int k = 0; k < PER; k++)
      pid[k] = ws.ids[min(start + BATCH + (int)threadIdx.x + k * NT, end - 1)];
  }

  for (int b = start; b < end; b += BATCH) {
    bool mine = true;
#pragma unroll
    for (int k = 0; k < PPT; k++) mine &= done[k];
    if (__syncthreads_count(mine) == NT) break;
    const int nb = min(BATCH, end - b);
#pragma unroll
    for (int k = 0; k < PER; k++) {
      const int i = threadIdx.x + k * NT;
      const bool have = i < nb;
      // the off-diagonal conic term is staged doubled (exact in FP32)
      if (have) {
        e0s[i] = make_float4(p0[k].x, p0[k].y, p0[k].z, 2.0f * p0[k].w);
        e1s[i] = p1[k]; e2s[i] = p2[k];
      }
      stage_masks<TILE, NCH>(masks, i, have && pok[k], p0[k], p1[k].x, p1[k].w, qcut, (float)ox,
                             (float)oy);
    }
    __syncthreads();
    // (past the last batch the clamped loads repeat the list's last entry)
#pragma unroll
    for (int k = 0; k < PER; k++) fetch_record(ws, n_rec, rec_base, pid[k], p0[k], p1[k], p2[k], pok[k]);
#pragma unroll
    for (int k = 0; k < PER; k++)
      pid[k] = ws.ids[min(b + 2 * BATCH + (int)threadIdx.x + k * NT, end - 1)];
    if (wave_done()) continue;
    const uint32_t base = (uint32_t)(b - start + 1);
    const int nch = (nb + kWave - 1) / kWave;
    for (int g0 = 0; g0 < nch; g0 += G) {
      uint32_t ns[PPT], seq[PPT];
#pragma unroll
      for (int k = 0; k < PPT; k++) ns[k] = seq[k] = 0u;
      const int cend = min(g0 + G, nch);
      for (int c = g0; c < cend; c++) {
        const unsigned long long m = uniform_u64(masks[w][c]);
        if (m == 0ull) continue;
        // 1. which of the chunk's entries reach each of this lane's pixels
        // bits 0-31 and 32-63 of the chunk in two words; entry j is uniform,
        // so the half it lands in is a scalar choice
        uint32_t own_lo[PPT], own_hi[PPT];
#pragma unroll
        for (int k = 0; k < PPT; k++) own_lo[k] = own_hi[k] = 0u;
        for (int h = 0; h < 2; h++) {
          uint32_t mh = (uint32_t)(m >> (32 * h));
          while (mh) {  // four entries per step, all loads issued first
            // past the last set bit: entry 31 of the half, whose bit the
            // chunk mask clears below unless it is a visited entry anyway
            int j[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
              j[u] = __builtin_ctz(mh | 0x80000000u);
              mh &= mh - 1u;
            }
            float4 a[4];
            float aq[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
              const int ia = c * kWave + 32 * h + j[u];
              a[u] = e0s[ia];
              aq[u] = e1s[ia].x;
            }
#pragma unroll
            for (int k = 0; k < PPT; k++) {
              uint32_t bits = 0u;
#pragma unroll
              for (int u = 0; u < 4; u++)
                bits |= (uint32_t)(quad2(a[u], aq[u], px[k], py[k]) <= qcut) << j[u];
              bits = done[k] ? 0u : bits;
              if (h == 0) own_lo[k] |= bits; else own_hi[k] |= bits;
            }
          }
        }
#pragma unroll
        for (int k = 0; k < PPT; k++) {
          own_lo[k] &= (uint32_t)m;
          own_hi[k] &= (uint32_t)(m >> 32);
        }
        {
          // kept for the backward, which replays the same chunks
          unsigned long long *dst = ws.lane_bits + chunk_word(start, b - start, c, t, w, NW, PPT);
#pragma unroll
          for (int k = 0; k < PPT; k++)
            dst[k * kWave + lane_id()] = ((unsigned long long)own_hi[k] << 32) | own_lo[k];
        }
#pragma unroll
        for (int k = 0; k < PPT; k++) {
          const uint32_t hh = 2u * (uint32_t)(c - g0);
          push_word<NS, NR>(words, w * PPT + k, own_lo[k], hh, ns[k], seq[k]);
          push_word<NS, NR>(words, w * PPT + k, own_hi[k], hh + 1u, ns[k], seq[k]);
        }
      }
      // 2. each lane composites its own entries of the group in list order,
      // one step per entry; the wave runs until its last lane is through
#pragma unroll
      for (int k = 0; k < PPT; k++) {
        const int row = w * PPT + k;
        words[ns[k]][row][lane_id()] = 0u;
        uint32_t cur = words[0][row][lane_id()], nxt = words[1][row][lane_id()];
        uint32_t sq = seq[k], sp = 0u;
        const int gb = g0 * kWave;
        // the next entry's LDS reads are issued before this one is composited
        int i = gb + (int)((sq & 15u) << 5) + low_bit(cur);
        float4 n0 = e0s[i], n1 = e1s[i], n2 = e2s[i];
        while (cur != 0u) {
          const float4 e0 = n0, e1 = n1, e2 = n2;
          const uint32_t pos = base + (uint32_t)i;
          cur &= cur - 1u;
          const bool z = cur == 0u;
          cur = z ? nxt : cur;
          sq = z ? sq >> 4 : sq;
          sp += z ? 1u : 0u;
          nxt = words[sp + 1u][row][lane_id()];
          i = gb + (int)((sq & 15u) << 5) + low_bit(cur);
          n0 = e0s[i]; n1 = e1s[i]; n2 = e2s[i];
          const float q = quad2(e0, e1.x, px[k], py[k]);
          const float gau = __builtin_amdgcn_exp2f(q * kNegHalfLog2e);
          const float a = fminf(amax, e1.y * gau);
          const bool ok = a >= amin;
          const float Tn = T[k] * (1.0f - a);
          const bool stop = ok && (Tn < tmin);
          const bool take = ok && !stop;
          done[k] = done[k] || stop;
          cur = stop ? 0u : cur;
          const float wgt = take ? a * T[k] : 0.f;
          C0[k] = fmaf(e2.x, wgt, C0[k]);
          C1[k] = fmaf(e2.y, wgt, C1[k]);
          C2[k] = fmaf(e2.z, wgt, C2[k]);
          D[k] = fmaf(e1.z, wgt, D[k]);
          T[k] = take ? Tn : T[k];
          last[k] = take ? pos : last[k];
        }
      }
      if (wave_done()) break;
    }
  }
  const int64_t P = ws.P;
#pragma unroll
  for (int k = 0; k < PPT; k++) {
    if (!valid[k]) continue;
    const int64_t p = vw.pix_off + (int64_t)((int)py[k]) * vw.width + (int)px[k];
    if (out_rgb) {
      out_rgb[p] = fmaf(T[k], ws.bg[0], C0[k]);
      out_rgb[P + p] = fmaf(T[k], ws.bg[1], C1[k]);
      out_rgb[2 * P + p] = fmaf(T[k], ws.bg[2], C2[k]);
    }
    if (out_depth) out_depth[p] = D[k];
    if (out_sil) out_sil[p] = 1.0f - T[k];
    ws.t_final[p] = T[k];
    ws.last[p] = last[k];
  }
}

// Backward staging of one list entry: the forward record, the camera-frame
// centre and learnable flag, and (slot mode) the record's tile rectangle and
// first slot.  Gathered without branches, as in the forward.
struct BwdEntry {
  float4 e0, e1, e2, eb;
  uint2 rc;
  uint32_t off;
  bool ok;
};

template <bool kSlots>
__device__ __forceinline__ void fetch_bwd_entry(const Ws &ws, int n_rec, int rec_base, uint32_t id,
                                                BwdEntry &E) {
  E.ok = id < (uint32_t)n_rec;
  const int64_t rec = (int64_t)rec_base + (E.ok ? id : 0u);
  const float4 *A = ws.recA + 3 * rec;
  E.e0 = A[0]; E.e1 = A[1]; E.e2 = A[2];
  E.eb = ws.recB[rec];
  if (kSlots) { E.rc = ws.rect[rec]; E.off = ws.rec_off[rec]; }
}

// The (record, tile) slot of a staged entry of tile (tx, ty), or ~0u when
// it has none (an id out of range, or past the capacity after an overflow).
__device__ __forceinline__ uint32_t entry_slot(const Ws &ws, const BwdEntry &E, int tx, int ty) {
  const int x0 = E.rc.x & 0xffff, y0 = E.rc.x >> 16, x1 = E.rc.y & 0xffff;
  const uint32_t sl = E.off + (uint32_t)((ty - y0) * (x1 - x0 + 1) + (tx - x0));
  return E.ok && sl < (uint64_t)ws.cap ? sl : 0xffffffffu;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
// LDS pointers
#define LDS_AS __attribute__((address_space(3)))
// An empty statement that the compiler must take as reading and writing all
// memory: LDS accesses keep their program order across it (and the LDS
// keeps a wave's order).
__device__ __forceinline__ void kLdsOrder() { asm volatile("" ::: "memory"); }
// The accumulator floats past the first four: one (dL/dr) or, with
// geometry, four (dL/dr, dL/dp).
template <bool kGeo>
using AccB = typename std::conditional<kGeo, f32x4, float>::type;

// Slot modes hold three waves per SIMD (their LDS allows three blocks per CU)
// unless they carry geometry (two).
template <int TILE, int BATCH, int MODE>
__global__ __launch_bounds__(Shape<TILE>::NT, (MODE & 2) ? ((MODE & 4) ? 2 : 3) : 1) void k_bwd(Ws ws, const float *g_rgb,
                                                         const float *g_depth,
                                                         const float *g_sil, TrackArgs tr) {
  constexpr int NT = Shape<TILE>::NT, PPT = Shape<TILE>::PPT;
  constexpr int NW = NT / kWave;
  constexpr int PER = (BATCH + NT - 1) / NT;
  constexpr int NCH = PER * NT / kWave;
  constexpr bool kTwist = (MODE & 1) != 0, kSlots = (MODE & 2) != 0;
  constexpr bool kGeo = kSlots && (MODE & 4) != 0;  // slots also carry dL/dp
  constexpr int NA = kGeo ? 8 : 5;                   // floats per slot
  constexpr int AB = kSlots ? BATCH : 1;
  constexpr int G = Group<TILE, BATCH>::G, NS = Group<TILE, BATCH>::NS, NR = NW * PPT;
  // staged entry: e0 (mx, my, qa, 2 qb), e1 (qc, o, z, qb), e2 (c, r)
  __shared__ float4 e0s[BATCH], e1s[BATCH], e2s[BATCH];
  __shared__ float4 ejs[BATCH];   // (fx/z, fy/z, -fx px/z^2, -fy py/z^2)
  __shared__ float4 eps_[BATCH];  // (px, py, 2 r^2 / z, learnable)
  __shared__ uint32_t slot_s[AB];
  // per-wave slot accumulators: floats 0-3 in accA, 4 (4-7 with geometry)
  // in accB, and the claim tags of their read-modify-write
  __shared__ f32x4 accA[NW][AB];
  __shared__ AccB<kGeo> accB[NW][AB];
  __shared__ uint8_t tag_s[kSlots ? NW : 1][AB + kWave];  // + a tag per lane
  __shared__ int maxlast_s;
  __shared__ float red_s[NW][7];
  __shared__ unsigned long long masks[NW][NCH];
  __shared__ uint32_t words[NS][NR][kWave];

  const int t = tile_of_block(ws);
  const DevView &vw = ws.views[find_view_by_tile(ws, t)];
  const int lt = t - vw.tile_base;
  const int tx = lt % vw.tiles_x, ty = lt / vw.tiles_x;
  const int ox = tx * TILE, oy = ty * TILE;
  const uint2 rg = ws.ranges[t];
  const int start = (int)rg.x, end = (int)rg.y;
  const int64_t P = ws.P;
  const int w = threadIdx.x / kWave;

  float px[PPT], py[PPT], T[PPT], gC0[PPT], gC1[PPT], gC2[PPT], gD[PPT], gS[PPT];
  // the difference recurrence: (1 - alpha_b) g.(x_b - B_b) of the
  // contributor b behind (0 at the back), its colour and depth (the
  // background and 0 at the back) and g_S (1 - its coverage x_S)
  float E[PPT], XP0[PPT], XP1[PPT], XP2[PPT], XPZ[PPT], GS1[PPT];
  uint32_t last[PPT];
  uint32_t mylast = 0;
  float lsum = 0.f;  // this lane's share of the tile's Eq. 1 loss
#pragma unroll
  for (int k = 0; k < PPT; k++) {
    int x, y;
    lane_pixel<TILE>(k, x, y);
    px[k] = (float)(ox + x);
    py[k] = (float)(oy + y);
    const bool valid = (ox + x) < vw.width && (oy + y) < vw.height;
    const int64_t p = vw.pix_off + (int64_t)(oy + y) * vw.width + (ox + x);
    T[k] = valid ? ws.t_final[p] : 1.f;
    last[k] = valid ? ws.last[p] : 0u;
    if (tr.on) {
      // Eq. 1: alpha W |V - V'| + beta W |D - D'|, W = vis & (D > 0) & (S' > thr)
      const int64_t lp = p - vw.pix_off;
      const int64_t Pv = (int64_t)vw.width * vw.height;
      float od = 0.f;
      bool W = false;
      if (valid) {
        od = vw.obs_depth[lp];
        W = (!vw.vis || vw.vis[lp] != 0) && od > 0.f && ws.img[4 * P + p] > tr.sil_thr;
      }
      const float r0 = valid ? vw.obs_rgb[lp] - ws.img[p] : 0.f;
      const float r1 = valid ? vw.obs_rgb[Pv + lp] - ws.img[P + p] : 0.f;
      const float r2 = valid ? vw.obs_rgb[2 * Pv + lp] - ws.img[2 * P + p] : 0.f;
      const float rd = valid ? od - ws.img[3 * P + p] : 0.f;
      gC0[k] = W ? -tr.alpha * sgn(r0) : 0.f;
      gC1[k] = W ? -tr.alpha * sgn(r1) : 0.f;
      gC2[k] = W ? -tr.alpha * sgn(r2) : 0.f;
      gD[k] = W ? -tr.beta * sgn(rd) : 0.f;
      gS[k] = 0.f;
      lsum += W ? tr.alpha * ((fabsf(r0) + fabsf(r1)) + fabsf(r2)) + tr.beta * fabsf(rd) : 0.f;
    } else {
      gC0[k] = (valid && g_rgb) ? g_rgb[p] : 0.f;
      gC1[k] = (valid && g_rgb) ? g_rgb[P + p] : 0.f;
      gC2[k] = (valid && g_rgb) ? g_rgb[2 * P + p] : 0.f;
      gD[k] = (valid && g_depth) ? g_depth[p] : 0.f;
      gS[k] = (valid && g_sil) ? g_sil[p] : 0.f;
    }
    E[k] = 0.f;
    XP0[k] = ws.bg[0]; XP1[k] = ws.bg[1]; XP2[k] = ws.bg[2]; XPZ[k] = 0.f;
    GS1[k] = gS[k];
    mylast = max(mylast, last[k]);
  }
  if (threadIdx.x == 0) maxlast_s = 0;
  __syncthreads();
  atomicMax(&maxlast_s, (int)mylast);
  __syncthreads();
  const int stop = start + maxlast_s;
  // this wave's own last contributor: entries past it touch none of its lanes
  const int wstop = start + __builtin_amdgcn_readfirstlane(wave_max_i((int)mylast));

  float tw[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  const float amin = ws.amin, amax = ws.amax, qcut = ws.qcut;
  const float vfx = vw.fx, vfy = vw.fy;

  // batches walk the list from the block's last contributor towards the front
  // batches on the forward's grid (start + multiples of BATCH), so each
  // 64-entry chunk is the forward's chunk and its lane bits apply
  const int nbat = (stop - start + BATCH - 1) / BATCH;
  // the batch below is gathered while the current one is replayed, and its
  // ids one batch ahead (positions clamped to the list, extra loads unused)
  BwdEntry st[PER];
  uint32_t pid[PER];
  const int n_rec = vw.n_rec, rec_base = vw.rec_base;
  // position of this thread's entry k in the batch starting at `blo`,
  // clamped to the list (batches below the first repeat its first entry)
  auto bpos = [&](int blo, int k) {
    return max(blo + min((int)threadIdx.x + k * NT, BATCH - 1), start);
  };
  if (nbat > 0) {
    const int lo = start + (nbat - 1) * BATCH;
#pragma unroll
    for (int k = 0; k < PER; k++) pid[k] = ws.ids[min(lo + (int)threadIdx.x + k * NT, stop - 1)];
#pragma unroll
    for (int k = 0; k < PER; k++) fetch_bwd_entry<kSlots>(ws, n_rec, rec_base, pid[k], st[k]);
#pragma unroll
    for (int k = 0; k < PER; k++) pid[k] = ws.ids[bpos(lo - BATCH, k)];
  }
  for (int bi = nbat - 1; bi >= 0; bi--) {
    const int lo = start + bi * BATCH;
    const int nb = min(stop, lo + BATCH) - lo;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; k++) {
      const int i = threadIdx.x + k * NT;
      stage_masks<TILE, NCH>(masks, i, i < nb && st[k].ok, st[k].e0, st[k].e1.x, st[k].e1.w, qcut,
                             (float)ox, (float)oy);
      if (i >= nb) continue;
      const BwdEntry &E = st[k];
      // the doubled off-diagonal conic term (exact) for q, the plain one
      // (in place of the extent, which staging no longer needs) for dq
      e0s[i] = make_float4(E.e0.x, E.e0.y, E.e0.z, 2.0f * E.e0.w);
      e1s[i] = make_float4(E.e1.x, E.e1.y, E.e1.z, E.e0.w);
      e2s[i] = E.e2;
      const float iz = 1.0f / E.e1.z;
      ejs[i] = make_float4(vfx * iz, vfy * iz, -vfx * E.eb.x * iz * iz, -vfy * E.eb.y * iz * iz);
      const uint32_t sl = kSlots ? entry_slot(ws, E, tx, ty) : 0xffffffffu;
      // no slot (only after a capacity overflow): the entry learns nothing
      const float learn = !kSlots || sl != 0xffffffffu ? E.eb.z : 0.f;
      eps_[i] = make_float4(E.eb.x, E.eb.y, 2.0f * E.e2.w * E.e2.w * iz, learn);
      if (kSlots) {
        slot_s[i] = sl;
#pragma unroll
        for (int ww = 0; ww < NW; ww++) {
          accA[ww][i] = f32x4{0.f, 0.f, 0.f, 0.f};
          accB[ww][i] = AccB<kGeo>{};
        }
      }
    }
    __syncthreads();
    // the batches below are full ones (below the first: clamped, unused)
#pragma unroll
    for (int k = 0; k < PER; k++) fetch_bwd_entry<kSlots>(ws, n_rec, rec_base, pid[k], st[k]);
#pragma unroll
    for (int k = 0; k < PER; k++) pid[k] = ws.ids[bpos(lo - 2 * BATCH, k)];
    // this wave's entries, last to first, below its own last contributor
    const int lim = min(nb, wstop - lo);
    const int ctop = (lim - 1) / kWave;
    for (int g0 = (ctop / G) * G; lim > 0 && g0 >= 0; g0 -= G) {
      // 1. the entries of the group's chunks that reached each of this lane's
      // pixels in the forward, cut at the pixel's last contributor; the words
      // go in bit-reversed, top half first, so the lowest set bit of a word is
      // the lane's next entry towards the front
      uint32_t ns[PPT], seq[PPT];
#pragma unroll
      for (int k = 0; k < PPT; k++) ns[k] = seq[k] = 0u;
      // the group's lane bits, all loads issued at once (chunks past the top
      // one reload the top one's, unused)
      unsigned long long lb[G][PPT];
#pragma unroll
      for (int cc = 0; cc < G; cc++) {
        const unsigned long long *src =
            ws.lane_bits + chunk_word(start, lo - start, min(g0 + cc, ctop), t, w, NW, PPT);
#pragma unroll
        for (int k = 0; k < PPT; k++) lb[cc][k] = src[k * kWave + lane_id()];
      }
#pragma unroll
      for (int cc = G - 1; cc >= 0; cc--) {
        const int c = g0 + cc;
        if (c > ctop) continue;
        unsigned long long m = uniform_u64(masks[w][c]);
        const int top = lim - c * kWave;  // entries [c*64, c*64 + top) are below the limit
        if (top < kWave) m &= (1ull << top) - 1ull;
        if (m == 0ull) continue;
        const int base = lo - start + c * kWave;
#pragma unroll
        for (int k = 0; k < PPT; k++) {
          const int lim_k = (int)last[k] - base;
          const unsigned long long below =
              lim_k >= kWave ? ~0ull : (lim_k <= 0 ? 0ull : (1ull << lim_k) - 1ull);
          const unsigned long long own = lb[cc][k] & below & m;
          const uint32_t hh = 2u * (uint32_t)(c - g0);
          push_word<NS, NR>(words, w * PPT + k, __builtin_bitreverse32((uint32_t)(own >> 32)),
                            hh + 1u, ns[k], seq[k]);
          push_word<NS, NR>(words, w * PPT + k, __builtin_bitreverse32((uint32_t)own), hh,
                            ns[k], seq[k]);
        }
      }
      // 2. each lane replays its own entries of the group, last to first, one
      // step per entry; the wave runs until its last lane is through
#pragma unroll
      for (int k = 0; k < PPT; k++) {
        const int row = w * PPT + k;
        words[ns[k]][row][lane_id()] = 0u;
        uint32_t cur = words[0][row][lane_id()], nxt = words[1][row][lane_id()];
        uint32_t sq = seq[k], sp = 0u;
        const int gb = g0 * kWave + 31;
        // the next entry's LDS reads are issued before this one is replayed
        int i = gb + (int)((sq & 15u) << 5) - low_bit(cur);
        float4 n0 = e0s[i], n1 = e1s[i], n2 = e2s[i], nj = ejs[i], np = eps_[i];
        // Slots (mapping): each lane's adds of a step go into its wave's
        // accumulators by read-modify-write.  The lanes that replay one
        // entry in a step claim it by writing their lane number to its tag;
        // with the claim they read the tag back and the accumulators.  The
        // claim is settled in the lane's next step, after that step's
        // arithmetic has covered the reads' latency: the lane whose number
        // stayed in the tag (one per entry) adds what it read to its values
        // and writes them back, and the lanes that lost then add theirs with
        // LDS float atomics (6 % of the lane steps of a mapping wave, against
        // all of them with atomics alone, which the LDS runs at about a lane
        // per three clocks).  A lane runs one idle step after its last entry
        // to settle its last claim.  Compiler barriers (kLdsOrder) keep each
        // claim and settle in its step and in program order.
        bool pp = false;  // an open claim (values pva/pvb for entry pidx)
        int pidx = 0, rt = 0;
        f32x4 pva = {0.f, 0.f, 0.f, 0.f}, ra = {0.f, 0.f, 0.f, 0.f};
        AccB<kGeo> pvb{}, rb{};
        const int me = lane_id();
        // a claim: tag slot `ti` claimed, then read back with entry j's
        // accumulators
        auto claim = [&](int ti, int j) {
          uint8_t LDS_AS *tg = (uint8_t LDS_AS *)&tag_s[w][ti];
          *tg = (uint8_t)me;
          kLdsOrder();
          rt = *tg;
          ra = *(f32x4 LDS_AS *)&accA[w][j];
          rb = *(AccB<kGeo> LDS_AS *)&accB[w][j];
          kLdsOrder();
        };
        // the loop is entered, as it is re-entered, with a claim's LDS
        // operations behind the first entry's reads (here one on the lane's
        // own tag, not settled)
        if constexpr (kSlots) claim(AB + me, 0);
        while (cur != 0u || (kSlots && pp)) {
          const bool live = !kSlots || cur != 0u;
          const float4 e0 = n0, e1 = n1, e2 = n2, ej = nj, ep = np;
          const int cur_i = i;  // this entry's batch position
          {
            uint32_t c2 = cur & (cur - 1u);
            const bool z = c2 == 0u;
            c2 = z ? nxt : c2;
            cur = live ? c2 : cur;
            sq = live && z ? sq >> 4 : sq;
            sp += live && z ? 1u : 0u;
          }
          nxt = words[sp + 1u][row][lane_id()];
          i = gb + (int)((sq & 15u) << 5) - low_bit(cur);
          n0 = e0s[i]; n1 = e1s[i]; n2 = e2s[i]; nj = ejs[i]; np = eps_[i];
          const float dx = px[k] - e0.x, dy = py[k] - e0.y;
          const float q = quad2(e0, e1.x, px[k], py[k]);
          const float gau = __builtin_amdgcn_exp2f(q * kNegHalfLog2e);
          const float a = fminf(amax, e1.y * gau);
          const bool ok = live && a >= amin;
          const float oG = e1.y * gau;
          const float om = 1.0f - a;
          const float Tk = ok ? T[k] * __builtin_amdgcn_rcpf(om) : T[k];
          T[k] = Tk;
          const float wgt = ok ? a * Tk : 0.f;
          // g . (x - B) for this Gaussian, x = (colour, depth, 1)
          const float gdi =
              fmaf(gC0[k], e2.x - XP0[k],
                   fmaf(gC1[k], e2.y - XP1[k],
                        fmaf(gC2[k], e2.z - XP2[k], fmaf(gD[k], e1.z - XPZ[k], GS1[k] + E[k]))));
          const float dLda = ok ? gdi * Tk : 0.f;
          E[k] = ok ? om * gdi : E[k];
          XP0[k] = ok ? e2.x : XP0[k];
          XP1[k] = ok ? e2.y : XP1[k];
          XP2[k] = ok ? e2.z : XP2[k];
          XPZ[k] = ok ? e1.z : XPZ[k];
          GS1[k] = ok ? 0.f : GS1[k];
          const bool pass = oG <= amax;
          const float dLdq = pass ? -0.5f * oG * dLda : 0.f;
          const float qb = e1.w;
          const float w0 = fmaf(e0.z, dx, qb * dy), w1 = fmaf(qb, dx, e1.x * dy);
          const float t0 = ej.x * w0, t1 = ej.y * w1, t2 = fmaf(ej.z, w0, ej.w * w1);
          // dL/dp of this pair (camera-frame centre)
          float g0v = 0.f, g1v = 0.f, g2v = 0.f;
          if (kTwist || kGeo) {
            const float kk = ep.z;
            g0v = dLdq * fmaf(kk * t0, t2, -2.0f * t0);
            g1v = dLdq * fmaf(kk * t1, t2, -2.0f * t1);
            const float s2 = fmaf(t0, t0, fmaf(t1, t1, 2.0f * t2 * t2));
            g2v = fmaf(dLdq, fmaf(kk, s2, -2.0f * t2), wgt * gD[k]);
          }
          if (kTwist && live) {
            const float pz = e1.z;
            tw[0] += g0v; tw[1] += g1v; tw[2] += g2v;
            tw[3] += ep.y * g2v - pz * g1v;
            tw[4] += pz * g0v - ep.x * g2v;
            tw[5] += ep.x * g1v - ep.y * g0v;
          }
          if constexpr (kSlots) {
            // this step's values
            const bool real = ok && ep.w != 0.f;
            const float tt = fmaf(t0, t0, fmaf(t1, t1, t2 * t2));
            const f32x4 nva = {wgt * gC0[k], wgt * gC1[k], wgt * gC2[k], pass ? gau * dLda : 0.f};
            const float v4 = dLdq * (-2.0f * e2.w * tt);
            AccB<kGeo> nvb;
            if constexpr (kGeo) nvb = f32x4{v4, g0v, g1v, g2v};
            else nvb = v4;
            // the settle below waits for the previous claim's reads: after
            // the step's arithmetic (which this empty statement consumes)
            asm volatile("" ::"v"(nva[0]), "v"(nva[1]), "v"(nva[2]), "v"(nva[3]), "v"(v4) : "memory");
            // settle the previous step's claim: the lane whose number stayed
            // in the tag writes its sum back; then the lanes that lost add
            // theirs with LDS atomics (after that write, in the LDS's order)
            const bool won = pp && rt == me;
            if (won) {
              *(f32x4 LDS_AS *)&accA[w][pidx] = ra + pva;
              *(AccB<kGeo> LDS_AS *)&accB[w][pidx] = rb + pvb;
            }
            kLdsOrder();
            if (pp && !won) {
              float *fa = (float *)&accA[w][pidx];
              float *fb = (float *)&accB[w][pidx];
              atomicAdd(fa + 0, pva[0]);
              atomicAdd(fa + 1, pva[1]);
              atomicAdd(fa + 2, pva[2]);
              atomicAdd(fa + 3, pva[3]);
              if constexpr (kGeo) {
#pragma unroll
                for (int c = 0; c < 4; c++) atomicAdd(fb + c, pvb[c]);
              } else {
                atomicAdd(fb, pvb);
              }
            }
            kLdsOrder();
            // this step's claim; every lane makes one (a lane with nothing to
            // add on its own tag), so that the LDS operations behind the next
            // entry's reads are the same on every path and the next step
            // waits for those reads only
            pp = ok && ep.w != 0.f;
            pva = nva;
            pvb = nvb;
            pidx = cur_i;
            claim(pp ? cur_i : AB + me, cur_i);
          }
        }
      }
    }
    if (kSlots) {
      __syncthreads();
      for (int i = threadIdx.x; i < nb; i += NT) {
        if (eps_[i].w == 0.f) continue;
        float *o = ws.slots + NA * (int64_t)slot_s[i];
        f32x4 sa = accA[0][i];
        AccB<kGeo> sb = accB[0][i];
#pragma unroll
        for (int ww = 1; ww < NW; ww++) {
          sa = sa + accA[ww][i];
          sb = sb + accB[ww][i];
        }
#pragma unroll
        for (int c = 0; c < 4; c++) o[c] = sa[c];
        if constexpr (kGeo) {
#pragma unroll
          for (int c = 0; c < 4; c++) o[4 + c] = sb[c];
        } else {
          o[4] = sb;
        }
      }
    }
  }
  if (kSlots) {
    // list entries past every pixel's last contributor: zero slots
    for (int i = stop + (int)threadIdx.x; i < end; i += NT) {
      BwdEntry E;
      fetch_bwd_entry<true>(ws, n_rec, rec_base, ws.ids[i], E);
      const uint32_t sl = entry_slot(ws, E, tx, ty);
      if (sl == 0xffffffffu) continue;
      float *o = ws.slots + NA * (int64_t)sl;
#pragma unroll
      for (int c = 0; c < NA; c++) o[c] = 0.f;
    }
  }
  if (kTwist) {
    // per tile: the six twist sums and (tracking) the Eq. 1 loss
#pragma unroll
    for (int c = 0; c < 6; c++) {
      const float s = wave_sum(tw[c]);
      if (lane_id() == 0) red_s[w][c] = s;
    }
    const float ls = wave_sum(lsum);
    if (lane_id() == 0) red_s[w][6] = ls;
    __syncthreads();
    if (threadIdx.x < 7) {
      float s = 0.f;
#pragma unroll
      for (int ww = 0; ww < NW; ww++) s += red_s[ww][threadIdx.x];
      ws.twist_part[8 * (int64_t)t + threadIdx.x] = s;
    }
  }
}

template <int TILE, int BATCH>
hipError_t fwd_launch(const Ws &ws, float *rgb, float *depth, float *sil, hipStream_t st) {
  hipLaunchKernelGGL((k_fwd<TILE, BATCH>), dim3(ws.n_tiles), dim3(Shape<TILE>::NT), 0, st, ws,
                     rgb, depth, sil);
  return hipGetLastError();
}

template <int TILE, int BATCH>
hipError_t bwd_launch(const Ws &ws, const float *g_rgb, const float *g_depth, const float *g_sil,
                      int mode, hipStream_t st, TrackArgs tr) {
  const dim3 g(ws.n_tiles), b(Shape<TILE>::NT);
  switch (mode) {
    case 1: hipLaunchKernelGGL((k_bwd<TILE, BATCH, 1>), g, b, 0, st, ws, g_rgb, g_depth, g_sil, tr); break;
    case 2: hipLaunchKernelGGL((k_bwd<TILE, BATCH, 2>), g, b, 0, st, ws, g_rgb, g_depth, g_sil, tr); break;
    case 3: hipLaunchKernelGGL((k_bwd<TILE, BATCH, 3>), g, b, 0, st, ws, g_rgb, g_depth, g_sil, tr); break;
    case 6: hipLaunchKernelGGL((k_bwd<TILE, BATCH, 6>), g, b, 0, st, ws, g_rgb, g_depth, g_sil, tr); break;
    case 7: hipLaunchKernelGGL((k_bwd<TILE, BATCH, 7>), g, b, 0, st, ws, g_rgb, g_depth, g_sil, tr); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TILE>
hipError_t fwd_tile(const Ws &ws, float *rgb, float *depth, float *sil, hipStream_t st) {
  switch (ws.batch) {
    case 128: return fwd_launch<TILE, 128>(ws, rgb, depth, sil, st);
    case 256: return fwd_launch<TILE, 256>(ws, rgb, depth, sil, st);
    case 512: return fwd_launch<TILE, 512>(ws, rgb, depth, sil, st);
  }
  return hipErrorInvalidValue;
}

template <int TILE>
hipError_t bwd_tile(const Ws &ws, const float *a, const float *b, const float *c, int mode,
                    hipStream_t st, TrackArgs tr) {
  switch (ws.batch) {
    case 128: return bwd_launch<TILE, 128>(ws, a, b, c, mode, st, tr);
    case 256: return bwd_launch<TILE, 256>(ws, a, b, c, mode, st, tr);
    case 512: return bwd_launch<TILE, 512>(ws, a, b, c, mode, st, tr);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_composite_fwd(const Ws &ws, float *rgb, float *depth, float *sil,
                                hipStream_t st) {
  if (ws.n_tiles == 0) return hipSuccess;
  switch (ws.tile) {
    case 8: return fwd_tile<8>(ws, rgb, depth, sil, st);
    case 16: return fwd_tile<16>(ws, rgb, depth, sil, st);
    case 32: return fwd_tile<32>(ws, rgb, depth, sil, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_composite_bwd(const Ws &ws, const float *g_rgb, const float *g_depth,
                                const float *g_sil, int mode, hipStream_t st,
                                const vtgs_track_cfg *track) {
  if (ws.n_tiles == 0) return hipSuccess;
  TrackArgs tr{0.f, 0.f, 0.f, 0};
  if (((mode & 4) != 0) != (ws.slot_w == 8) && (mode & 2)) return hipErrorInvalidValue;
  if (track) {
    if (mode != 1) return hipErrorInvalidValue;
    tr = TrackArgs{track->alpha, track->beta, track->sil_thr, 1};
  }
  switch (ws.tile) {
    case 8: return bwd_tile<8>(ws, g_rgb, g_depth, g_sil, mode, st, tr);
    case 16: return bwd_tile<16>(ws, g_rgb, g_depth, g_sil, mode, st, tr);
    case 32: return bwd_tile<32>(ws, g_rgb, g_depth, g_sil, mode, st, tr);
  }
  return hipErrorInvalidValue;
}

}  // namespace vtgs
