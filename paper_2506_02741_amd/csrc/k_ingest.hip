// Keyframe ingestion: a view-tied Gaussian at every valid depth pixel of the
// stride grid (Sec. 3.2), radius initialised to stride * depth / focal
// length (App. A); the complement mask of pixels the current Gaussians leave
// uncovered (Sec. 3.4).  Stream compaction in row-major order: per-block counts,
// a single-block scan of the block counts, then an order-preserving fill.
#include "vtgs_internal.h"

namespace vtgs {

namespace {
constexpr int kNT = 256;
constexpr int kPer = 4;                 // grid cells per thread
constexpr int kCells = kNT * kPer;      // grid cells per block

__device__ __forceinline__ bool valid_cell(const float *depth, const uint8_t *mask, int H, int W,
                                           int s, int nx, int64_t M, int64_t c, int64_t *pix) {
  if (c >= M) return false;
  const int gy = (int)(c / nx), gx = (int)(c - (int64_t)gy * nx);
  const int64_t p = (int64_t)(gy * s) * W + gx * s;
  *pix = p;
  const float d = depth[p];
  return d > 0.f && d <= 3.402823466e38f && (!mask || mask[p] != 0);
}

__global__ __launch_bounds__(kNT) void k_ingest_counts(const float *depth, const uint8_t *mask,
                                                       int H, int W, int s, int nx, int64_t M,
                                                       uint32_t *block_counts) {
  __shared__ uint32_t lw[kNT / kWave];
  uint32_t n = 0;
  const int64_t c0 = (int64_t)blockIdx.x * kCells + threadIdx.x * kPer;
  for (int k = 0; k < kPer; k++) {
    int64_t p;
    n += valid_cell(depth, mask, H, W, s, nx, M, c0 + k, &p) ? 1u : 0u;
  }
  uint32_t tot;
  block_exclusive_scan<kNT>(n, lw, &tot);
  if (threadIdx.x == 0) block_counts[blockIdx.x] = tot;
}

// One block: exclusive scan of the block counts, total to *count.
__global__ __launch_bounds__(1024) void k_ingest_scan(const uint32_t *block_counts, int nb,
                                                      uint32_t *block_off, int32_t *count) {
  __shared__ uint32_t lw[1024 / kWave];
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < nb ? block_counts[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<1024>(v, lw, &tot);
    if (i < nb) block_off[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *count = (int32_t)carry;
}

__global__ __launch_bounds__(kNT) void k_ingest_fill(const float *depth, const float *rgb,
                                                     const uint8_t *mask, int H, int W, int s,
                                                     int nx, int64_t M, float fx, float o_init,
                                                     const uint32_t *block_off, int n,
                                                     uint32_t *pix, float *dep, float *col,
                                                     float *opa, float *rad) {
  __shared__ uint32_t lw[kNT / kWave];
  const int64_t c0 = (int64_t)blockIdx.x * kCells + threadIdx.x * kPer;
  bool ok[kPer];
  int64_t pp[kPer];
  uint32_t cnt = 0;
  for (int k = 0; k < kPer; k++) {
    ok[k] = valid_cell(depth, mask, H, W, s, nx, M, c0 + k, &pp[k]);
    cnt += ok[k] ? 1u : 0u;
  }
  uint32_t i = block_off[blockIdx.x] + block_exclusive_scan<kNT>(cnt, lw, nullptr);
  const int64_t P = (int64_t)H * W;
  for (int k = 0; k < kPer; k++) {
    if (!ok[k]) continue;
    if ((int)i < n) {
      const float d = depth[pp[k]];
      pix[i] = (uint32_t)pp[k];
      dep[i] = d;
      if (rgb)
        for (int c = 0; c < 3; c++) col[(int64_t)c * n + i] = rgb[c * P + pp[k]];
      opa[i] = o_init;
      rad[i] = __fdiv_rn((float)s * d, fx);
    }
    i++;
  }
}

inline void grid_dims(int H, int W, int s, int *nx, int64_t *M, int *nb) {
  *nx = (W + s - 1) / s;
  const int ny = (H + s - 1) / s;
  *M = (int64_t)*nx * ny;
  *nb = (int)((*M + kCells - 1) / kCells);
}

// Complement initialisation (Sec. 3.4): a pixel is left uncovered by the
// current Gaussians when the silhouette of their rendering there is below
// thr, and gets a new Gaussian if its depth is valid.
__global__ __launch_bounds__(kNT) void k_uncovered(const float *sil, const float *depth, int64_t n,
                                                   float thr, uint8_t *mask) {
  const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (i >= n) return;
  const float d = depth[i];
  mask[i] = (uint8_t)(sil[i] < thr && d > 0.f && d <= 3.402823466e38f);
}
}  // namespace

hipError_t launch_uncovered(const float *sil, const float *depth, int64_t n, float thr,
                            uint8_t *mask, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_uncovered, dim3((unsigned)((n + kNT - 1) / kNT)), dim3(kNT), 0, st, sil,
                     depth, n, thr, mask);
  return hipGetLastError();
}

int64_t ingest_scratch_words(int H, int W, int s) {
  int nx, nb;
  int64_t M;
  grid_dims(H, W, s, &nx, &M, &nb);
  return 2 * (int64_t)nb + 2;
}

hipError_t launch_ingest_count(const float *depth, const uint8_t *mask, int H, int W, int s,
                               uint32_t *scratch, int32_t *count, hipStream_t st) {
  int nx, nb;
  int64_t M;
  grid_dims(H, W, s, &nx, &M, &nb);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ingest_counts, dim3(nb), dim3(kNT), 0, st, depth, mask, H, W, s, nx, M,
                     scratch);
  hipLaunchKernelGGL(k_ingest_scan, dim3(1), dim3(1024), 0, st, scratch, nb, scratch + nb, count);
  return hipGetLastError();
}

hipError_t launch_ingest_fill(const float *depth, const float *rgb, const uint8_t *mask, int H,
                              int W, int s, float fx, float o_init, const uint32_t *scratch,
                              int n, uint32_t *pix, float *dep, float *col, float *opa,
                              float *rad, hipStream_t st) {
  int nx, nb;
  int64_t M;
  grid_dims(H, W, s, &nx, &M, &nb);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ingest_fill, dim3(nb), dim3(kNT), 0, st, depth, rgb, mask, H, W, s, nx, M,
                     fx, o_init, scratch + nb, n, pix, dep, col, opa, rad);
  return hipGetLastError();
}

}  // namespace vtgs
