// C ABI of the gfx950 view-tied splatting library (declared in vtgs.h):
// argument validation, plans (descriptor tables and workspace layout) and
// the launch sequences of render_fwd, render_bwd, track_step and map_step.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "vtgs.h"
#include "vtgs_internal.h"

using namespace vtgs;

namespace {

thread_local std::string g_err;

// Pinned host staging buffers for descriptor uploads, reused across plans
// (a request loop creates plans often; pinned allocation is slow).  A buffer
// returns to the pool only after the upload that read it has completed.
std::mutex g_pin_mu;
std::vector<std::pair<size_t, void *>> g_pin_free;  // (capacity, pointer)

void *pinned_take(size_t bytes, size_t *cap) {
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    for (size_t i = 0; i < g_pin_free.size(); i++)
      if (g_pin_free[i].first >= bytes) {
        void *p = g_pin_free[i].second;
        *cap = g_pin_free[i].first;
        g_pin_free.erase(g_pin_free.begin() + i);
        return p;
      }
  }
  size_t b = 4096;
  while (b < bytes) b <<= 1;
  void *p = nullptr;
  if (hipHostMalloc(&p, b) != hipSuccess) return nullptr;
  *cap = b;
  return p;
}

void pinned_give(void *p, size_t cap) {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  if (g_pin_free.size() < 64) {
    g_pin_free.push_back({cap, p});
    return;
  }
  (void)hipHostFree(p);
}

// The library's own scratch for vtgs_render_fwd_static: one copy per GPU
// (each device that loads the library holds it until the process ends).
// Host code never passes `g_scratch` itself to a kernel or a copy (in host
// code the name is a host-side stand-in, not a device address): it uses the
// address hipGetSymbolAddress gives for the current device.
static __device__ __align__(256) char g_scratch[VTGS_STATIC_SCRATCH_BYTES];

constexpr int kMaxStaticDevices = 64;
struct StaticSlot {
  char *ptr = nullptr;  // device address of g_scratch on this device
  uint64_t owner = 0;   // id of the plan whose descriptors it holds (0: none)
};
std::mutex g_static_mu;
StaticSlot g_static[kMaxStaticDevices];
std::atomic<uint64_t> g_plan_ids{0};

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIP_OK(expr)                                                               \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) return fail(VTGS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Region {
  int64_t off = 0, bytes = 0;
};

}  // namespace

struct vtgs_plan {
  uint64_t id = 0;  // unique per plan (owner tag of the static scratch)
  std::vector<DevKF> kfs;
  std::vector<DevView> views;
  std::vector<DevSeg> segs;
  std::vector<int32_t> kf_use_off;
  std::vector<DevKFUse> kf_use;
  vtgs_params prm{};
  int64_t cap = 0, P = 0;
  int32_t n_rec = 0, n_tiles = 0, loss_blocks = 0, ssim_gx = 0, ssim_gy = 0;
  int32_t max_learn_n = 0;
  bool any_learnable = false;
  bool any_geo = false;  // a learnable keyframe wants depth / pose gradients
  bool tile_order = false;  // composite the longest tile lists first
  // workspace layout
  Region r_hdr, r_desc, r_recA, r_recB, r_rect, r_rec_cnt, r_zbits, r_rec_off, r_scan, r_tcount, r_tcount_ns, r_tfill, r_woff,
      r_ranges, r_long, r_order, r_keys, r_keys_tmp, r_ids, r_slots, r_kpose, r_bits, r_tfinal, r_last,
      r_img, r_gimg, r_twist, r_loss, r_ssim_map, r_ssim_part;
  int64_t desc_kf = 0, desc_view = 0, desc_seg = 0, desc_use_off = 0, desc_use = 0, desc_bytes = 0;
  std::vector<char> desc_host;  // the descriptor tables as laid out in the workspace
  int64_t ws_bytes = 0;
  // binding
  char *ws = nullptr;
  Ws w{};
  void *pinned = nullptr;
  size_t pinned_cap = 0;
  hipEvent_t upload_done = nullptr;
  bool bound = false, fwd_done = false, slots_done = false;
  // stage timing (HIP events around every stage while enabled)
  bool timing = false;
  // captured tracking iterations (replayed by track_step), one per frame
  // length, loss array and configuration, least recently used dropped first
  struct TrackGraph {
    hipGraphExec_t exec = nullptr;
    int32_t iters = 0;
    float *loss = nullptr;
    vtgs_track_cfg cfg{};
    uint64_t used = 0;
  };
  std::vector<TrackGraph> graphs;
  uint64_t graph_clock = 0;
  // the captured mapping iteration (replayed by map_step) and what it was
  // captured with
  hipGraphExec_t map_graph = nullptr;
  vtgs_map_cfg map_cfg{};
  int32_t *map_step_ptr = nullptr;
  float *map_loss = nullptr;
  std::vector<hipEvent_t> ev_pool;
  struct EvUse { int stage; size_t start, stop; int launches; };
  std::vector<EvUse> ev_used;  // recorded stage intervals
  int timing_repeat = 1;       // launches per compositing stage while timing
};

namespace {

bool finite_pos(float x) { return std::isfinite(x) && x > 0.f; }

int validate_cam(const vtgs_camera &c, const char *what, int idx) {
  if (c.width <= 0 || c.height <= 0 || c.width > 65535 || c.height > 65535 || !finite_pos(c.fx) ||
      !finite_pos(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
    return fail(VTGS_E_ARG, std::string(what) + " " + std::to_string(idx) +
                                ": camera needs 0 < width, height <= 65535 and finite fx, fy > 0");
  return VTGS_OK;
}

// Floats per (record, tile) gradient slot: dL/dc (3), dL/do, dL/dr, and with
// geometry dL/dp (3).
int64_t slot_width(const vtgs_plan *p) { return p->any_geo ? 8 : 5; }
// Blocks of the per-Gaussian gather over the largest learnable keyframe.
int64_t gather_blocks(const vtgs_plan *p) { return (p->max_learn_n + 255) / 256; }

void layout(vtgs_plan *p) {
  int64_t off = 0;
  auto take = [&](Region &r, int64_t bytes) {
    r.off = off;
    r.bytes = bytes;
    off += align_up(std::max<int64_t>(bytes, 0));
  };
  const int64_t nk = (int64_t)p->kfs.size(), nv = (int64_t)p->views.size();
  const int64_t ns = (int64_t)p->segs.size(), nu = (int64_t)p->kf_use.size();
  take(p->r_hdr, 256);
  p->desc_kf = 0;
  p->desc_view = align_up(nk * (int64_t)sizeof(DevKF));
  p->desc_seg = p->desc_view + align_up(nv * (int64_t)sizeof(DevView));
  p->desc_use_off = p->desc_seg + align_up(ns * (int64_t)sizeof(DevSeg));
  p->desc_use = p->desc_use_off + align_up((nk + 1) * 4);
  p->desc_bytes = p->desc_use + align_up(nu * (int64_t)sizeof(DevKFUse));
  take(p->r_desc, p->desc_bytes);
  const int64_t nr = p->n_rec, nt = p->n_tiles, cap = p->cap, P = p->P;
  take(p->r_recA, nr * 48);
  take(p->r_recB, nr * 16);
  take(p->r_rect, nr * 8);
  take(p->r_rec_cnt, nr * 4);
  take(p->r_zbits, nr * 4);
  take(p->r_rec_off, (nr + 1) * 4);
  take(p->r_scan, (rec_scan_blocks(nr) + 1) * 4);
  take(p->r_tcount, nt * 4);
  take(p->r_tcount_ns, nt * 4);
  take(p->r_tfill, nt * 4);
  take(p->r_woff, (nr + 63) / 64 * 64 * 4);
  take(p->r_ranges, nt * 8);
  take(p->r_long, nt * 4);
  take(p->r_order, nt * 4);
  take(p->r_keys, cap * 8);
  take(p->r_keys_tmp, cap * 8);
  take(p->r_ids, cap * 4);
  take(p->r_slots, p->any_learnable ? cap * 4 * slot_width(p) : 0);
  take(p->r_kpose, p->any_geo ? nk * gather_blocks(p) * 32 : 0);
  // per 64-entry chunk of a tile list: each lane's bit mask of the entries
  // that reach its pixel(s), written by the forward, read by the backward
  take(p->r_bits, (cap / 64 + nt + 2) * (int64_t)lane_bits_per_chunk(p->prm.tile) * 8);
  take(p->r_tfinal, P * 4);
  take(p->r_last, P * 4);
  take(p->r_img, 5 * P * 4);
  take(p->r_gimg, 5 * P * 4);
  take(p->r_twist, nt * 32);
  take(p->r_loss, nv * (int64_t)p->loss_blocks * 16);
  take(p->r_ssim_map, 9 * P * 8);
  take(p->r_ssim_part, nv * 3 * (int64_t)p->ssim_gx * p->ssim_gy * 4);
  p->ws_bytes = off;
}

template <typename T>
T *at(char *base, const Region &r) {
  return reinterpret_cast<T *>(base + r.off);
}

void make_ws(vtgs_plan *p) {
  Ws &w = p->w;
  char *b = p->ws;
  w.flags = reinterpret_cast<uint32_t *>(b + p->r_hdr.off);
  w.n_pairs = reinterpret_cast<unsigned long long *>(b + p->r_hdr.off + 8);
  w.iter = reinterpret_cast<uint32_t *>(b + p->r_hdr.off + 16);
  w.n_long = reinterpret_cast<uint32_t *>(b + p->r_hdr.off + 24);
  w.long_next = reinterpret_cast<uint32_t *>(b + p->r_hdr.off + 28);
  w.long_tiles = at<uint32_t>(b, p->r_long);
  w.tile_order = p->tile_order ? at<uint32_t>(b, p->r_order) : nullptr;
  char *d = b + p->r_desc.off;
  w.kfs = reinterpret_cast<const DevKF *>(d + p->desc_kf);
  w.views = reinterpret_cast<const DevView *>(d + p->desc_view);
  w.segs = reinterpret_cast<DevSeg *>(d + p->desc_seg);
  w.kf_use_off = reinterpret_cast<const int32_t *>(d + p->desc_use_off);
  w.kf_use = reinterpret_cast<const DevKFUse *>(d + p->desc_use);
  w.n_kf = (int32_t)p->kfs.size();
  w.n_views = (int32_t)p->views.size();
  w.n_segs = (int32_t)p->segs.size();
  w.n_rec = p->n_rec;
  w.n_tiles = p->n_tiles;
  w.P = p->P;
  w.cap = p->cap;
  w.recA = at<float4>(b, p->r_recA);
  w.recB = at<float4>(b, p->r_recB);
  w.rect = at<uint2>(b, p->r_rect);
  w.rec_cnt = at<uint32_t>(b, p->r_rec_cnt);
  w.zbits = at<uint32_t>(b, p->r_zbits);
  w.rec_off = at<uint32_t>(b, p->r_rec_off);
  w.scan_part = at<uint32_t>(b, p->r_scan);
  w.tile_count = at<uint32_t>(b, p->r_tcount);
  w.tile_count_ns = at<uint32_t>(b, p->r_tcount_ns);
  w.tile_fill = at<uint32_t>(b, p->r_tfill);
  w.wave_off = at<uint32_t>(b, p->r_woff);
  w.ranges = at<uint2>(b, p->r_ranges);
  w.keys = at<unsigned long long>(b, p->r_keys);
  w.keys_tmp = at<unsigned long long>(b, p->r_keys_tmp);
  w.ids = at<uint32_t>(b, p->r_ids);
  w.slots = p->any_learnable ? at<float>(b, p->r_slots) : nullptr;
  w.kpose_part = p->any_geo ? at<float>(b, p->r_kpose) : nullptr;
  w.slot_w = (int32_t)slot_width(p);
  w.gblocks = (int32_t)gather_blocks(p);
  w.lane_bits = at<unsigned long long>(b, p->r_bits);
  w.t_final = at<float>(b, p->r_tfinal);
  w.last = at<uint32_t>(b, p->r_last);
  w.img = at<float>(b, p->r_img);
  w.gimg = at<float>(b, p->r_gimg);
  w.twist_part = at<float>(b, p->r_twist);
  w.loss_part = at<float>(b, p->r_loss);
  w.ssim_map = at<double>(b, p->r_ssim_map);
  w.ssim_part = at<float>(b, p->r_ssim_part);
  w.loss_blocks = p->loss_blocks;
  w.ssim_gx = p->ssim_gx;
  w.ssim_gy = p->ssim_gy;
  w.amin = p->prm.alpha_min;
  w.amax = p->prm.alpha_max;
  w.tmin = p->prm.t_min;
  w.qcut = p->prm.q_cut;
  w.znear = p->prm.z_near;
  w.lowpass = p->prm.lowpass;
  for (int c = 0; c < 3; c++) w.bg[c] = p->prm.bg[c];
  w.tile = p->prm.tile;
  w.batch = p->prm.batch;
}

// The descriptor tables in their workspace layout, kept on the host.
void desc_image(vtgs_plan *p) {
  p->desc_host.assign((size_t)std::max<int64_t>(p->desc_bytes, 256), 0);
  char *h = p->desc_host.data();
  if (!p->kfs.empty()) std::memcpy(h + p->desc_kf, p->kfs.data(), p->kfs.size() * sizeof(DevKF));
  std::memcpy(h + p->desc_view, p->views.data(), p->views.size() * sizeof(DevView));
  if (!p->segs.empty()) std::memcpy(h + p->desc_seg, p->segs.data(), p->segs.size() * sizeof(DevSeg));
  std::memcpy(h + p->desc_use_off, p->kf_use_off.data(), p->kf_use_off.size() * 4);
  if (!p->kf_use.empty()) std::memcpy(h + p->desc_use, p->kf_use.data(), p->kf_use.size() * sizeof(DevKFUse));
}

int check_bound(vtgs_plan *p) {
  if (!p) return fail(VTGS_E_ARG, "plan is NULL");
  if (!p->bound) return fail(VTGS_E_WORKSPACE, "plan has no bound workspace (vtgs_plan_bind)");
  return VTGS_OK;
}

// Optional roctx ranges (VTGS_ROCTX=1): one per entry point call and one per
// stage launch, named after them, so that a rocprofv3 --marker-trace puts
// the kernels of a trace under their entry point and stage.  The roctx
// library is opened at the first call only when asked for, so the library
// has no link-time dependency on it.
struct Roctx {
  int (*push)(const char *) = nullptr;
  int (*pop)() = nullptr;
};
const Roctx &roctx() {
  static const Roctx r = [] {
    Roctx x;
    const char *e = std::getenv("VTGS_ROCTX");
    if (!e || std::atoi(e) == 0) return x;
    void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
    if (!h) return x;
    x.push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
    x.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
    if (!x.push || !x.pop) x.push = nullptr, x.pop = nullptr;
    return x;
  }();
  return r;
}
struct RoctxRange {
  bool on;
  explicit RoctxRange(const char *name) : on(roctx().push != nullptr) {
    if (on) roctx().push(name);
  }
  ~RoctxRange() {
    if (on) roctx().pop();
  }
};

enum Stage {
  ST_PRE, ST_SCAN, ST_FILL, ST_SORT, ST_FWD, ST_LOSS, ST_RSCAN, ST_BWD, ST_REDUCE, ST_UPDATE, ST_N
};
static_assert(ST_N == VTGS_N_STAGES, "stage table");
const char *kStageNames[ST_N] = {"preprocess",   "scan_tiles",    "fill_keys", "sort_tiles",
                                 "composite_fwd", "loss",         "scan_records",
                                 "composite_bwd", "reduce",       "update"};

hipError_t event_at(vtgs_plan *p, size_t i, hipEvent_t *e) {
  while (p->ev_pool.size() <= i) {
    hipEvent_t ne;
    hipError_t r = hipEventCreate(&ne);
    if (r != hipSuccess) return r;
    p->ev_pool.push_back(ne);
  }
  *e = p->ev_pool[i];
  return hipSuccess;
}

// Launch `expr` as stage `stg`, bracketed by events when timing is on.  A
// compositing stage (idempotent: it overwrites what it writes) is launched
// `timing_repeat` times between its events, so that its per-launch time
// leaves out the events' own overhead.
#define STAGE(p, stg, st, expr)                                                  \
  do {                                                                           \
    size_t i0_ = 0;                                                              \
    int rep_ = 1;                                                                \
    if ((p)->timing) {                                                           \
      hipEvent_t ev_;                                                             \
      i0_ = (p)->ev_used.size() * 2;                                             \
      HIP_OK(event_at((p), i0_, &ev_));                                           \
      HIP_OK(hipEventRecord(ev_, (st)));                                          \
      if ((stg) == ST_FWD || (stg) == ST_BWD) rep_ = (p)->timing_repeat;         \
    }                                                                            \
    {                                                                            \
      RoctxRange rr_(kStageNames[(stg)]);                                        \
      for (int r_ = 0; r_ < rep_; r_++) HIP_OK(expr);                           \
    }                                                                            \
    if ((p)->timing) {                                                           \
      hipEvent_t ev_;                                                             \
      HIP_OK(event_at((p), i0_ + 1, &ev_));                                       \
      HIP_OK(hipEventRecord(ev_, (st)));                                          \
      (p)->ev_used.push_back({(stg), i0_, i0_ + 1, rep_});                       \
    }                                                                            \
  } while (0)

// The binning pipeline and the forward compositing into (rgb, depth, sil).
int run_forward(vtgs_plan *p, float *rgb, float *depth, float *sil, hipStream_t st) {
  const Ws &w = p->w;
  STAGE(p, ST_PRE, st, launch_preprocess(w, st));  // (+ relative poses)
  STAGE(p, ST_SCAN, st, launch_scan_tiles(w, st));
  STAGE(p, ST_FILL, st, launch_fill_keys(w, st));
  STAGE(p, ST_SORT, st, launch_sort_tiles(w, st));
  STAGE(p, ST_FWD, st, launch_composite_fwd(w, rgb, depth, sil, st));
  p->fwd_done = true;
  return VTGS_OK;
}

// One tracking iteration of every view: forward into the internal images,
// Eq. 1 loss and gradients, backward to the twist, Adam step + retraction.
int track_iteration(vtgs_plan *p, const vtgs_track_cfg &cfg, float *loss, hipStream_t st) {
  const Ws &w = p->w;
  const int64_t P = p->P;
  if (int rc = run_forward(p, w.img, w.img + 3 * P, w.img + 4 * P, st)) return rc;
  (void)P;
  // Eq. 1 and its upstream gradient are evaluated by the backward per pixel
  STAGE(p, ST_BWD, st, launch_composite_bwd(w, nullptr, nullptr, nullptr, 1, st, &cfg));
  STAGE(p, ST_UPDATE, st, launch_track_update(w, cfg, loss, st));
  return VTGS_OK;
}

// Point the plan at workspace `ws`: upload the descriptor tables from the
// host copy `h` (pinned, or the plan's own), clear the header and the tile
// counters, and drop graphs captured against the previous binding.
int bind_to(vtgs_plan *p, char *ws, const char *h, hipStream_t st) {
  if (!p->upload_done) HIP_OK(hipEventCreateWithFlags(&p->upload_done, hipEventDisableTiming));
  p->ws = ws;
  make_ws(p);
  for (auto &g : p->graphs) (void)hipGraphExecDestroy(g.exec);
  p->graphs.clear();
  if (p->map_graph) (void)hipGraphExecDestroy(p->map_graph);
  p->map_graph = nullptr;
  HIP_OK(hipMemcpyAsync(p->ws + p->r_desc.off, h, p->desc_bytes, hipMemcpyHostToDevice, st));
  HIP_OK(hipEventRecord(p->upload_done, st));
  HIP_OK(launch_fill_u32((uint32_t *)(p->ws + p->r_hdr.off), 0u, 64, st));
  HIP_OK(launch_fill_u32(p->w.tile_count, 0u, p->n_tiles, st));
  HIP_OK(launch_fill_u32(p->w.tile_fill, 0u, p->n_tiles, st));
  HIP_OK(launch_fill_u32(p->w.tile_count_ns, 0u, p->n_tiles, st));
  p->bound = true;
  p->fwd_done = false;
  p->slots_done = false;
  return VTGS_OK;
}

// One mapping iteration of every view: forward into the internal images,
// Eq. 2 and its upstream gradients, backward to the learnable keyframes,
// Adam steps.
int map_iteration(vtgs_plan *p, const vtgs_map_cfg &cfg, int32_t *step, float *loss,
                  hipStream_t st) {
  const Ws &w = p->w;
  const int64_t P = p->P;
  if (int rc = run_forward(p, w.img, w.img + 3 * P, w.img + 4 * P, st)) return rc;
  STAGE(p, ST_LOSS, st, launch_map_loss(w, cfg, st));
  if (p->any_learnable) {
    STAGE(p, ST_RSCAN, st, launch_scan_records(w, st));
    STAGE(p, ST_BWD, st, launch_composite_bwd(w, w.gimg, w.gimg + 3 * P, nullptr,
                                               p->any_geo ? 6 : 2, st));
    p->slots_done = true;
  }
  STAGE(p, ST_UPDATE, st,
        launch_map_update(w, cfg, step, loss, p->any_learnable ? p->max_learn_n : 0, st));
  return VTGS_OK;
}

}  // namespace

extern "C" {

int32_t vtgs_abi_version(void) { return VTGS_ABI_VERSION; }

const char *vtgs_last_error(void) { return g_err.c_str(); }

void vtgs_default_params(vtgs_params *out) {
  if (!out) return;
  out->alpha_min = 1.0f / 255.0f;
  out->alpha_max = 0.99f;
  out->t_min = 1e-4f;
  out->q_cut = 11.0826f;
  out->z_near = 0.01f;
  out->lowpass = 0.3f;
  out->bg[0] = out->bg[1] = out->bg[2] = 0.f;
  out->tile = 16;
  out->batch = 256;
}

int64_t vtgs_ingest_scratch_bytes(int32_t H, int32_t W, int32_t stride) {
  if (H <= 0 || W <= 0 || stride <= 0) return 0;
  return 4 * ingest_scratch_words(H, W, stride);
}

int vtgs_ingest_count(const float *depth_img, const uint8_t *mask, int32_t H, int32_t W,
                      int32_t stride, void *scratch, int64_t scratch_bytes, int32_t *count,
                      void *stream) {
  try {
    if (!depth_img || !scratch || !count) return fail(VTGS_E_ARG, "ingest_count: NULL pointer");
    if (H <= 0 || W <= 0 || stride <= 0 || (int64_t)H * W > (1ll << 31) - 1)
      return fail(VTGS_E_ARG, "ingest_count: need H, W, stride > 0 and H*W < 2^31");
    if (scratch_bytes < vtgs_ingest_scratch_bytes(H, W, stride))
      return fail(VTGS_E_WORKSPACE, "ingest_count: scratch too small");
    HIP_OK(launch_ingest_count(depth_img, mask, H, W, stride, (uint32_t *)scratch, count,
                               (hipStream_t)stream));
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "ingest_count: unexpected exception");
  }
}

int vtgs_ingest_fill(const float *depth_img, const float *rgb_img, const uint8_t *mask,
                     int32_t H, int32_t W, int32_t stride, float fx, float o_init,
                     const void *scratch, int64_t scratch_bytes, int32_t n, uint32_t *pix,
                     float *depth, float *color, float *opacity, float *radius, void *stream) {
  RoctxRange rr_("vtgs_ingest_fill");
  try {
    if (!depth_img || !scratch) return fail(VTGS_E_ARG, "ingest_fill: NULL pointer");
    if (n > 0 && (!pix || !depth || !opacity || !radius || (rgb_img && !color)))
      return fail(VTGS_E_ARG, "ingest_fill: NULL output pointer");
    if (H <= 0 || W <= 0 || stride <= 0 || n < 0 || (int64_t)H * W > (1ll << 31) - 1)
      return fail(VTGS_E_ARG, "ingest_fill: need H, W, stride > 0, n >= 0");
    if (!finite_pos(fx)) return fail(VTGS_E_ARG, "ingest_fill: fx must be finite and > 0");
    if (scratch_bytes < vtgs_ingest_scratch_bytes(H, W, stride))
      return fail(VTGS_E_WORKSPACE, "ingest_fill: scratch too small");
    HIP_OK(launch_ingest_fill(depth_img, rgb_img, mask, H, W, stride, fx, o_init,
                              (const uint32_t *)scratch, n, pix, depth, color, opacity, radius,
                              (hipStream_t)stream));
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "ingest_fill: unexpected exception");
  }
}

int vtgs_plan_create(const vtgs_keyframe *kfs, int32_t n_kf, const vtgs_view *views,
                     int32_t n_views, const vtgs_params *prm, int64_t pair_capacity,
                     vtgs_plan **out) {
  try {
    if (!out) return fail(VTGS_E_ARG, "plan_create: out is NULL");
    *out = nullptr;
    if (n_kf < 0 || n_views < 1 || (n_kf > 0 && !kfs) || !views)
      return fail(VTGS_E_ARG, "plan_create: need n_kf >= 0, n_views >= 1 and their arrays");
    vtgs_params P;
    if (prm) P = *prm; else vtgs_default_params(&P);
    if (P.tile != 8 && P.tile != 16 && P.tile != 32)
      return fail(VTGS_E_ARG, "plan_create: tile must be 8, 16 or 32");
    if (P.batch != 128 && P.batch != 256 && P.batch != 512)
      return fail(VTGS_E_ARG, "plan_create: batch must be 128, 256 or 512");
    if (!(P.alpha_min >= 0.f && P.alpha_max >= P.alpha_min && P.alpha_max < 1.f && P.t_min >= 0.f &&
          P.t_min < 1.f && P.q_cut > 0.f && std::isfinite(P.q_cut) && P.lowpass >= 0.f &&
          std::isfinite(P.lowpass) && std::isfinite(P.z_near)))
      return fail(VTGS_E_ARG, "plan_create: need 0 <= alpha_min <= alpha_max < 1, 0 <= t_min < 1, "
                              "finite q_cut > 0, lowpass >= 0, finite z_near");
    auto *p = new vtgs_plan();
    p->prm = P;
    int64_t n_rec = 0, n_tiles = 0, Ptot = 0;
    int32_t loss_blocks = 0, maxw = 0, maxh = 0;
    for (int k = 0; k < n_kf; k++) {
      const vtgs_keyframe &K = kfs[k];
      if (K.n < 0) { delete p; return fail(VTGS_E_ARG, "plan_create: keyframe " + std::to_string(k) + " has n < 0"); }
      if (int rc = validate_cam(K.cam, "keyframe", k)) { delete p; return rc; }
      if (K.n > 0 && (!K.pix || !K.depth || !K.color || !K.opacity || !K.radius || !K.pose)) {
        delete p;
        return fail(VTGS_E_ARG, "plan_create: keyframe " + std::to_string(k) + " has a NULL array");
      }
      if (K.n > 0 && !K.pose) { delete p; return fail(VTGS_E_ARG, "plan_create: keyframe pose NULL"); }
      DevKF d{};
      d.pix = K.pix; d.depth = K.depth; d.color = K.color; d.opacity = K.opacity;
      d.radius = K.radius; d.pose = K.pose;
      d.fx = K.cam.fx; d.fy = K.cam.fy; d.cx = K.cam.cx; d.cy = K.cam.cy;
      d.width = K.cam.width; d.height = K.cam.height; d.n = K.n; d.learnable = K.learnable ? 1 : 0;
      d.g_color = K.g_color; d.g_opacity = K.g_opacity; d.g_radius = K.g_radius; d.adam = K.adam;
      if (d.learnable) {
        d.g_depth = K.g_depth; d.g_pose = K.g_pose;
        d.depth_adam = K.depth_adam; d.pose_adam = K.pose_adam;
        d.geo = (K.g_depth || K.g_pose || K.depth_adam || K.pose_adam) ? 1 : 0;
      }
      p->kfs.push_back(d);
      if (d.learnable && d.n > 0) {
        p->any_learnable = true;
        p->max_learn_n = std::max(p->max_learn_n, d.n);
        if (d.geo) p->any_geo = true;
      }
    }
    for (int v = 0; v < n_views; v++) {
      const vtgs_view &V = views[v];
      if (int rc = validate_cam(V.cam, "view", v)) { delete p; return rc; }
      if (!V.pose) { delete p; return fail(VTGS_E_ARG, "plan_create: view " + std::to_string(v) + " pose is NULL"); }
      if (V.kf_first < 0 || V.kf_count < 0 || (int64_t)V.kf_first + V.kf_count > n_kf) {
        delete p;
        return fail(VTGS_E_ARG, "plan_create: view " + std::to_string(v) + " keyframe slice out of range");
      }
      DevView d{};
      d.fx = V.cam.fx; d.fy = V.cam.fy; d.cx = V.cam.cx; d.cy = V.cam.cy;
      d.width = V.cam.width; d.height = V.cam.height;
      d.tiles_x = (V.cam.width + P.tile - 1) / P.tile;
      d.tiles_y = (V.cam.height + P.tile - 1) / P.tile;
      d.pose = V.pose; d.kf_first = V.kf_first; d.kf_count = V.kf_count;
      d.rec_base = (int32_t)n_rec;
      d.tile_base = (int32_t)n_tiles;
      d.n_tiles = d.tiles_x * d.tiles_y;
      d.pix_off = Ptot;
      d.obs_rgb = V.obs_rgb; d.obs_depth = V.obs_depth; d.vis = V.vis; d.pose_adam = V.pose_adam;
      d.seg_first = (int32_t)p->segs.size();
      d.seg_count = V.kf_count;
      int64_t local = 0;
      for (int s = 0; s < V.kf_count; s++) {
        const int k = V.kf_first + s;
        DevSeg sg{};
        sg.view = v; sg.kf = k; sg.rec_start = (int32_t)(n_rec + local); sg.n = kfs[k].n;
        p->segs.push_back(sg);
        local += kfs[k].n;
      }
      d.n_rec = (int32_t)local;
      n_rec += local;
      n_tiles += d.n_tiles;
      const int64_t Pv = (int64_t)V.cam.width * V.cam.height;
      Ptot += Pv;
      loss_blocks = std::max<int32_t>(loss_blocks, (int32_t)((Pv + 255) / 256));
      maxw = std::max(maxw, V.cam.width);
      maxh = std::max(maxh, V.cam.height);
      if (n_rec > (1ll << 31) - 1 || n_tiles > (1ll << 31) - 1 || Ptot > (1ll << 31) - 1) {
        delete p;
        return fail(VTGS_E_ARG, "plan_create: more than 2^31 records, tiles or pixels");
      }
      p->views.push_back(d);
    }
    // per keyframe, the (view, record start) pairs that render it
    p->kf_use_off.assign(n_kf + 1, 0);
    for (const DevSeg &s : p->segs) p->kf_use_off[s.kf + 1]++;
    for (int k = 0; k < n_kf; k++) p->kf_use_off[k + 1] += p->kf_use_off[k];
    p->kf_use.resize(p->segs.size());
    {
      std::vector<int32_t> fill(p->kf_use_off.begin(), p->kf_use_off.end() - 1);
      for (size_t i = 0; i < p->segs.size(); i++) {
        const DevSeg &s = p->segs[i];
        p->kf_use[fill[s.kf]++] = DevKFUse{s.rec_start, s.view, (int32_t)i};
      }
    }
    p->n_rec = (int32_t)n_rec;
    p->n_tiles = (int32_t)n_tiles;
    p->P = Ptot;
    // longest tile lists first where views of different sizes and list
    // lengths share a grid (a multi-view plan); VTGS_TILE_ORDER=0 / 1 forces it
    {
      const char *e = std::getenv("VTGS_TILE_ORDER");
      p->tile_order = e ? std::atoi(e) != 0 : n_views > 1;
    }
    p->loss_blocks = std::max(loss_blocks, 1);
    p->ssim_gx = (maxw + 15) / 16;
    p->ssim_gy = (maxh + 15) / 16;
    // default room: a Gaussian of extent R ~ 4-5 px covers about (1 + 10/B)^2
    // tiles of side B; keep 50% headroom
    // the compositing kernels index tile lists with 32-bit signed positions
    constexpr int64_t kMaxCap = (1ll << 31) - 1;
    if (pair_capacity > kMaxCap) {
      delete p;
      return fail(VTGS_E_ARG, "plan_create: pair_capacity above 2^31 - 1");
    }
    const double per = 1.5 * (1.0 + 10.0 / P.tile) * (1.0 + 10.0 / P.tile);
    const double want = pair_capacity > 0 ? (double)pair_capacity : std::ceil(per * (double)n_rec) + 65536.0;
    const int64_t cap = std::max<int64_t>(1, (int64_t)std::min(want, (double)kMaxCap));
    p->cap = cap;
    layout(p);
    desc_image(p);
    p->id = ++g_plan_ids;
    *out = p;
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "plan_create: unexpected exception (out of host memory?)");
  }
}

void vtgs_plan_destroy(vtgs_plan *p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    for (StaticSlot &s : g_static)
      if (s.owner == p->id) s.owner = 0;
  }
  if (p->upload_done) {
    (void)hipEventSynchronize(p->upload_done);
    (void)hipEventDestroy(p->upload_done);
  }
  if (p->pinned) pinned_give(p->pinned, p->pinned_cap);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  for (auto &g : p->graphs) (void)hipGraphExecDestroy(g.exec);
  if (p->map_graph) (void)hipGraphExecDestroy(p->map_graph);
  delete p;
}

int vtgs_uncovered_mask(const float *sil, const float *depth_img, int64_t n, float thr,
                        uint8_t *mask, void *stream) {
  RoctxRange rr_("vtgs_uncovered_mask");
  try {
    if (n < 0 || (n > 0 && (!sil || !depth_img || !mask)))
      return fail(VTGS_E_ARG, "uncovered_mask: need n >= 0 and non-NULL arrays");
    if (!std::isfinite(thr)) return fail(VTGS_E_ARG, "uncovered_mask: thr must be finite");
    HIP_OK(launch_uncovered(sil, depth_img, n, thr, mask, (hipStream_t)stream));
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "uncovered_mask: unexpected exception");
  }
}

int64_t vtgs_plan_workspace_bytes(const vtgs_plan *p) { return p ? p->ws_bytes : -1; }
int64_t vtgs_plan_pixels(const vtgs_plan *p) { return p ? p->P : -1; }
int64_t vtgs_plan_records(const vtgs_plan *p) { return p ? p->n_rec : -1; }
int64_t vtgs_plan_tiles(const vtgs_plan *p) { return p ? p->n_tiles : -1; }
int64_t vtgs_plan_pair_capacity(const vtgs_plan *p) { return p ? p->cap : -1; }
int64_t vtgs_plan_view_offset(const vtgs_plan *p, int32_t v) {
  if (!p || v < 0 || v >= (int32_t)p->views.size()) return -1;
  return p->views[v].pix_off;
}

int vtgs_plan_bind(vtgs_plan *p, void *ws, int64_t ws_bytes, void *stream) {
  try {
    if (!p) return fail(VTGS_E_ARG, "plan_bind: plan is NULL");
    if (!ws) return fail(VTGS_E_WORKSPACE, "plan_bind: workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
      return fail(VTGS_E_WORKSPACE, "plan_bind: workspace must be 256-byte aligned");
    if (ws_bytes < p->ws_bytes)
      return fail(VTGS_E_WORKSPACE, "plan_bind: workspace has " + std::to_string(ws_bytes) +
                                        " bytes, needs " + std::to_string(p->ws_bytes));
    hipStream_t st = (hipStream_t)stream;
    if (p->upload_done) HIP_OK(hipEventSynchronize(p->upload_done));
    if (!p->pinned) {
      p->pinned = pinned_take((size_t)std::max<int64_t>(p->desc_bytes, 256), &p->pinned_cap);
      if (!p->pinned) return fail(VTGS_E_HIP, "plan_bind: pinned host allocation failed");
    }
    char *h = (char *)p->pinned;
    std::memcpy(h, p->desc_host.data(), p->desc_bytes);
    return bind_to(p, (char *)ws, h, st);
  } catch (...) {
    return fail(VTGS_E_HIP, "plan_bind: unexpected exception");
  }
}

int vtgs_plan_status(vtgs_plan *p, int64_t *pairs_needed, int32_t clear, void *stream) {
  if (int rc = check_bound(p)) return rc;
  hipStream_t st = (hipStream_t)stream;
  HIP_OK(hipStreamSynchronize(st));
  uint32_t flags = 0;
  unsigned long long np = 0;
  HIP_OK(hipMemcpy(&flags, p->w.flags, 4, hipMemcpyDeviceToHost));
  HIP_OK(hipMemcpy(&np, p->w.n_pairs, 8, hipMemcpyDeviceToHost));
  if (pairs_needed) *pairs_needed = (int64_t)np;
  if (clear && flags) {
    HIP_OK(launch_fill_u32(p->w.flags, 0u, 1, st));
    HIP_OK(hipStreamSynchronize(st));
  }
  if (flags & kFlagCapacity)
    return fail(VTGS_E_CAPACITY, "pair capacity " + std::to_string(p->cap) + " exceeded: " +
                                     std::to_string(np) + " (Gaussian, tile) pairs needed");
  if (flags & kFlagNonfinite) return fail(VTGS_E_NONFINITE, "a loss was not finite");
  return VTGS_OK;
}

int vtgs_render_fwd(vtgs_plan *p, float *rgb, float *depth, float *sil, void *stream) {
  RoctxRange rr_("vtgs_render_fwd");
  try {
    if (int rc = check_bound(p)) return rc;
    return run_forward(p, rgb, depth, sil, (hipStream_t)stream);
  } catch (...) {
    return fail(VTGS_E_HIP, "render_fwd: unexpected exception");
  }
}

int vtgs_render_fwd_static(vtgs_plan *p, float *rgb, float *depth, float *sil, void *stream) {
  RoctxRange rr_("vtgs_render_fwd_static");
  try {
    if (!p) return fail(VTGS_E_ARG, "render_fwd_static: plan is NULL");
    if (p->ws_bytes > (int64_t)VTGS_STATIC_SCRATCH_BYTES)
      return fail(VTGS_E_WORKSPACE, "render_fwd_static: the plan needs " +
                                        std::to_string(p->ws_bytes) + " bytes, the static scratch holds " +
                                        std::to_string((int64_t)VTGS_STATIC_SCRATCH_BYTES));
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxStaticDevices)
      return fail(VTGS_E_ARG, "render_fwd_static: device index beyond " + std::to_string(kMaxStaticDevices));
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_static_mu);
    StaticSlot &slot = g_static[dev];
    if (!slot.ptr) {
      // this device's copy of the array, with the device current
      void *ptr = nullptr;
      HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_scratch)));
      if (!ptr || reinterpret_cast<uintptr_t>(ptr) % kAlign)
        return fail(VTGS_E_HIP, "render_fwd_static: static scratch address unusable");
      slot.ptr = (char *)ptr;
    }
    if (slot.owner != p->id || p->ws != slot.ptr) {
      slot.owner = 0;
      if (int rc = bind_to(p, slot.ptr, p->desc_host.data(), st)) return rc;
      slot.owner = p->id;
    }
    return run_forward(p, rgb, depth, sil, st);
  } catch (...) {
    return fail(VTGS_E_HIP, "render_fwd_static: unexpected exception");
  }
}

int vtgs_render_bwd(vtgs_plan *p, const float *g_rgb, const float *g_depth, const float *g_sil,
                    float *g_twist, void *stream) {
  RoctxRange rr_("vtgs_render_bwd");
  try {
    if (int rc = check_bound(p)) return rc;
    if (!p->fwd_done) return fail(VTGS_E_ARG, "render_bwd: no render_fwd on this plan yet");
    hipStream_t st = (hipStream_t)stream;
    bool want_kf = false;
    for (const DevKF &k : p->kfs)
      if (k.learnable && k.n > 0 && (k.g_color || k.g_opacity || k.g_radius)) want_kf = true;
    bool want_geo = false;
    for (const DevKF &k : p->kfs)
      if (k.learnable && k.n > 0 && (k.g_depth || k.g_pose)) want_geo = true;
    const int mode = (g_twist ? 1 : 0) | (want_kf || want_geo ? 2 : 0) | (p->any_geo && (want_kf || want_geo) ? 4 : 0);
    if (mode == 0) return VTGS_OK;
    const Ws &w = p->w;
    if (mode & 2) STAGE(p, ST_RSCAN, st, launch_scan_records(w, st));
    STAGE(p, ST_BWD, st, launch_composite_bwd(w, g_rgb, g_depth, g_sil, mode, st));
    if (mode & 2) p->slots_done = true;
    if (mode & 2) STAGE(p, ST_REDUCE, st, launch_gather(w, p->max_learn_n, st));
    if (mode & 1) STAGE(p, ST_REDUCE, st, launch_twist_reduce(w, g_twist, st));
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "render_bwd: unexpected exception");
  }
}

int vtgs_track_step(vtgs_plan *p, const vtgs_track_cfg *cfg, int32_t iters, float *loss,
                    void *stream) {
  RoctxRange rr_("vtgs_track_step");
  try {
    if (int rc = check_bound(p)) return rc;
    if (!cfg) return fail(VTGS_E_ARG, "track_step: cfg is NULL");
    if (iters < 0) return fail(VTGS_E_ARG, "track_step: iters < 0");
    for (size_t v = 0; v < p->views.size(); v++) {
      const DevView &d = p->views[v];
      if (!d.obs_rgb || !d.obs_depth || !d.pose_adam)
        return fail(VTGS_E_ARG, "track_step: view " + std::to_string(v) +
                                    " needs obs_rgb, obs_depth and pose_adam");
    }
    hipStream_t st = (hipStream_t)stream;
    HIP_OK(launch_fill_u32(p->w.iter, 0xFFFFFFFFu, 1, st));
    if (iters == 0) return VTGS_OK;
    // Replay a captured graph of `g` iterations when the stream can be
    // captured (not the legacy default stream) and stage timing is off.
    const bool graphs = st != nullptr && !p->timing && iters >= 2 && !std::getenv("VTGS_NO_GRAPH");
    if (!graphs) {
      for (int it = 0; it < iters; it++)
        if (int rc = track_iteration(p, *cfg, loss, st)) return rc;
      return VTGS_OK;
    }
    const int32_t g = iters <= 64 ? iters : 1;
    vtgs_plan::TrackGraph *tg = nullptr;
    for (auto &e : p->graphs)
      if (e.iters == g && e.loss == loss && std::memcmp(&e.cfg, cfg, sizeof(vtgs_track_cfg)) == 0)
        tg = &e;
    if (!tg) {
      constexpr size_t kMaxGraphs = 4;
      if (p->graphs.size() >= kMaxGraphs) {
        size_t old = 0;
        for (size_t i = 1; i < p->graphs.size(); i++)
          if (p->graphs[i].used < p->graphs[old].used) old = i;
        HIP_OK(hipGraphExecDestroy(p->graphs[old].exec));
        p->graphs.erase(p->graphs.begin() + (std::ptrdiff_t)old);
      }
      HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      int rc = VTGS_OK;
      for (int it = 0; it < g && rc == VTGS_OK; it++) rc = track_iteration(p, *cfg, loss, st);
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &graph);
      if (rc != VTGS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ec != hipSuccess) return fail(VTGS_E_HIP, std::string("stream capture: ") + hipGetErrorString(ec));
      vtgs_plan::TrackGraph e;
      const hipError_t ei = hipGraphInstantiate(&e.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return fail(VTGS_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
      e.iters = g;
      e.loss = loss;
      e.cfg = *cfg;
      p->graphs.push_back(e);
      tg = &p->graphs.back();
    }
    tg->used = ++p->graph_clock;
    for (int done = 0; done + g <= iters; done += g) HIP_OK(hipGraphLaunch(tg->exec, st));
    for (int it = (iters / g) * g; it < iters; it++)
      if (int rc = track_iteration(p, *cfg, loss, st)) return rc;
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "track_step: unexpected exception");
  }
}

int vtgs_map_step(vtgs_plan *p, const vtgs_map_cfg *cfg, int32_t *step, float *loss,
                  void *stream) {
  RoctxRange rr_("vtgs_map_step");
  try {
    if (int rc = check_bound(p)) return rc;
    if (!cfg || !step) return fail(VTGS_E_ARG, "map_step: cfg and step are required");
    for (size_t v = 0; v < p->views.size(); v++) {
      const DevView &d = p->views[v];
      if (!d.obs_rgb || !d.obs_depth)
        return fail(VTGS_E_ARG, "map_step: view " + std::to_string(v) + " needs obs_rgb and obs_depth");
    }
    for (size_t k = 0; k < p->kfs.size(); k++)
      if (p->kfs[k].learnable && p->kfs[k].n > 0 && !p->kfs[k].adam)
        return fail(VTGS_E_ARG, "map_step: learnable keyframe " + std::to_string(k) + " has no adam state");
    hipStream_t st = (hipStream_t)stream;
    // Replay the captured iteration when the stream can be captured (not
    // the legacy default stream), stage timing is off and it was captured
    // with the same configuration, step counter and loss array (the step
    // counter lives on the device, so nothing the host writes changes
    // between replays).
    const bool graphs = st != nullptr && !p->timing && !std::getenv("VTGS_NO_GRAPH");
    if (!graphs) return map_iteration(p, *cfg, step, loss, st);
    if (p->map_graph && (p->map_step_ptr != step || p->map_loss != loss ||
                         std::memcmp(&p->map_cfg, cfg, sizeof(vtgs_map_cfg)) != 0)) {
      HIP_OK(hipGraphExecDestroy(p->map_graph));
      p->map_graph = nullptr;
    }
    if (!p->map_graph) {
      HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      const int rc = map_iteration(p, *cfg, step, loss, st);
      hipGraph_t graph = nullptr;
      const hipError_t ec = hipStreamEndCapture(st, &graph);
      if (rc != VTGS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ec != hipSuccess) return fail(VTGS_E_HIP, std::string("stream capture: ") + hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&p->map_graph, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        p->map_graph = nullptr;
        return fail(VTGS_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
      }
      p->map_cfg = *cfg;
      p->map_step_ptr = step;
      p->map_loss = loss;
    }
    HIP_OK(hipGraphLaunch(p->map_graph, st));
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "map_step: unexpected exception");
  }
}

int vtgs_visibility(const float *src_depth, const vtgs_camera *src_cam, const float *src_pose,
                    const vtgs_frame_ref *targets, int32_t n_targets, float rel_tol, float z_near,
                    uint8_t *mask, int32_t *counts, void *stream) {
  RoctxRange rr_("vtgs_visibility");
  try {
    if (!src_depth || !src_cam || !src_pose || !targets || n_targets < 1)
      return fail(VTGS_E_ARG, "visibility: need the source arrays and n_targets >= 1 targets");
    if (int rc = validate_cam(*src_cam, "visibility source", 0)) return rc;
    if (!(rel_tol >= 0.f) || !std::isfinite(rel_tol) || !std::isfinite(z_near))
      return fail(VTGS_E_ARG, "visibility: need a finite rel_tol >= 0 and a finite z_near");
    for (int t = 0; t < n_targets; t++) {
      if (!targets[t].depth || !targets[t].pose)
        return fail(VTGS_E_ARG, "visibility: target " + std::to_string(t) + " has a NULL array");
      if (int rc = validate_cam(targets[t].cam, "visibility target", t)) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    if (counts) HIP_OK(launch_fill_u32(reinterpret_cast<uint32_t *>(counts), 0u, n_targets, st));
    const VisCam sc{src_cam->fx, src_cam->fy, src_cam->cx, src_cam->cy, src_cam->width,
                    src_cam->height};
    for (int t0 = 0; t0 < n_targets; t0 += kVisMaxTargets) {
      VisTargets tg{};
      tg.n = std::min(kVisMaxTargets, n_targets - t0);
      for (int j = 0; j < tg.n; j++) {
        const vtgs_frame_ref &F = targets[t0 + j];
        tg.depth[j] = F.depth;
        tg.pose[j] = F.pose;
        tg.fx[j] = F.cam.fx; tg.fy[j] = F.cam.fy; tg.cx[j] = F.cam.cx; tg.cy[j] = F.cam.cy;
        tg.width[j] = F.cam.width; tg.height[j] = F.cam.height;
      }
      HIP_OK(launch_visibility(src_depth, sc, src_pose, tg, rel_tol, z_near, mask,
                               counts ? counts + t0 : nullptr, t0 == 0 ? 1 : 0, st));
    }
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "visibility: unexpected exception");
  }
}

const char *vtgs_stage_name(int32_t stage) {
  return (stage >= 0 && stage < ST_N) ? kStageNames[stage] : "";
}

int vtgs_plan_timing(vtgs_plan *p, int32_t enable, double *ms, int64_t *count) {
  try {
    if (!p) return fail(VTGS_E_ARG, "plan_timing: plan is NULL");
    if (enable) {
      p->timing = true;
      p->timing_repeat = enable > 1 ? std::min(enable, 64) : 1;
      p->ev_used.clear();
      return VTGS_OK;
    }
    p->timing = false;
    double acc[ST_N] = {0};
    int64_t cnt[ST_N] = {0};
    for (auto &u : p->ev_used) {
      HIP_OK(hipEventSynchronize(p->ev_pool[u.stop]));
      float t = 0.f;
      HIP_OK(hipEventElapsedTime(&t, p->ev_pool[u.start], p->ev_pool[u.stop]));
      acc[u.stage] += t;
      cnt[u.stage] += u.launches;
    }
    p->ev_used.clear();
    for (int i = 0; i < ST_N; i++) {
      if (ms) ms[i] = acc[i];
      if (count) count[i] = cnt[i];
    }
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "plan_timing: unexpected exception");
  }
}

int vtgs_debug_state(vtgs_plan *p, float *records, int32_t *rect, uint32_t *ranges, uint32_t *ids,
                     int64_t *n_pairs, void *stream) {
  try {
    if (int rc = check_bound(p)) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (records || rect) HIP_OK(launch_debug_copy(p->w, records, rect, st));
    if (ranges) HIP_OK(hipMemcpyAsync(ranges, p->w.ranges, (size_t)p->n_tiles * 8, hipMemcpyDeviceToDevice, st));
    if (ids) HIP_OK(hipMemcpyAsync(ids, p->w.ids, (size_t)p->cap * 4, hipMemcpyDeviceToDevice, st));
    if (n_pairs) HIP_OK(hipMemcpyAsync(n_pairs, p->w.n_pairs, 8, hipMemcpyDeviceToDevice, st));
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "debug_state: unexpected exception");
  }
}

int vtgs_debug_images(vtgs_plan *p, float *img, float *gimg, void *stream) {
  try {
    if (int rc = check_bound(p)) return rc;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = (size_t)p->P * 5 * sizeof(float);
    if (img) HIP_OK(hipMemcpyAsync(img, p->w.img, bytes, hipMemcpyDeviceToDevice, st));
    if (gimg) {
      // the silhouette plane map_step never forms is reported as zeros
      HIP_OK(hipMemcpyAsync(gimg, p->w.gimg, bytes * 4 / 5, hipMemcpyDeviceToDevice, st));
      HIP_OK(launch_fill_f32(gimg + 4 * p->P, 0.f, p->P, st));
    }
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "debug_images: unexpected exception");
  }
}

int vtgs_debug_gather(vtgs_plan *p, void *stream) {
  try {
    if (int rc = check_bound(p)) return rc;
    if (!p->any_learnable) return fail(VTGS_E_ARG, "debug_gather: no learnable keyframe");
    if (!p->slots_done)
      return fail(VTGS_E_ARG, "debug_gather: no backward to colour/opacity/radius on this plan yet");
    HIP_OK(launch_gather(p->w, p->max_learn_n, (hipStream_t)stream));
    return VTGS_OK;
  } catch (...) {
    return fail(VTGS_E_HIP, "debug_gather: unexpected exception");
  }
}

}  // extern "C"
