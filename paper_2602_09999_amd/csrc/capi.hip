// C ABI entry points (include/fastergs.h): argument validation, workspace
// layout and the launch sequence of one forward / backward rasterization.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "fgs_internal.h"

using namespace fgs;

namespace {
thread_local std::string g_last_error;
}  // namespace

fgs_status fgs::fail(fgs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

namespace {

fgs_status hip_fail(hipError_t e, const char* where) {
  return fail(FGS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

#define FGS_HIP(expr, where)                     \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

// One-shot timing hook (fgs_time_next_launch): when armed for `name`, events
// are recorded on the launch stream around the next run of that step.
struct TimerHook {
  std::string name;
  hipEvent_t start = nullptr, stop = nullptr;
  bool armed = false;
};
thread_local TimerHook g_timer;

struct TimedStep {
  bool on;
  hipStream_t s;
  TimedStep(const char* name, hipStream_t st) : on(g_timer.armed && g_timer.name == name), s(st) {
    if (on) on = hipEventRecord(g_timer.start, s) == hipSuccess;
  }
  ~TimedStep() {
    if (on) {
      (void)hipEventRecord(g_timer.stop, s);
      g_timer.armed = false;
    }
  }
};

// Runs a launch (or a short sequence) as one timed step.
#define FGS_TIMED(name, stream, expr, where) \
  do {                                       \
    TimedStep timed_(name, stream);          \
    FGS_HIP(expr, where);                    \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

// 16-bit sort keys when every global tile id and the out-of-range id `tiles`
// fit in them, else 32-bit.
static int tile_key_bytes(uint64_t tiles) { return tiles < 65536 ? 2 : 4; }

int tile_key_bits(uint64_t tiles) {
  int b = 1;
  while (b < 32 && (uint64_t(1) << b) < tiles) ++b;
  return b;
}

fgs_status check_camera(const fgs_camera* cam) {
  if (!cam) return fail(FGS_ERR_INVALID_ARGUMENT, "camera is NULL");
  if (cam->width <= 0 || cam->height <= 0)
    return fail(FGS_ERR_INVALID_ARGUMENT, "image size %dx%d must be positive", cam->width, cam->height);
  if ((int64_t)cam->width * cam->height > (int64_t(1) << 30))
    return fail(FGS_ERR_INVALID_ARGUMENT, "image of %dx%d pixels exceeds 2^30 pixels", cam->width, cam->height);
  if (!finite_pos(cam->fx) || !finite_pos(cam->fy))
    return fail(FGS_ERR_INVALID_ARGUMENT, "focal lengths must be finite and positive");
  if (!std::isfinite(cam->cx) || !std::isfinite(cam->cy))
    return fail(FGS_ERR_INVALID_ARGUMENT, "principal point must be finite");
  // z > 0 for every rendered Gaussian makes the float bits of z an ordered key
  if (!finite_pos(cam->near_z)) return fail(FGS_ERR_INVALID_ARGUMENT, "near plane must be finite and > 0");
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(cam->world_to_cam[k]))
      return fail(FGS_ERR_INVALID_ARGUMENT, "world_to_cam[%d] is not finite", k);
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(cam->bg[k])) return fail(FGS_ERR_INVALID_ARGUMENT, "bg[%d] is not finite", k);
  return FGS_OK;
}

fgs_status check_settings(const fgs_settings* st) {
  if (!st) return fail(FGS_ERR_INVALID_ARGUMENT, "settings is NULL");
  if (st->tile != 8 && st->tile != 16 && st->tile != 32)
    return fail(FGS_ERR_INVALID_ARGUMENT, "tile must be 8, 16 or 32 (got %d)", st->tile);
  if (st->flags &
      ~(uint32_t)(FGS_FLAG_FP64_CONIC | FGS_FLAG_LOOKBACK_FALLBACK | FGS_FLAG_BLEND_QUEUE | FGS_FLAG_SORT_LARGE_BLOCKS |
                  FGS_FLAG_KEEP_ACCUM_ZERO))
    return fail(FGS_ERR_INVALID_ARGUMENT, "unknown bits in settings.flags 0x%x", st->flags);
  // alpha_max < 1: the backward divides by 1 - alpha (App. B.1's front-to-back
  // gradient), which the cap keeps at least 1 - alpha_max away from zero
  if (!(st->alpha_min > 0.0f && st->alpha_min < st->alpha_max && st->alpha_max < 1.0f))
    return fail(FGS_ERR_INVALID_ARGUMENT, "need 0 < alpha_min < alpha_max < 1");
  if (!(st->t_min > 0.0f && st->t_min < 1.0f)) return fail(FGS_ERR_INVALID_ARGUMENT, "need 0 < t_min < 1");
  if (!(st->dilation >= 0.0f && std::isfinite(st->dilation)))
    return fail(FGS_ERR_INVALID_ARGUMENT, "dilation must be finite and >= 0");
  if (!(st->quat_min >= 0.0f && std::isfinite(st->quat_min)) || !(st->det_min >= 0.0f && std::isfinite(st->det_min)))
    return fail(FGS_ERR_INVALID_ARGUMENT, "quat_min and det_min must be finite and >= 0");
  return FGS_OK;
}

fgs_status check_gaussians(const fgs_gaussians* g) {
  if (!g) return fail(FGS_ERR_INVALID_ARGUMENT, "gaussians is NULL");
  if (g->n < 0 || g->n > INT32_MAX) return fail(FGS_ERR_INVALID_ARGUMENT, "n = %lld out of range", (long long)g->n);
  if (g->sh_dtype != FGS_F32 && g->sh_dtype != FGS_BF16)
    return fail(FGS_ERR_INVALID_ARGUMENT, "unknown sh_dtype %d", g->sh_dtype);
  if (g->sh_degree < 0 || g->sh_degree > 3)
    return fail(FGS_ERR_INVALID_ARGUMENT, "sh_degree %d not in 0..3", g->sh_degree);
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh_dc ||
                   (g->sh_degree > 0 && !g->sh_rest)))
    return fail(FGS_ERR_INVALID_ARGUMENT, "a parameter pointer is NULL");
  if ((g->velocity == nullptr) != (g->accel == nullptr))
    return fail(FGS_ERR_INVALID_ARGUMENT, "velocity and accel are given together or not at all");
  const int n4 = (g->mean_t != nullptr) + (g->log_scale_t != nullptr) + (g->quats_r != nullptr);
  if (n4 != 0 && n4 != 3)
    return fail(FGS_ERR_INVALID_ARGUMENT, "mean_t, log_scale_t and quats_r are given together or not at all");
  if (n4 == 3 && g->velocity != nullptr)
    return fail(FGS_ERR_INVALID_ARGUMENT, "conditional 4D Gaussians take no velocity or accel");
  return FGS_OK;
}

// Workspace of n Gaussians seen from n_views cameras (index j = v n + i for
// the per-(view, Gaussian) regions) with room for `cap` instances.
fgs_status make_layout(int64_t n, const fgs_camera* cams, int32_t n_views, const fgs_settings* st, int64_t cap,
                       fgs_layout* L) {
  if (n < 0 || n > INT32_MAX) return fail(FGS_ERR_INVALID_ARGUMENT, "n = %lld out of range", (long long)n);
  // the device sorts take fewer than 2^30 pairs (32-bit byte offsets)
  if (cap < 0 || cap >= kMaxSortPairs)
    return fail(FGS_ERR_INVALID_ARGUMENT, "instance_capacity = %lld not below 2^30", (long long)cap);
  if (n_views < 1 || n_views > kMaxViews)
    return fail(FGS_ERR_INVALID_ARGUMENT, "n_views = %d not in 1..%d", n_views, kMaxViews);
  if (!cams) return fail(FGS_ERR_INVALID_ARGUMENT, "cameras are NULL");
  if ((int64_t)n * n_views >= kMaxSortPairs)
    return fail(FGS_ERR_INVALID_ARGUMENT, "n * n_views = %lld not below 2^30", (long long)n * n_views);
  fgs_status s = check_settings(st);
  if (s != FGS_OK) return s;
  const int t = st->tile;
  uint64_t tiles = 0;
  for (int v = 0; v < n_views; ++v) {
    s = check_camera(cams + v);
    if (s != FGS_OK) return s;
    const int64_t tx = (cams[v].width + t - 1) / t, ty = (cams[v].height + t - 1) / t;
    if (tx > 65535 || ty > 65535) return fail(FGS_ERR_INVALID_ARGUMENT, "tile grid too large");
    tiles += (uint64_t)(tx * ty);
  }
  if (tiles > (uint64_t(1) << 30)) return fail(FGS_ERR_INVALID_ARGUMENT, "more than 2^30 tiles");
  std::memset(L, 0, sizeof(*L));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t un = (size_t)n, vn = un * (size_t)n_views, uc = (size_t)cap;
  L->rec = take(vn * 64);
  L->n_tiles = take(vn * 4);
  L->depth_key = take(vn * 4);
  L->counters = take(64);
  L->vis_keys[0] = take(vn * 4);
  L->vis_keys[1] = take(vn * 4);
  L->vis_ids[0] = take(vn * 4);
  L->vis_ids[1] = take(vn * 4);
  L->dup_scan = take(dup_scan_words(vn) * 4);
  const int key_bytes = tile_key_bytes(tiles);
  L->inst_keys[0] = take(uc * key_bytes);
  L->inst_keys[1] = take(uc * key_bytes);
  L->inst_vals[0] = take(uc * 4);
  L->inst_vals[1] = take(uc * 4);
  L->ranges = take(tiles * 8);
  L->accum = take(vn * 9 * 4);
  L->marks = take(vn);  // directly after accum: one fill clears both
  L->touched = take((un + 3) / 4);
  L->touched_list = take(un * 4);
  L->slot_of = take(un * 4);
  L->sparse_grads = take(un * 59 * 4);
  L->queues = take(kQueueWords * 4);
  size_t words = radix_scratch_words(vn);
  words = std::max(words, radix_scratch_words(uc));
  words = std::max(words, stats_scratch_words((uint32_t)((size_t)n_views * ((un + kBlock - 1) / kBlock))));
  L->scratch = take(words * 4 + 256);
  L->total = off;
  L->inst_final = ((tile_key_bits(tiles) + kRadixBits - 1) / kRadixBits) & 1;
  L->inst_key_bytes = key_bytes;
  L->tiles_x = (int32_t)((cams[0].width + t - 1) / t);
  L->tiles_y = (int32_t)((cams[0].height + t - 1) / t);
  L->instance_capacity = cap;
  L->n_views = n_views;
  L->total_tiles = (int64_t)tiles;
  return FGS_OK;
}

CamDev make_cam(const fgs_camera* c, int tile) {
  CamDev d;
  for (int k = 0; k < 12; ++k) d.w[k] = c->world_to_cam[k];
  // camera centre -W3^T t, computed in double and rounded once
  for (int k = 0; k < 3; ++k) {
    double v = 0.0;
    for (int r = 0; r < 3; ++r) v -= (double)c->world_to_cam[4 * r + k] * (double)c->world_to_cam[4 * r + 3];
    d.campos[k] = (float)v;
  }
  d.fx = c->fx; d.fy = c->fy; d.cx = c->cx; d.cy = c->cy;
  d.width = c->width; d.height = c->height;
  d.tiles_x = (c->width + tile - 1) / tile;
  d.tiles_y = (c->height + tile - 1) / tile;
  d.near_z = c->near_z;
  for (int k = 0; k < 3; ++k) d.bg[k] = c->bg[k];
  return d;
}

ViewSet make_views(const fgs_camera* cams, int32_t n_views, int tile, const float* times) {
  ViewSet vs;
  std::memset(&vs, 0, sizeof(vs));
  vs.n_views = (uint32_t)n_views;
  uint32_t tb = 0;
  uint64_t pb = 0;
  for (int v = 0; v < n_views; ++v) {
    vs.cam[v] = make_cam(cams + v, tile);
    vs.time[v] = times ? times[v] : 0.0f;
    vs.tile_base[v] = tb;
    vs.pix_base[v] = pb;
    tb += (uint32_t)(vs.cam[v].tiles_x * vs.cam[v].tiles_y);
    pb += (uint64_t)cams[v].width * (uint64_t)cams[v].height;
  }
  vs.tile_base[n_views] = tb;
  vs.pix_base[n_views] = pb;
  return vs;
}

SetDev make_set(const fgs_settings* s) {
  return SetDev{s->alpha_min, s->alpha_max, s->t_min, s->dilation, s->quat_min, s->det_min,
                (s->flags & FGS_FLAG_FP64_CONIC) ? 1 : 0};
}

GaussDev make_gauss(const fgs_gaussians* g) {
  GaussDev d;
  d.means = g->means;
  d.log_scales = g->log_scales;
  d.quats = g->quats;
  d.logits = g->opacity_logits;
  d.sh_dc = g->sh_dc;
  d.sh_rest = g->sh_rest;
  d.n = (uint32_t)g->n;
  d.sh_coeffs = (g->sh_degree + 1) * (g->sh_degree + 1);
  d.sh_bf16 = g->sh_dtype == FGS_BF16 ? 1 : 0;
  d.velocity = g->velocity;
  d.accel = g->accel;
  d.mean_t = g->mean_t;
  d.log_scale_t = g->log_scale_t;
  d.quats_r = g->quats_r;
  return d;
}

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// The blend's tile queues when the settings ask for them, else NULL.
uint32_t* blend_queues(const fgs_settings* st, void* workspace, const fgs_layout& L) {
  return (st->flags & FGS_FLAG_BLEND_QUEUE) ? at<uint32_t>(workspace, L.queues) : nullptr;
}

}  // namespace

extern "C" {

int32_t fgs_abi_version(void) { return FGS_ABI_VERSION; }

const char* fgs_status_string(fgs_status s) {
  switch (s) {
    case FGS_OK: return "ok";
    case FGS_ERR_INVALID_ARGUMENT: return "invalid argument";
    case FGS_ERR_CAPACITY: return "instance capacity exceeded";
    case FGS_ERR_HIP: return "HIP runtime error";
    case FGS_ERR_UNSUPPORTED: return "unsupported option";
  }
  return "unknown status";
}

const char* fgs_last_error(void) { return g_last_error.c_str(); }

fgs_status fgs_default_settings(fgs_settings* out) {
  if (!out) return fail(FGS_ERR_INVALID_ARGUMENT, "out is NULL");
  out->tile = 16;
  out->alpha_min = 1.0f / 255.0f;
  out->alpha_max = 0.99f;
  out->t_min = 1e-4f;
  out->dilation = 0.3f;
  out->quat_min = 1e-4f;
  out->det_min = 1e-6f;
  out->flags = 0;
  return FGS_OK;
}

fgs_status fgs_workspace_size(int64_t n, const fgs_camera* cam, const fgs_settings* st, int64_t instance_capacity,
                              size_t* bytes) {
  return fgs_batch_workspace_size(n, cam, 1, st, instance_capacity, bytes);
}

fgs_status fgs_workspace_layout(int64_t n, const fgs_camera* cam, const fgs_settings* st, int64_t instance_capacity,
                                fgs_layout* out) {
  return fgs_batch_workspace_layout(n, cam, 1, st, instance_capacity, out);
}

fgs_status fgs_batch_workspace_size(int64_t n, const fgs_camera* cams, int32_t n_views, const fgs_settings* st,
                                    int64_t instance_capacity, size_t* bytes) {
  if (!bytes) return fail(FGS_ERR_INVALID_ARGUMENT, "bytes is NULL");
  fgs_layout L;
  fgs_status s = make_layout(n, cams, n_views, st, instance_capacity, &L);
  if (s != FGS_OK) return s;
  *bytes = L.total;
  return FGS_OK;
}

fgs_status fgs_batch_workspace_layout(int64_t n, const fgs_camera* cams, int32_t n_views, const fgs_settings* st,
                                      int64_t instance_capacity, fgs_layout* out) {
  if (!out) return fail(FGS_ERR_INVALID_ARGUMENT, "out is NULL");
  return make_layout(n, cams, n_views, st, instance_capacity, out);
}

fgs_status fgs_rasterize_forward(const fgs_gaussians* g, const fgs_camera* cam, const fgs_settings* st,
                                 void* workspace, size_t workspace_bytes, int64_t instance_capacity, float* image,
                                 float* t_final, uint32_t* last, fgs_forward_stats* stats, void* stream) {
  if (g && (g->velocity || g->accel || g->quats_r))
    return fail(FGS_ERR_INVALID_ARGUMENT, "dynamic Gaussians take fgs_rasterize_forward_batch with times");
  return fgs_rasterize_forward_batch(g, cam, nullptr, 1, st, workspace, workspace_bytes, instance_capacity, image,
                                     t_final, last, 0u, stats, stream);
}

fgs_status fgs_rasterize_forward_batch(const fgs_gaussians* g, const fgs_camera* cams, const float* times,
                                       int32_t n_views, const fgs_settings* st, void* workspace,
                                       size_t workspace_bytes, int64_t instance_capacity, float* images,
                                       float* t_finals, uint32_t* lasts, uint32_t mode, fgs_forward_stats* stats,
                                       void* stream) {
  fgs_status s = check_gaussians(g);
  if (s != FGS_OK) return s;
  fgs_layout L;
  s = make_layout(g->n, cams, n_views, st, instance_capacity, &L);
  if (s != FGS_OK) return s;
  if (mode & ~(uint32_t)(FGS_FORWARD_NO_SYNC | FGS_FORWARD_DEPTH_BITS(0x3f)))
    return fail(FGS_ERR_INVALID_ARGUMENT, "unknown mode bits 0x%x", mode);
  const bool no_sync = (mode & FGS_FORWARD_NO_SYNC) != 0;
  const int depth_hint = (int)((mode >> 8) & 0x3fu);
  if (depth_hint > 31) return fail(FGS_ERR_INVALID_ARGUMENT, "FGS_FORWARD_DEPTH_BITS(%d) not in 1..31", depth_hint);
  if (depth_hint && !no_sync)
    return fail(FGS_ERR_INVALID_ARGUMENT, "FGS_FORWARD_DEPTH_BITS goes with FGS_FORWARD_NO_SYNC");
  if (!workspace) return fail(FGS_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (workspace_bytes < L.total)
    return fail(FGS_ERR_INVALID_ARGUMENT, "workspace holds %zu bytes, %zu needed", workspace_bytes, L.total);
  if ((uintptr_t)workspace % 256) return fail(FGS_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  if (!images || !lasts) return fail(FGS_ERR_INVALID_ARGUMENT, "images and lasts are required");
  if (times)
    for (int v = 0; v < n_views; ++v)
      if (!std::isfinite(times[v])) return fail(FGS_ERR_INVALID_ARGUMENT, "times[%d] is not finite", v);

  hipStream_t hs = static_cast<hipStream_t>(stream);
  const GaussDev gd = make_gauss(g);
  const ViewSet vs = make_views(cams, n_views, st->tile, times);
  const SetDev sd = make_set(st);
  const uint32_t n = gd.n;
  const uint32_t vn = n * (uint32_t)n_views;
  float4* rec = at<float4>(workspace, L.rec);
  uint32_t* n_tiles = at<uint32_t>(workspace, L.n_tiles);
  uint32_t* depth_key = at<uint32_t>(workspace, L.depth_key);
  uint32_t* counters = at<uint32_t>(workspace, L.counters);
  uint32_t* vis_keys[2] = {at<uint32_t>(workspace, L.vis_keys[0]), at<uint32_t>(workspace, L.vis_keys[1])};
  uint32_t* vis_ids[2] = {at<uint32_t>(workspace, L.vis_ids[0]), at<uint32_t>(workspace, L.vis_ids[1])};
  uint32_t* dup_scan = at<uint32_t>(workspace, L.dup_scan);
  void* ikeys[2] = {at<uint8_t>(workspace, L.inst_keys[0]), at<uint8_t>(workspace, L.inst_keys[1])};
  const int key_bytes = L.inst_key_bytes;
  uint32_t* ivals[2] = {at<uint32_t>(workspace, L.inst_vals[0]), at<uint32_t>(workspace, L.inst_vals[1])};
  uint2* ranges = at<uint2>(workspace, L.ranges);
  uint32_t* scratch = at<uint32_t>(workspace, L.scratch);
  const uint32_t tiles = (uint32_t)L.total_tiles;
  const uint32_t cap = (uint32_t)instance_capacity;

  // Statistics after the preprocess: the visible count, the instance count I
  // and the depth-key range.  By default the host reads them once (one
  // synchronisation) to size every later launch; with FGS_FORWARD_NO_SYNC
  // every launch is sized by the capacities and reads the counts on the device.
  uint32_t stats_host[8] = {0, 0xffffffffu, 0, 0, 0, 0, 0, 0};
  if (n > 0) {
    uint4* partials = reinterpret_cast<uint4*>(scratch);  // free until the compaction scan
    FGS_TIMED("preprocess", hs, launch_preprocess(gd, vs, sd, st->tile, rec, n_tiles, depth_key, partials, hs),
              "preprocess");
    // without a host synchronisation the depth sort covers the hinted bits
    // (all 31 without a hint); keys differing above them are flagged
    FGS_HIP(launch_stats(partials, (uint32_t)n_views * ceil_div(n, kBlock), (uint64_t)cap,
                         no_sync ? (depth_hint ? depth_hint : 31) : 32, counters, hs),
            "stats");
    if (!no_sync) {
      FGS_HIP(hipMemcpyAsync(stats_host, counters, sizeof(stats_host), hipMemcpyDeviceToHost, hs), "stats copy");
      FGS_HIP(hipStreamSynchronize(hs), "stats sync");
    }
  } else {
    FGS_HIP(launch_fill_u32(counters, 0u, 8, hs), "counters clear");
  }
  uint32_t nvis = vn;  // capacity of the visible list
  uint64_t inst64 = cap;
  int depth_bits = depth_hint ? depth_hint : 31;  // z > 0: the sign bit of every key is 0
  if (!no_sync) {
    nvis = stats_host[kStatVisible];
    std::memcpy(&inst64, stats_host + kStatInstances, sizeof(inst64));
    const uint32_t span = stats_host[kStatKeyMax] - stats_host[kStatKeyMin];  // of the offset keys
    depth_bits = span ? 32 - __builtin_clz(span) : 0;
    if (stats) {
      stats->n_visible = nvis;
      stats->n_instances = (int64_t)inst64;
      stats->tiles_x = L.tiles_x;
      stats->tiles_y = L.tiles_y;
      stats->depth_key_bits = nvis > 0 ? depth_bits : 0;
    }
    if (inst64 > (uint64_t)instance_capacity)
      return fail(FGS_ERR_CAPACITY, "%llu instances exceed the capacity of %lld", (unsigned long long)inst64,
                  (long long)instance_capacity);
  } else if (stats) {
    stats->n_visible = -1;
    stats->n_instances = -1;
    stats->tiles_x = L.tiles_x;
    stats->tiles_y = L.tiles_y;
    stats->depth_key_bits = -1;
  }
  const uint32_t* d_vis = counters + kStatVisible;
  const uint32_t* d_sorted = no_sync ? counters + kStatSortCount : nullptr;
  const uint32_t inst = (uint32_t)inst64;

  int vis_final = 0;
  if (nvis > 0) {
    // visible compaction (block offsets from the statistics, index order kept) and the depth
    // sort over the key bits that vary among the visible entries
    // (the compacted keys are offset by the smallest visible key: they span [0, max - min])
    // (and the compaction clears the look-back words and the tile ranges)
    FGS_HIP(launch_compact_visible(n_tiles, depth_key, n, (uint32_t)n_views, reinterpret_cast<uint4*>(scratch),
                                   counters + kStatKeyMin, vis_keys[0], vis_ids[0], dup_scan, dup_scan_words(vn),
                                   reinterpret_cast<uint32_t*>(ranges), (size_t)tiles * 2, hs),
            "compact");
    // with the device's key span, trailing passes whose digit every visible key shares are
    // skipped, and the buffer holding the sorted ids is noted in counters[kStatDepthBuf]
    // (0, set by the statistics, when no pass runs)
    FGS_HIP(radix_sort_pairs(vis_keys, vis_ids, nvis, no_sync ? d_vis : nullptr, 0, depth_bits, scratch, &vis_final,
                             hs, counters + kStatKeySpan, false, counters + kStatDepthBuf),
            "depth sort");
  }

  if (nvis == 0) {  // no compaction ran to clear the tile ranges
    FGS_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, (uint64_t)tiles * 2, hs), "ranges clear");
  }
  if (inst > 0 && nvis > 0) {
    const uint32_t* depth_ids[2] = {vis_ids[0], vis_ids[1]};
    FGS_TIMED("duplicate", hs,
              launch_duplicate(depth_ids, counters + kStatDepthBuf, d_vis, nvis, dup_scan, dup_scan,
                               (st->flags & FGS_FLAG_LOOKBACK_FALLBACK) != 0, rec, vs, n, st->tile, cap,
                               ikeys[0], key_bytes, ivals[0], hs),
              "duplicate");
    int inst_final = 0;
    const int bits = tile_key_bits(tiles);
    const bool large_blocks = (st->flags & FGS_FLAG_SORT_LARGE_BLOCKS) != 0;
    if (key_bytes == 2) {
      uint16_t* k16[2] = {static_cast<uint16_t*>(ikeys[0]), static_cast<uint16_t*>(ikeys[1])};
      FGS_TIMED("tile_sort", hs,
                radix_sort_pairs16(k16, ivals, inst, d_sorted, 0, bits, scratch, &inst_final, hs, large_blocks),
                "tile sort");
    } else {
      uint32_t* k32[2] = {static_cast<uint32_t*>(ikeys[0]), static_cast<uint32_t*>(ikeys[1])};
      FGS_TIMED("tile_sort", hs,
                radix_sort_pairs(k32, ivals, inst, d_sorted, 0, bits, scratch, &inst_final, hs, nullptr, true,
                                 nullptr, large_blocks),
                "tile sort");
    }
    if (inst_final != L.inst_final) return fail(FGS_ERR_HIP, "internal: tile sort buffer mismatch");
    FGS_HIP(launch_tile_ranges(ikeys[inst_final], key_bytes, inst, d_sorted, tiles, ranges, hs), "tile ranges");
  }
  FGS_TIMED("blend_forward", hs,
            launch_blend_forward(ranges, ivals[L.inst_final], rec, vs, sd, st->tile, images, t_finals, lasts,
                                 blend_queues(st, workspace, L), hs),
            "blend");
  return FGS_OK;
}

// Checks shared by the backward entry points; on success fills the layout.
static fgs_status check_backward(const fgs_gaussians* g, const fgs_camera* cams, int32_t n_views,
                                 const fgs_settings* st, void* workspace, size_t workspace_bytes,
                                 int64_t instance_capacity, const float* image, const uint32_t* last,
                                 const float* dl_dimage, fgs_layout* L) {
  fgs_status s = check_gaussians(g);
  if (s != FGS_OK) return s;
  s = make_layout(g->n, cams, n_views, st, instance_capacity, L);
  if (s != FGS_OK) return s;
  if (!workspace) return fail(FGS_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (workspace_bytes < L->total)
    return fail(FGS_ERR_INVALID_ARGUMENT, "workspace holds %zu bytes, %zu needed", workspace_bytes, L->total);
  if ((uintptr_t)workspace % 256) return fail(FGS_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  if (!image || !last || !dl_dimage) return fail(FGS_ERR_INVALID_ARGUMENT, "image, last and dl_dimage are required");
  return FGS_OK;
}

// The tag of a layout's accumulator state (the pair kStatAccumClean holds
// {kAccumClean, tag} while accum and marks are known to be zero): the
// accumulators' place and extent.
static uint32_t accum_tag(const fgs_layout& L, uint64_t vn) {
  uint64_t h = (uint64_t)L.total * 0x9e3779b97f4a7c15ull ^ (uint64_t)L.accum * 0xc2b2ae3d27d4eb4full ^
               (uint64_t)L.marks * 0x165667b19e3779f9ull ^ vn;
  h ^= h >> 29;
  h *= 0xbf58476d1ce4e5b9ull;
  return (uint32_t)(h ^ (h >> 32)) | 1u;
}

static bool keep_accum_zero(const fgs_settings* st) { return (st->flags & FGS_FLAG_KEEP_ACCUM_ZERO) != 0; }

// Clears the accumulators (with FGS_FLAG_KEEP_ACCUM_ZERO: unless they are
// known to be zero) and runs the blend backward over all views' tiles
// (per-(view, Gaussian) 2D gradients into accum[n_views n][9]); the
// accumulators are then no longer known to be zero.
static fgs_status blend_backward(const fgs_gaussians* g, const ViewSet& vs, const fgs_settings* st, void* workspace,
                                 const fgs_layout& L, const float* images, const uint32_t* lasts,
                                 const float* dl_dimages, hipStream_t hs, uint32_t* reset_word = nullptr) {
  const uint32_t vn = (uint32_t)g->n * vs.n_views;
  const SetDev sd = make_set(st);
  float4* rec = at<float4>(workspace, L.rec);
  uint2* ranges = at<uint2>(workspace, L.ranges);
  uint32_t* ivals = at<uint32_t>(workspace, L.inst_vals[L.inst_final]);
  float* accum = at<float>(workspace, L.accum);
  uint8_t* marks = at<uint8_t>(workspace, L.marks);
  uint32_t* clean = at<uint32_t>(workspace, L.counters) + kStatAccumClean;
  // accum and the marks after it, one clear (skipped on the device when the
  // last backward on this layout left them zero)
  const uint64_t clear_words = (L.marks - L.accum) / 4 + ((uint64_t)vn + 3) / 4;
  if (keep_accum_zero(st))
    FGS_HIP(launch_clear_unless(reinterpret_cast<uint32_t*>(accum), clear_words, clean, accum_tag(L, vn), hs),
            "accum clear");
  else
    FGS_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(accum), 0u, clear_words, hs), "accum clear");
  FGS_TIMED("blend_backward", hs,
            launch_blend_backward(ranges, ivals, rec, vs, sd, st->tile, images, lasts, dl_dimages, accum, marks,
                                  reset_word, clean, vn, blend_queues(st, workspace, L), hs),
            "blend bwd");
  return FGS_OK;
}

// After a backward whose chain rule cleared every row and mark it read: the
// accumulators are known to be zero again.
static fgs_status note_accum_clean(void* workspace, const fgs_layout& L, uint64_t vn, hipStream_t hs) {
  uint32_t* clean = at<uint32_t>(workspace, L.counters) + kStatAccumClean;
  FGS_HIP(launch_fill_u32(clean, kAccumClean, 1, hs, clean + 1, accum_tag(L, vn)), "accum state");
  return FGS_OK;
}

static GradDev grad_dev(const fgs_gaussian_grads* grads) {
  GradDev gr;
  gr.means = grads->means;
  gr.log_scales = grads->log_scales;
  gr.quats = grads->quats;
  gr.logits = grads->opacity_logits;
  gr.sh_dc = grads->sh_dc;
  gr.sh_rest = grads->sh_rest;
  gr.velocity = grads->velocity;
  gr.accel = grads->accel;
  gr.mean_t = grads->mean_t;
  gr.log_scale_t = grads->log_scale_t;
  gr.quats_r = grads->quats_r;
  return gr;
}

fgs_status fgs_rasterize_backward(const fgs_gaussians* g, const fgs_camera* cam, const fgs_settings* st,
                                  void* workspace, size_t workspace_bytes, int64_t instance_capacity,
                                  const float* image, const uint32_t* last, const float* dl_dimage,
                                  const fgs_gaussian_grads* grads, void* stream) {
  if (g && (g->velocity || g->accel || g->quats_r))
    return fail(FGS_ERR_INVALID_ARGUMENT, "dynamic Gaussians take fgs_rasterize_backward_batch with times");
  return fgs_rasterize_backward_batch(g, cam, nullptr, 1, st, workspace, workspace_bytes, instance_capacity, image,
                                      last, dl_dimage, grads, stream);
}

fgs_status fgs_rasterize_backward_batch(const fgs_gaussians* g, const fgs_camera* cams, const float* times,
                                        int32_t n_views, const fgs_settings* st, void* workspace,
                                        size_t workspace_bytes, int64_t instance_capacity, const float* images,
                                        const uint32_t* lasts, const float* dl_dimages,
                                        const fgs_gaussian_grads* grads, void* stream) {
  fgs_layout L;
  fgs_status s = check_backward(g, cams, n_views, st, workspace, workspace_bytes, instance_capacity, images, lasts,
                                dl_dimages, &L);
  if (s != FGS_OK) return s;
  if (!grads) return fail(FGS_ERR_INVALID_ARGUMENT, "grads is NULL");
  if (g->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits ||
                   !grads->sh_dc || !grads->sh_rest))
    return fail(FGS_ERR_INVALID_ARGUMENT, "a gradient pointer is NULL");
  const bool dyn = g->velocity != nullptr, cond4 = g->quats_r != nullptr;
  if (dyn && g->n > 0 && (!grads->velocity || !grads->accel))
    return fail(FGS_ERR_INVALID_ARGUMENT, "dynamic Gaussians need velocity and accel gradients");
  if (cond4 && g->n > 0 && (!grads->mean_t || !grads->log_scale_t || !grads->quats_r))
    return fail(FGS_ERR_INVALID_ARGUMENT, "conditional 4D Gaussians need mean_t, log_scale_t and quats_r gradients");
  if (g->n == 0) return FGS_OK;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const ViewSet vs = make_views(cams, n_views, st->tile, times);
  s = blend_backward(g, vs, st, workspace, L, images, lasts, dl_dimages, hs);
  if (s != FGS_OK) return s;
  const GradDev gr = grad_dev(grads);
  const GaussDev gd = make_gauss(g);
  if (n_views == 1 && !dyn && !cond4) {
    FGS_TIMED("preprocess_backward", hs,
              launch_preprocess_backward(gd, vs.cam[0], at<float4>(workspace, L.rec), at<float>(workspace, L.accum),
                                         gr, hs),
              "preprocess bwd");
  } else {
    FGS_TIMED("preprocess_backward", hs,
              launch_preprocess_backward_views(gd, vs, at<float4>(workspace, L.rec), at<float>(workspace, L.accum),
                                               at<uint8_t>(workspace, L.marks), gr, keep_accum_zero(st), hs),
              "preprocess bwd (views)");
    if (keep_accum_zero(st)) return note_accum_clean(workspace, L, (uint64_t)g->n * n_views, hs);
  }
  return FGS_OK;
}

static fgs_status check_adam_hyper(int64_t step, double beta1, double beta2, double eps) {
  if (step < 1) return fail(FGS_ERR_INVALID_ARGUMENT, "step must be >= 1");
  if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0))
    return fail(FGS_ERR_INVALID_ARGUMENT, "betas must lie in [0, 1)");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(FGS_ERR_INVALID_ARGUMENT, "eps must be finite, >= 0");
  return FGS_OK;
}

fgs_status fgs_rasterize_backward_adam(const fgs_gaussians* g, const fgs_camera* cam, const fgs_settings* st,
                                       void* workspace, size_t workspace_bytes, int64_t instance_capacity,
                                       const float* image, const uint32_t* last, const float* dl_dimage,
                                       const fgs_adam_moments* opt, int64_t step, double beta1, double beta2,
                                       double eps, void* stream) {
  fgs_layout L;
  fgs_status s = check_backward(g, cam, 1, st, workspace, workspace_bytes, instance_capacity, image, last, dl_dimage,
                                &L);
  if (s != FGS_OK) return s;
  if (g->velocity || g->accel || g->quats_r)
    return fail(FGS_ERR_UNSUPPORTED, "the fused backward + Adam takes static Gaussians");
  if (!opt) return fail(FGS_ERR_INVALID_ARGUMENT, "opt is NULL");
  s = check_adam_hyper(step, beta1, beta2, eps);
  if (s != FGS_OK) return s;
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(opt->lr[k])) return fail(FGS_ERR_INVALID_ARGUMENT, "lr[%d] not finite", k);
  if (g->n == 0) return FGS_OK;
  if (!g->sh_rest) return fail(FGS_ERR_INVALID_ARGUMENT, "sh_rest (all 45 planes) is required");
  for (int k = 0; k < 6; ++k)
    if (!opt->exp_avg[k] || !opt->exp_avg_sq[k]) return fail(FGS_ERR_INVALID_ARGUMENT, "moment %d is NULL", k);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  const ViewSet vs = make_views(cam, 1, st->tile, nullptr);
  uint32_t* touch_count = at<uint32_t>(workspace, L.counters) + kStatTouched;
  s = blend_backward(g, vs, st, workspace, L, image, last, dl_dimage, hs, touch_count);
  if (s != FGS_OK) return s;
  void* const params[6] = {const_cast<float*>(g->means), const_cast<float*>(g->log_scales),
                           const_cast<float*>(g->quats), const_cast<float*>(g->opacity_logits),
                           const_cast<void*>(g->sh_dc), const_cast<void*>(g->sh_rest)};
  const GaussDev gd = make_gauss(g);
  uint8_t* touched = at<uint8_t>(workspace, L.touched);
  uint32_t* slot_of = at<uint32_t>(workspace, L.slot_of);
  float* sparse = at<float>(workspace, L.sparse_grads);
  FGS_TIMED("touched_gradients", hs,
            launch_touched_gradients(gd, vs.cam[0], at<float4>(workspace, L.rec), at<float>(workspace, L.accum),
                                     at<uint8_t>(workspace, L.marks), touched, touch_count,
                                     at<uint32_t>(workspace, L.touched_list), slot_of, sparse, keep_accum_zero(st),
                                     hs),
            "touched gradients");
  // with FGS_FLAG_KEEP_ACCUM_ZERO the Adam launch also records that the
  // accumulators are zero again
  uint32_t* clean = keep_accum_zero(st) ? at<uint32_t>(workspace, L.counters) + kStatAccumClean : nullptr;
  FGS_TIMED("adam_sparse", hs,
            launch_adam_sparse(params, opt->exp_avg, opt->exp_avg_sq, opt->lr, gd.sh_bf16 != 0, gd.n, touched,
                               slot_of, sparse, step, beta1, beta2, eps, clean, accum_tag(L, (uint64_t)g->n), hs),
            "adam (sparse gradients)");
  return FGS_OK;
}

static fgs_status adam_impl(const fgs_adam_group* groups, int32_t n_groups, int64_t step, void* d_state,
                            double beta1, double beta2, double eps, void* stream);

fgs_status fgs_adam_step(const fgs_adam_group* groups, int32_t n_groups, int64_t step, double beta1, double beta2,
                         double eps, void* stream) {
  if (step < 1) return fail(FGS_ERR_INVALID_ARGUMENT, "step must be >= 1");
  return adam_impl(groups, n_groups, step, nullptr, beta1, beta2, eps, stream);
}

fgs_status fgs_adam_step_device(const fgs_adam_group* groups, int32_t n_groups, void* d_state, double beta1,
                                double beta2, double eps, void* stream) {
  if (!d_state || (uintptr_t)d_state % 8) return fail(FGS_ERR_INVALID_ARGUMENT, "d_state must be 8-byte aligned");
  return adam_impl(groups, n_groups, 0, d_state, beta1, beta2, eps, stream);
}

static fgs_status adam_impl(const fgs_adam_group* groups, int32_t n_groups, int64_t step, void* d_state,
                            double beta1, double beta2, double eps, void* stream) {
  if (!groups) return fail(FGS_ERR_INVALID_ARGUMENT, "groups is NULL");
  if (n_groups < 1 || n_groups > 16) return fail(FGS_ERR_INVALID_ARGUMENT, "n_groups %d not in 1..16", n_groups);
  fgs_status hs = check_adam_hyper(step > 0 ? step : 1, beta1, beta2, eps);
  if (hs != FGS_OK) return hs;
  for (int k = 0; k < n_groups; ++k) {
    const fgs_adam_group& G = groups[k];
    if (G.numel < 0) return fail(FGS_ERR_INVALID_ARGUMENT, "group %d: numel < 0", k);
    if (G.dtype != FGS_F32 && G.dtype != FGS_BF16) return fail(FGS_ERR_INVALID_ARGUMENT, "group %d: bad dtype", k);
    if (G.numel > 0 && (!G.param || !G.grad || !G.exp_avg || !G.exp_avg_sq))
      return fail(FGS_ERR_INVALID_ARGUMENT, "group %d: NULL pointer", k);
    if (!std::isfinite(G.lr)) return fail(FGS_ERR_INVALID_ARGUMENT, "group %d: lr not finite", k);
  }
  FGS_TIMED("adam", static_cast<hipStream_t>(stream),
            launch_adam(groups, n_groups, step, beta1, beta2, eps, d_state, static_cast<hipStream_t>(stream)),
            "adam");
  return FGS_OK;
}

fgs_status fgs_zorder_workspace_size(int64_t n, size_t* bytes) {
  if (!bytes) return fail(FGS_ERR_INVALID_ARGUMENT, "bytes is NULL");
  if (n < 0 || n >= kMaxSortPairs) return fail(FGS_ERR_INVALID_ARGUMENT, "n = %lld not in 0..2^30-1", (long long)n);
  *bytes = zorder_scratch_bytes((uint64_t)n);
  return FGS_OK;
}

fgs_status fgs_zorder_permutation(const float* means, int64_t n, void* workspace, size_t workspace_bytes,
                                  uint32_t* perm, void* stream) {
  if (n < 0 || n >= kMaxSortPairs) return fail(FGS_ERR_INVALID_ARGUMENT, "n = %lld not in 0..2^30-1", (long long)n);
  if (n == 0) return FGS_OK;
  if (!means || !workspace || !perm) return fail(FGS_ERR_INVALID_ARGUMENT, "NULL pointer");
  const size_t need = zorder_scratch_bytes((uint64_t)n);
  if (workspace_bytes < need)
    return fail(FGS_ERR_INVALID_ARGUMENT, "workspace holds %zu bytes, %zu needed", workspace_bytes, need);
  if ((uintptr_t)workspace % 256) return fail(FGS_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  FGS_HIP(launch_zorder(means, (uint32_t)n, workspace, perm, static_cast<hipStream_t>(stream)), "zorder");
  return FGS_OK;
}

fgs_status fgs_permute_planes(const void* src, void* dst, int64_t n, int32_t planes, int32_t elem_bytes,
                              const uint32_t* perm, void* stream) {
  if (n < 0 || n > INT32_MAX) return fail(FGS_ERR_INVALID_ARGUMENT, "n = %lld out of range", (long long)n);
  if (planes < 0 || planes > 65535) return fail(FGS_ERR_INVALID_ARGUMENT, "planes %d not in 0..65535", planes);
  if (elem_bytes != 2 && elem_bytes != 4) return fail(FGS_ERR_INVALID_ARGUMENT, "elem_bytes must be 2 or 4");
  if (n == 0 || planes == 0) return FGS_OK;
  if (!src || !dst || !perm) return fail(FGS_ERR_INVALID_ARGUMENT, "NULL pointer");
  const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst, len = (uintptr_t)n * planes * elem_bytes;
  if (a < b + len && b < a + len) return fail(FGS_ERR_INVALID_ARGUMENT, "src and dst overlap");
  FGS_HIP(launch_permute(src, dst, (uint32_t)n, planes, elem_bytes, perm, static_cast<hipStream_t>(stream)),
          "permute");
  return FGS_OK;
}

static size_t sort_workspace_bytes(uint64_t n, int key_bytes) {
  auto a256 = [](size_t b) { return (b + 255) & ~size_t(255); };
  return a256(n * key_bytes) + a256(n * 4) + a256(radix_scratch_words(n) * 4);
}

fgs_status fgs_sort_workspace_size(int64_t n, int32_t key_bytes, size_t* bytes) {
  if (!bytes) return fail(FGS_ERR_INVALID_ARGUMENT, "bytes is NULL");
  if (n < 0 || n >= kMaxSortPairs) return fail(FGS_ERR_INVALID_ARGUMENT, "n = %lld not in 0..2^30-1", (long long)n);
  if (key_bytes != 2 && key_bytes != 4) return fail(FGS_ERR_INVALID_ARGUMENT, "key_bytes must be 2 or 4");
  *bytes = sort_workspace_bytes((uint64_t)n, key_bytes);
  return FGS_OK;
}

fgs_status fgs_sort_pairs(void* keys, uint32_t* vals, int64_t n, int32_t key_bytes, int32_t key_bits,
                          void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 0 || n >= kMaxSortPairs) return fail(FGS_ERR_INVALID_ARGUMENT, "n = %lld not in 0..2^30-1", (long long)n);
  if (key_bytes != 2 && key_bytes != 4) return fail(FGS_ERR_INVALID_ARGUMENT, "key_bytes must be 2 or 4");
  if (key_bits < 0 || key_bits > 8 * key_bytes)
    return fail(FGS_ERR_INVALID_ARGUMENT, "key_bits %d not in 0..%d", key_bits, 8 * key_bytes);
  if (n == 0 || key_bits == 0) return FGS_OK;
  if (!keys || !vals || !workspace) return fail(FGS_ERR_INVALID_ARGUMENT, "NULL pointer");
  const size_t need = sort_workspace_bytes((uint64_t)n, key_bytes);
  if (workspace_bytes < need)
    return fail(FGS_ERR_INVALID_ARGUMENT, "workspace holds %zu bytes, %zu needed", workspace_bytes, need);
  if ((uintptr_t)workspace % 256) return fail(FGS_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  if ((uintptr_t)keys % 16 || (uintptr_t)vals % 16)
    return fail(FGS_ERR_INVALID_ARGUMENT, "keys and vals must be 16-byte aligned");
  const hipStream_t hs = static_cast<hipStream_t>(stream);
  const size_t key_region = ((size_t)n * key_bytes + 255) & ~size_t(255);
  const size_t val_region = ((size_t)n * 4 + 255) & ~size_t(255);
  char* w = static_cast<char*>(workspace);
  uint32_t* alt_vals = reinterpret_cast<uint32_t*>(w + key_region);
  uint32_t* scratch = reinterpret_cast<uint32_t*>(w + key_region + val_region);
  uint32_t* vbuf[2] = {vals, alt_vals};
  int final_buf = 0;
  if (key_bytes == 2) {
    uint16_t* kbuf[2] = {static_cast<uint16_t*>(keys), reinterpret_cast<uint16_t*>(w)};
    FGS_HIP(radix_sort_pairs16(kbuf, vbuf, (uint32_t)n, nullptr, 0, key_bits, scratch, &final_buf, hs), "sort");
  } else {
    uint32_t* kbuf[2] = {static_cast<uint32_t*>(keys), reinterpret_cast<uint32_t*>(w)};
    FGS_HIP(radix_sort_pairs(kbuf, vbuf, (uint32_t)n, nullptr, 0, key_bits, scratch, &final_buf, hs), "sort");
  }
  if (final_buf == 1) {
    FGS_HIP(hipMemcpyAsync(keys, w, (size_t)n * key_bytes, hipMemcpyDeviceToDevice, hs), "sort copy");
    FGS_HIP(hipMemcpyAsync(vals, alt_vals, (size_t)n * 4, hipMemcpyDeviceToDevice, hs), "sort copy");
  }
  return FGS_OK;
}

fgs_status fgs_time_next_launch(const char* step, void* start_event, void* stop_event) {
  static const char* const kSteps[] = {"preprocess",          "duplicate",
                                       "tile_sort",           "blend_forward",
                                       "blend_backward",      "preprocess_backward",
                                       "touched_gradients", "adam_sparse",
                                       "adam"};
  if (!step) {
    g_timer.armed = false;
    return FGS_OK;
  }
  bool known = false;
  for (const char* k : kSteps) known |= std::strcmp(k, step) == 0;
  if (!known) return fail(FGS_ERR_INVALID_ARGUMENT, "unknown step '%s'", step);
  if (!start_event || !stop_event) return fail(FGS_ERR_INVALID_ARGUMENT, "events must not be NULL");
  g_timer.name = step;
  g_timer.start = static_cast<hipEvent_t>(start_event);
  g_timer.stop = static_cast<hipEvent_t>(stop_event);
  g_timer.armed = true;
  return FGS_OK;
}

fgs_status fgs_l1_loss_backward(const float* image, const float* target, int64_t n, float* dl_dimage, double* loss,
                                void* stream) {
  if (n < 0 || n > UINT32_MAX) return fail(FGS_ERR_INVALID_ARGUMENT, "n out of range");
  if (n > 0 && (!image || !target || !dl_dimage)) return fail(FGS_ERR_INVALID_ARGUMENT, "NULL pointer");
  FGS_HIP(launch_l1_backward(image, target, (uint32_t)n, dl_dimage, loss, static_cast<hipStream_t>(stream)), "l1");
  return FGS_OK;
}

}  // extern "C"
