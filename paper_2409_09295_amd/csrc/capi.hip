// C ABI of libgsmi: argument validation, workspace planning and launches.
// Every entry point validates all arguments before enqueuing anything.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "gs_internal.h"

namespace gsmi {

namespace {
thread_local char g_last_error[512] = "";
thread_local hipEvent_t g_events[GS_KERNEL_COUNT][2] = {};
}

namespace {
std::atomic<int> g_tuning[GS_TUNE_COUNT] = {{1}, {1}, {GS_SCHEDULE_HEAVIEST_FIRST},
                                            {GS_SCHEDULE_HEAVIEST_FIRST}, {0}, {0}};
}

int tuning(int key) { return g_tuning[key].load(std::memory_order_relaxed); }

int resident_workgroups(const void* kernel, int block) {
  struct Entry {
    const void* kernel;
    int dev, block, resident;
  };
  static std::mutex mu;
  static std::vector<Entry> known;   // the query costs microseconds: once per kernel and device
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lock(mu);
  for (const Entry& k : known)
    if (k.kernel == kernel && k.dev == dev && k.block == block) return k.resident;
  int per_cu = 0, cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess)
    return 0;
  known.push_back({kernel, dev, block, per_cu * cus});
  return per_cu * cus;
}

TileSchedule tile_schedule(int schedule, const gs_bins& bins, int call, int n_tiles,
                           int resident) {
  TileSchedule t{bins.order, nullptr, (unsigned)n_tiles};
  if (schedule == GS_SCHEDULE_TILE_ID) t.order = nullptr;
  const bool persistent =
      schedule == GS_SCHEDULE_PERSISTENT || schedule == GS_SCHEDULE_PERSISTENT_HALF;
  if (persistent && bins.queue && resident > 0) {
    if (schedule == GS_SCHEDULE_PERSISTENT_HALF) resident = std::max(1, resident / 2);
    t.counter = bins.queue + (size_t)GS_QUEUE_STRIDE * GS_QUEUE_COUNTERS * call;
    t.grid = (unsigned)std::min(n_tiles, resident);
  }
  return t;
}

void kernel_event_start(int kernel, hipStream_t s) {
  if (g_events[kernel][0]) (void)hipEventRecord(g_events[kernel][0], s);
}

void kernel_event_stop(int kernel, hipStream_t s) {
  if (g_events[kernel][1]) (void)hipEventRecord(g_events[kernel][1], s);
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return GS_ERR_HIP;
}

namespace {

int invalid(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return GS_ERR_INVALID_ARGUMENT;
}

constexpr int32_t kMaxImageSide = 16384;

// Builds the per-view layout table from host cameras; returns a status.
int build_view_table(const gs_views* views, ViewTable& vt) {
  if (!views) return invalid("views is NULL");
  if (views->n_views < 1 || views->n_views > GS_MAX_VIEWS)
    return invalid("n_views = %d outside [1, %d]", views->n_views, GS_MAX_VIEWS);
  if (!views->cams_host) return invalid("views->cams_host is NULL");
  if (!views->cams_dev) return invalid("views->cams_dev is NULL");
  if (views->tile_size != kTile) {
    set_error("tile_size %d unsupported (16 only)", views->tile_size);
    return GS_ERR_UNSUPPORTED;
  }
  std::memset(&vt, 0, sizeof(vt));
  vt.n_views = views->n_views;
  int64_t tiles = 0, pixels = 0;
  for (int v = 0; v < views->n_views; ++v) {
    const gs_camera& c = views->cams_host[v];
    if (c.width < 1 || c.height < 1 || c.width > kMaxImageSide || c.height > kMaxImageSide)
      return invalid("view %d: image size %dx%d outside [1, %d]", v, c.width, c.height,
                     kMaxImageSide);
    if (!(std::isfinite(c.fx) && std::isfinite(c.fy) && c.fx > 0.f && c.fy > 0.f &&
          std::isfinite(c.cx) && std::isfinite(c.cy)))
      return invalid("view %d: intrinsics must be finite with fx, fy > 0", v);
    ViewInfo& vi = vt.v[v];
    vi.width = c.width;
    vi.height = c.height;
    vi.tiles_x = (c.width + kTile - 1) / kTile;
    vi.tiles_y = (c.height + kTile - 1) / kTile;
    vi.tile_base = (int32_t)tiles;
    vi.pix_base = pixels;
    tiles += (int64_t)vi.tiles_x * vi.tiles_y;
    pixels += (int64_t)c.width * c.height;
  }
  if (tiles > 0x7FFFFFFF) return invalid("too many tiles (%lld)", (long long)tiles);
  vt.n_tiles = (int32_t)tiles;
  vt.n_pixels = pixels;
  return GS_OK;
}

int check_gaussians(const gs_gaussians* g, int n_views) {
  if (!g) return invalid("gaussians is NULL");
  if (g->n < 0) return invalid("n = %lld < 0", (long long)g->n);
  if (g->sh_degree < 0 || g->sh_degree > GS_MAX_SH_DEGREE)
    return invalid("sh_degree = %d outside [0, %d]", g->sh_degree, GS_MAX_SH_DEGREE);
  if ((uint64_t)g->n * (uint64_t)n_views > 0xFFFFFFFFull)
    return invalid("n * n_views = %lld exceeds 2^32 - 1", (long long)g->n * n_views);
  if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
    return invalid("a Gaussian parameter pointer is NULL");
  return GS_OK;
}

int check_projected(const gs_projected* p, int64_t n) {
  if (!p) return invalid("projected is NULL");
  if (n > 0 && (!p->xy || !p->conic_opacity || !p->rgb_depth || !p->radius))
    return invalid("a projected-splat pointer is NULL");
  return GS_OK;
}

int check_bins(const gs_bins* b, bool need_keys) {
  if (!b) return invalid("bins is NULL");
  if (!b->ranges || !b->n_keys || !b->values || (need_keys && !b->keys))
    return invalid("a bins pointer is NULL");
  if (b->capacity < 0 || b->capacity > 0xFFFFFFFFll)
    return invalid("capacity = %lld outside [0, 2^32 - 1]", (long long)b->capacity);
  return GS_OK;
}

int check_workspace(const void* ws, size_t have, size_t need) {
  if (have < need) {
    set_error("workspace of %zu bytes is smaller than the %zu required", have, need);
    return GS_ERR_CAPACITY;
  }
  if (need > 0 && !ws) return invalid("workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) & 255) return invalid("workspace is not 256-byte aligned");
  return GS_OK;
}

float3 read_bg(const float* bg) {
  return bg ? make_float3(bg[0], bg[1], bg[2]) : make_float3(0.f, 0.f, 0.f);
}

}  // namespace
}  // namespace gsmi

using namespace gsmi;

extern "C" {

const char* gs_status_string(int status) {
  switch (status) {
    case GS_OK: return "GS_OK";
    case GS_ERR_INVALID_ARGUMENT: return "GS_ERR_INVALID_ARGUMENT";
    case GS_ERR_CAPACITY: return "GS_ERR_CAPACITY";
    case GS_ERR_HIP: return "GS_ERR_HIP";
    case GS_ERR_UNSUPPORTED: return "GS_ERR_UNSUPPORTED";
    default: return "GS_ERR_UNKNOWN";
  }
}

const char* gs_last_error(void) { return g_last_error; }

#ifndef GSMI_SOURCE_ID
#define GSMI_SOURCE_ID "unknown"
#endif
const char* gs_version(void) { return "gsmi 0.1 (gfx950) src " GSMI_SOURCE_ID; }

int gs_set_kernel_events(int kernel, void* start_event, void* stop_event) {
  if (kernel < 0 || kernel >= GS_KERNEL_COUNT) return invalid("unknown kernel id %d", kernel);
  if ((start_event == nullptr) != (stop_event == nullptr))
    return invalid("start and stop events must both be set or both be NULL");
  g_events[kernel][0] = static_cast<hipEvent_t>(start_event);
  g_events[kernel][1] = static_cast<hipEvent_t>(stop_event);
  return GS_OK;
}

int gs_set_tuning(int key, int value) {
  if (key < 0 || key >= GS_TUNE_COUNT) return invalid("unknown tuning key %d", key);
  if (key == GS_TUNE_FWD_SCHEDULE || key == GS_TUNE_BWD_SCHEDULE) {
    if (value == 0) value = GS_SCHEDULE_HEAVIEST_FIRST;
    if (value < GS_SCHEDULE_HEAVIEST_FIRST || value > GS_SCHEDULE_PERSISTENT_HALF)
      return invalid("unknown tile schedule %d", value);
  } else if (key == GS_TUNE_FWD_STAGE || key == GS_TUNE_BWD_STAGE) {
    if (value < 0 || value > 2)
      return invalid("splats staged per thread must be 1 or 2 (got %d)", value);
  } else {
    if (value == 0) value = 1;
    if (value != 1 && value != 2 && value != 4)
      return invalid("pixels per lane must be 1, 2 or 4 (got %d)", value);
  }
  g_tuning[key].store(value, std::memory_order_relaxed);
  return GS_OK;
}

int gs_get_tuning(int key) {
  if (key < 0 || key >= GS_TUNE_COUNT) return -1;
  return tuning(key);
}

int64_t gs_num_tiles(const gs_views* views) {
  ViewTable vt;
  if (build_view_table(views, vt) != GS_OK) return -1;
  return vt.n_tiles;
}

int64_t gs_num_pixels(const gs_views* views) {
  ViewTable vt;
  if (build_view_table(views, vt) != GS_OK) return -1;
  return vt.n_pixels;
}

int gs_preprocess(const gs_gaussians* g, const gs_views* views, gs_projected* out,
                  gs_stream_t stream) {
  ViewTable vt;
  int st = build_view_table(views, vt);
  if (st) return st;
  if ((st = check_gaussians(g, vt.n_views))) return st;
  if ((st = check_projected(out, g->n))) return st;
  const hipError_t e = launch_preprocess(*g, views->cams_dev, vt.n_views, *out, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_preprocess");
}

size_t gs_bin_sort_workspace_size(int64_t n, const gs_views* views, int64_t capacity) {
  ViewTable vt;
  if (n < 0 || capacity < 0 || build_view_table(views, vt) != GS_OK) return 0;
  return make_bin_sort_plan(n, vt, capacity).total;
}

int gs_bin_sort(const gs_projected* p, int64_t n, const gs_views* views, gs_bins* bins,
                uint32_t* n_keys_host, void* workspace, size_t workspace_bytes,
                gs_stream_t stream) {
  ViewTable vt;
  int st = build_view_table(views, vt);
  if (st) return st;
  if (n < 0) return invalid("n = %lld < 0", (long long)n);
  if ((uint64_t)n * (uint64_t)vt.n_views > 0xFFFFFFFFull)
    return invalid("n * n_views exceeds 2^32 - 1");
  if ((st = check_projected(p, n))) return st;
  if ((st = check_bins(bins, false))) return st;   // keys are optional
  const BinSortPlan plan = make_bin_sort_plan(n, vt, bins->capacity);
  if ((st = check_workspace(workspace, workspace_bytes, plan.total))) return st;
  return run_bin_sort(*p, n, vt, *bins, n_keys_host, static_cast<char*>(workspace), plan, stream);
}

int gs_render_fwd(const gs_projected* p, int64_t n, const gs_bins* bins, const gs_views* views,
                  const float* bg, float* image, float* final_T, uint32_t* n_contrib,
                  float* depth, gs_stream_t stream) {
  ViewTable vt;
  int st = build_view_table(views, vt);
  if (st) return st;
  if (n < 0) return invalid("n = %lld < 0", (long long)n);
  if ((st = check_projected(p, n))) return st;
  if ((st = check_bins(bins, false))) return st;
  if (!image || !final_T || !n_contrib) return invalid("an output pointer is NULL");
  const hipError_t e = launch_render_fwd(*p, *bins, vt, read_bg(bg), image, final_T, n_contrib,
                                         depth, nullptr, nullptr, nullptr, nullptr, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_render_fwd");
}

size_t gs_render_fwd_l1_workspace_size(const gs_views* views) {
  ViewTable vt;
  if (build_view_table(views, vt) != GS_OK) return 0;
  return std::max<size_t>(256, sizeof(float) * (size_t)vt.n_tiles);
}

int gs_render_fwd_l1(const gs_projected* p, int64_t n, const gs_bins* bins,
                     const gs_views* views, const float* bg, float* image, float* final_T,
                     uint32_t* n_contrib, const float* target, float* dL_dimage, double* loss,
                     void* workspace, size_t workspace_bytes, gs_stream_t stream) {
  ViewTable vt;
  int st = build_view_table(views, vt);
  if (st) return st;
  if (n < 0) return invalid("n = %lld < 0", (long long)n);
  if ((st = check_projected(p, n))) return st;
  if ((st = check_bins(bins, false))) return st;
  if (!image || !final_T || !n_contrib) return invalid("an output pointer is NULL");
  if (!target || !dL_dimage) return invalid("target or dL_dimage is NULL");
  const size_t need = std::max<size_t>(256, sizeof(float) * (size_t)vt.n_tiles);
  if ((st = check_workspace(workspace, workspace_bytes, need))) return st;
  const hipError_t e =
      launch_render_fwd(*p, *bins, vt, read_bg(bg), image, final_T, n_contrib, nullptr, target,
                        dL_dimage, loss, static_cast<float*>(workspace), stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_render_fwd_l1");
}

int gs_render_fwd_l1_noalloc(const gs_projected* p, int64_t n, const gs_bins* bins,
                             const gs_views* views, const float* bg, float* image,
                             float* final_T, uint32_t* n_contrib, const float* target,
                             float* dL_dimage, double* loss, gs_stream_t stream) {
  ViewTable vt;
  int st = build_view_table(views, vt);
  if (st) return st;
  if (n < 0) return invalid("n = %lld < 0", (long long)n);
  if ((st = check_projected(p, n))) return st;
  if ((st = check_bins(bins, false))) return st;
  if (!image || !final_T || !n_contrib) return invalid("an output pointer is NULL");
  if (!target || !dL_dimage) return invalid("target or dL_dimage is NULL");
  if (vt.n_tiles > GS_NOALLOC_MAX_TILES) {
    set_error("%d tiles exceed the %d tile shares of the static scratch", vt.n_tiles,
              GS_NOALLOC_MAX_TILES);
    return GS_ERR_CAPACITY;
  }
  float* scratch = nullptr;
  hipError_t e = noalloc_scratch(&scratch);
  if (e != hipSuccess) return hip_fail(e, "gs_render_fwd_l1_noalloc: scratch address");
  e = launch_render_fwd(*p, *bins, vt, read_bg(bg), image, final_T, n_contrib, nullptr, target,
                        dL_dimage, loss, scratch, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_render_fwd_l1_noalloc");
}

size_t gs_render_bwd_workspace_size(int64_t n, const gs_views* views) {
  ViewTable vt;
  if (n < 0 || build_view_table(views, vt) != GS_OK) return 0;
  return make_bwd_plan(n, vt).total;
}

int gs_render_bwd(const gs_gaussians* g, const gs_projected* p, const gs_bins* bins,
                  const gs_views* views, const float* bg, const float* dL_dimage,
                  const float* final_T, const uint32_t* n_contrib, gs_grads* grads,
                  uint32_t flags, void* workspace, size_t workspace_bytes, gs_stream_t stream) {
  ViewTable vt;
  int st = build_view_table(views, vt);
  if (st) return st;
  if ((st = check_gaussians(g, vt.n_views))) return st;
  if ((st = check_projected(p, g->n))) return st;
  if ((st = check_bins(bins, false))) return st;
  if (flags & ~(uint32_t)(GS_BWD_NO_POSE | GS_BWD_POSE_ONLY | GS_BWD_OVERWRITE |
                          GS_BWD_KEEP_CLEAR))
    return invalid("unknown flags");
  if ((flags & GS_BWD_NO_POSE) && (flags & GS_BWD_POSE_ONLY))
    return invalid("GS_BWD_NO_POSE and GS_BWD_POSE_ONLY are exclusive");
  if (!dL_dimage || !final_T || !n_contrib || !grads) return invalid("an input pointer is NULL");
  if (!(flags & GS_BWD_POSE_ONLY) && g->n > 0 &&
      (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits ||
       !grads->sh))
    return invalid("a map-gradient pointer is NULL");
  if (!(flags & GS_BWD_NO_POSE) && !grads->xi) return invalid("grads->xi is NULL");
  const BwdPlan plan = make_bwd_plan(g->n, vt);
  if ((st = check_workspace(workspace, workspace_bytes, plan.total))) return st;
  const hipError_t e =
      launch_render_bwd(*g, *p, *bins, views->cams_dev, vt, read_bg(bg), dL_dimage, final_T,
                        n_contrib, *grads, flags, static_cast<char*>(workspace), plan, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_render_bwd");
}

int gs_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
                 float beta2, float eps, int32_t step, const uint8_t* mask, gs_stream_t stream) {
  if (n < 0) return invalid("n = %lld < 0", (long long)n);
  if (n > 0 && (!p || !g || !m || !v)) return invalid("a parameter pointer is NULL");
  if (step < 1) return invalid("step = %d < 1", step);
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f))
    return invalid("betas must lie in [0, 1)");
  if (!(eps >= 0.f) || !std::isfinite(lr)) return invalid("eps must be >= 0 and lr finite");
  const hipError_t e = launch_adam(p, g, m, v, n, lr, beta1, beta2, eps, step, mask, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_adam_step");
}

int gs_adam_step_dev(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                     float beta1, float beta2, float eps, int32_t* step_dev, int32_t commit,
                     const uint8_t* mask, const uint32_t* guard_n_keys, int64_t guard_capacity,
                     gs_stream_t stream) {
  if (n < 0) return invalid("n = %lld < 0", (long long)n);
  if (n > 0 && (!p || !g || !m || !v)) return invalid("a parameter pointer is NULL");
  if (!step_dev) return invalid("step_dev is NULL");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f))
    return invalid("betas must lie in [0, 1)");
  if (!(eps >= 0.f) || !std::isfinite(lr)) return invalid("eps must be >= 0 and lr finite");
  if (guard_n_keys && guard_capacity < 0) return invalid("guard_capacity < 0");
  const hipError_t e = launch_adam_dev(p, g, m, v, n, lr, beta1, beta2, eps, step_dev, commit,
                                       mask, guard_n_keys, guard_capacity, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_adam_step_dev");
}

int gs_adam_step_groups_dev(const gs_adam_group* groups, int32_t n_groups, float beta1,
                            float beta2, float eps, int32_t* step_dev,
                            const uint32_t* guard_n_keys, int64_t guard_capacity,
                            gs_stream_t stream) {
  if (!groups) return invalid("groups is NULL");
  if (n_groups < 1 || n_groups > GS_ADAM_MAX_GROUPS)
    return invalid("n_groups = %d outside 1..%d", n_groups, GS_ADAM_MAX_GROUPS);
  for (int k = 0; k < n_groups; ++k) {
    const gs_adam_group& q = groups[k];
    if (q.n < 0) return invalid("group %d: n = %lld < 0", k, (long long)q.n);
    if (q.n > 0 && (!q.p || !q.g || !q.m || !q.v)) return invalid("group %d: a pointer is NULL", k);
    if (!std::isfinite(q.lr)) return invalid("group %d: lr is not finite", k);
  }
  if (!step_dev) return invalid("step_dev is NULL");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f))
    return invalid("betas must lie in [0, 1)");
  if (!(eps >= 0.f)) return invalid("eps must be >= 0");
  if (guard_n_keys && guard_capacity < 0) return invalid("guard_capacity < 0");
  const hipError_t e = launch_adam_groups(groups, n_groups, beta1, beta2, eps, step_dev,
                                          guard_n_keys, guard_capacity, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_adam_step_groups_dev");
}

int gs_render_error(const gs_projected* p, int64_t n, const gs_bins* bins, const gs_views* views,
                    const float* image, const float* target, const uint32_t* n_contrib,
                    float* err, gs_stream_t stream) {
  ViewTable vt;
  int st = build_view_table(views, vt);
  if (st) return st;
  if (n < 0) return invalid("n = %lld < 0", (long long)n);
  if ((uint64_t)n * (uint64_t)vt.n_views > 0xFFFFFFFFull)
    return invalid("n * n_views exceeds 2^32 - 1");
  if ((st = check_projected(p, n))) return st;
  if ((st = check_bins(bins, false))) return st;
  if (!image || !target || !n_contrib) return invalid("an input image pointer is NULL");
  if (n > 0 && !err) return invalid("err is NULL");
  const hipError_t e = launch_render_error(*p, n, *bins, vt, image, target, n_contrib, err, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_render_error");
}

int gs_active_set(const float* err, int64_t n, int32_t n_views, float eps, const uint8_t* always,
                  uint8_t* mask, float* err_max, uint32_t* n_active, gs_stream_t stream) {
  if (n < 0) return invalid("n = %lld < 0", (long long)n);
  if (n_views < 1 || n_views > GS_MAX_VIEWS)
    return invalid("n_views = %d outside [1, %d]", n_views, GS_MAX_VIEWS);
  if (!std::isfinite(eps)) return invalid("eps must be finite");
  if (n > 0 && (!err || !mask)) return invalid("err or mask is NULL");
  const hipError_t e =
      launch_active_set(err, n, n_views, eps, always, mask, err_max, n_active, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_active_set");
}

int gs_adam_step_groups_masked_dev(const gs_adam_group* groups, int32_t n_groups, float beta1,
                                   float beta2, float eps, int32_t* step_dev,
                                   const uint8_t* gauss_mask, int64_t n_gauss,
                                   const uint32_t* guard_n_keys, int64_t guard_capacity,
                                   gs_stream_t stream) {
  if (!groups) return invalid("groups is NULL");
  if (n_groups < 1 || n_groups > GS_ADAM_MAX_GROUPS)
    return invalid("n_groups = %d outside 1..%d", n_groups, GS_ADAM_MAX_GROUPS);
  if (n_gauss < 1) return invalid("n_gauss = %lld < 1", (long long)n_gauss);
  if (!gauss_mask) return invalid("gauss_mask is NULL");
  for (int k = 0; k < n_groups; ++k) {
    const gs_adam_group& q = groups[k];
    if (q.n < 0 || q.n % n_gauss)
      return invalid("group %d: n = %lld is not a multiple of n_gauss", k, (long long)q.n);
    if (q.n > 0 && (!q.p || !q.g || !q.m || !q.v)) return invalid("group %d: a pointer is NULL", k);
    if (!std::isfinite(q.lr)) return invalid("group %d: lr is not finite", k);
  }
  if (!step_dev) return invalid("step_dev is NULL");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f))
    return invalid("betas must lie in [0, 1)");
  if (!(eps >= 0.f)) return invalid("eps must be >= 0");
  if (guard_n_keys && guard_capacity < 0) return invalid("guard_capacity < 0");
  const hipError_t e = launch_adam_groups(groups, n_groups, beta1, beta2, eps, step_dev,
                                          guard_n_keys, guard_capacity, stream, gauss_mask,
                                          n_gauss);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_adam_step_groups_masked_dev");
}

int gs_concat(const gs_concat_array* arrays, int32_t n_arrays, int64_t n_a, int64_t n_b,
              gs_stream_t stream) {
  if (!arrays) return invalid("arrays is NULL");
  if (n_arrays < 1 || n_arrays > GS_SOA_MAX_ARRAYS)
    return invalid("n_arrays = %d outside 1..%d", n_arrays, GS_SOA_MAX_ARRAYS);
  if (n_a < 0 || n_b < 0) return invalid("n_a and n_b must be >= 0");
  for (int k = 0; k < n_arrays; ++k) {
    const gs_concat_array& q = arrays[k];
    if (q.components < 1) return invalid("array %d: components < 1", k);
    if (n_a + n_b > 0 && !q.dst) return invalid("array %d: dst is NULL", k);
    if (n_a > 0 && !q.a) return invalid("array %d: a is NULL", k);
  }
  const hipError_t e = launch_concat(arrays, n_arrays, n_a, n_b, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_concat");
}

int gs_prune_mask(const float* opacity_logits, int64_t n, float min_opacity, uint8_t* keep,
                  gs_stream_t stream) {
  if (n < 0) return invalid("n = %lld < 0", (long long)n);
  if (!(min_opacity > 0.f && min_opacity < 1.f)) return invalid("min_opacity must lie in (0, 1)");
  if (n > 0 && (!opacity_logits || !keep)) return invalid("a pointer is NULL");
  const double p = (double)min_opacity;
  const float thr = (float)std::log(p / (1.0 - p));
  const hipError_t e = launch_prune_mask(opacity_logits, n, thr, keep, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_prune_mask");
}

size_t gs_compact_workspace_size(int64_t n) { return n < 0 ? 0 : compact_ws_bytes(n); }

int gs_compact(const gs_compact_array* arrays, int32_t n_arrays, int64_t n, const uint8_t* keep,
               uint32_t* n_kept, void* workspace, size_t workspace_bytes, gs_stream_t stream) {
  if (!arrays) return invalid("arrays is NULL");
  if (n_arrays < 1 || n_arrays > GS_SOA_MAX_ARRAYS)
    return invalid("n_arrays = %d outside 1..%d", n_arrays, GS_SOA_MAX_ARRAYS);
  if (n < 0 || n > 0xFFFFFFFFll) return invalid("n = %lld outside [0, 2^32 - 1]", (long long)n);
  if (!n_kept) return invalid("n_kept is NULL");
  if (n > 0 && !keep) return invalid("keep is NULL");
  for (int k = 0; k < n_arrays; ++k) {
    const gs_compact_array& q = arrays[k];
    if (q.components < 1) return invalid("array %d: components < 1", k);
    if (n > 0 && (!q.src || !q.dst)) return invalid("array %d: a pointer is NULL", k);
  }
  int st;
  if ((st = check_workspace(workspace, workspace_bytes, compact_ws_bytes(n)))) return st;
  const hipError_t e = launch_compact(arrays, n_arrays, n, keep, n_kept, workspace, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_compact");
}

int gs_pose_adam_step(gs_camera* cams_dev, const float* grad_xi, float* m, float* v,
                      int32_t n_views, const uint8_t* view_mask, float lr_trans, float lr_rot,
                      float beta1, float beta2, float eps, int32_t* step_dev, gs_stream_t stream) {
  if (n_views < 1 || n_views > GS_MAX_VIEWS)
    return invalid("n_views = %d outside [1, %d]", n_views, GS_MAX_VIEWS);
  if (!cams_dev || !grad_xi || !m || !v || !step_dev) return invalid("a pointer is NULL");
  if (!(std::isfinite(lr_trans) && std::isfinite(lr_rot))) return invalid("learning rates must be finite");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f))
    return invalid("betas must lie in [0, 1)");
  if (!(eps >= 0.f)) return invalid("eps must be >= 0");
  const hipError_t e = launch_pose_adam(cams_dev, grad_xi, m, v, n_views, view_mask, lr_trans,
                                        lr_rot, beta1, beta2, eps, step_dev, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_pose_adam_step");
}

int gs_iso_loss_grad(const float* log_scales, int64_t n, float weight, float* grad_log_scales,
                     double* loss, gs_stream_t stream) {
  if (n < 0) return invalid("n = %lld < 0", (long long)n);
  if (!std::isfinite(weight)) return invalid("weight must be finite");
  if (n > 0 && (!log_scales || !grad_log_scales)) return invalid("a pointer is NULL");
  const hipError_t e = launch_iso_loss_grad(log_scales, n, weight, grad_log_scales, loss, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_iso_loss_grad");
}

int gs_l1_loss_grad(const float* image, const float* target, const gs_views* views,
                    float* dL_dimage, double* loss, gs_stream_t stream) {
  ViewTable vt;
  int st = build_view_table(views, vt);
  if (st) return st;
  if (!image || !target || !dL_dimage) return invalid("an image pointer is NULL");
  const hipError_t e = launch_l1_loss_grad(image, target, vt, dL_dimage, loss, stream);
  return e == hipSuccess ? GS_OK : hip_fail(e, "gs_l1_loss_grad");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned and plain initialiser
// ---------------------------------------------------------------------------

namespace gsmi {
namespace {

int check_act(const gs_act* a, const char* name, bool conv_input) {
  if (!a) return invalid("%s is NULL", name);
  if (!a->data) return invalid("%s->data is NULL", name);
  if (a->n < 1 || a->h < 1 || a->w < 1 || a->c < 1)
    return invalid("%s: shape (%d, %d, %d, %d) must be positive", name, a->n, a->h, a->w, a->c);
  if (a->offset < 0 || a->stride < a->offset + a->c)
    return invalid("%s: stride %d too small for offset %d + %d channels", name, a->stride,
                   a->offset, a->c);
  if ((int64_t)a->n * a->h * a->w > 0x7FFFFFFFLL) return invalid("%s: too many pixels", name);
  if (conv_input) {
    if ((a->c % 8) || (a->stride % 8) || (a->offset % 8))
      return invalid("%s: channels, stride and offset must be multiples of 8", name);
    if (reinterpret_cast<uintptr_t>(a->data) & 15) return invalid("%s: data not 16-byte aligned", name);
  }
  return GS_OK;
}

bool same_grid(const gs_act* a, const gs_act* b) {
  return a->n == b->n && a->h == b->h && a->w == b->w;
}

int nn_status(hipError_t e, const char* what) { return e == hipSuccess ? GS_OK : hip_fail(e, what); }

}  // namespace
}  // namespace gsmi

extern "C" {

int gs_nn_conv3x3(const gs_act* x1, const gs_act* x2, const gs_act* mask, const void* weights,
                  int32_t cout, const float* bias, int32_t relu, gs_act* y, float* y_f32,
                  int32_t y_f32_stride, gs_stream_t stream) {
  int st;
  if ((st = check_act(x1, "x1", true))) return st;
  if (x2 && (st = check_act(x2, "x2", true))) return st;
  if (x2 && !same_grid(x1, x2)) return invalid("x1 and x2 differ in n, h or w");
  const int cin = x1->c + (x2 ? x2->c : 0);
  if (mask) {
    if ((st = check_act(mask, "mask", true))) return st;
    if (!same_grid(x1, mask) || mask->c != cin) return invalid("mask must match the input layout");
  }
  if (!weights) return invalid("weights is NULL");
  if (reinterpret_cast<uintptr_t>(weights) & 15) return invalid("weights not 16-byte aligned");
  if (cout < 1) return invalid("cout = %d < 1", cout);
  if (!y && !y_f32) return invalid("no output");
  if (y) {
    if ((st = check_act(y, "y", false))) return st;
    if (!same_grid(x1, y) || y->c != cout) return invalid("y must be (n, h, w, cout) like x1");
  }
  if (y_f32 && y_f32_stride < cout) return invalid("y_f32_stride < cout");
  return nn_status(nn_conv3x3(x1, x2, mask, weights, cout, bias, relu, y, y_f32, y_f32_stride,
                              stream), "gs_nn_conv3x3");
}

int gs_nn_conv3x3_wgrad(const gs_act* x1, const gs_act* x2, const gs_act* dy, const gs_act* mask,
                        float* dw, float* dbias, gs_stream_t stream) {
  int st;
  if ((st = check_act(x1, "x1", false))) return st;
  if (x2 && (st = check_act(x2, "x2", false))) return st;
  if ((st = check_act(dy, "dy", false))) return st;
  if (x2 && !same_grid(x1, x2)) return invalid("x1 and x2 differ in n, h or w");
  if (!same_grid(x1, dy)) return invalid("dy must share x1's n, h, w");
  if (mask) {
    if ((st = check_act(mask, "mask", false))) return st;
    if (!same_grid(x1, mask) || mask->c != dy->c) return invalid("mask must match dy's layout");
  }
  if (!dw) return invalid("dw is NULL");
  return nn_status(nn_conv3x3_wgrad(x1, x2, dy, mask, dw, dbias, stream), "gs_nn_conv3x3_wgrad");
}

int gs_nn_flip_weights(const void* weights, int32_t cout, int32_t cin, void* weights_t,
                       gs_stream_t stream) {
  if (!weights || !weights_t) return invalid("a weight pointer is NULL");
  if (cout < 1 || cin < 1) return invalid("cout and cin must be positive");
  return nn_status(nn_flip_weights(weights, cout, cin, weights_t, stream), "gs_nn_flip_weights");
}

int gs_nn_avgpool2(const gs_act* x, gs_act* y, gs_stream_t stream) {
  int st;
  if ((st = check_act(x, "x", false))) return st;
  if ((st = check_act(y, "y", false))) return st;
  if ((x->h % 2) || (x->w % 2)) return invalid("pooling needs even h and w");
  if (y->n != x->n || y->h != x->h / 2 || y->w != x->w / 2 || y->c != x->c || y->offset != 0)
    return invalid("y must be (n, h/2, w/2, c) with offset 0");
  return nn_status(nn_avgpool2(x, y, stream), "gs_nn_avgpool2");
}

int gs_nn_avgpool2_bwd(const gs_act* dy, const gs_act* add, gs_act* dx, int32_t accumulate,
                       gs_stream_t stream) {
  int st;
  if ((st = check_act(dy, "dy", false))) return st;
  if ((st = check_act(dx, "dx", false))) return st;
  if (dx->h % 2 || dx->w % 2 || dy->n != dx->n || dy->h != dx->h / 2 || dy->w != dx->w / 2 ||
      dy->c != dx->c)
    return invalid("dx must be (n, 2h, 2w, c) of dy");
  if (add) {
    if ((st = check_act(add, "add", false))) return st;
    if (!same_grid(add, dx) || add->c != dx->c) return invalid("add must match dx");
  }
  return nn_status(nn_avgpool2_bwd(dy, add, dx, accumulate, stream), "gs_nn_avgpool2_bwd");
}

int gs_nn_upsample2(const gs_act* x, gs_act* y, gs_stream_t stream) {
  int st;
  if ((st = check_act(x, "x", false))) return st;
  if ((st = check_act(y, "y", false))) return st;
  if (y->n != x->n || y->h != 2 * x->h || y->w != 2 * x->w || y->c != x->c)
    return invalid("y must be (n, 2h, 2w, c)");
  return nn_status(nn_upsample2(x, y, stream), "gs_nn_upsample2");
}

int gs_nn_upsample2_bwd(const gs_act* dy, gs_act* dx, gs_stream_t stream) {
  int st;
  if ((st = check_act(dy, "dy", false))) return st;
  if ((st = check_act(dx, "dx", false))) return st;
  if (dy->n != dx->n || dy->h != 2 * dx->h || dy->w != 2 * dx->w || dy->c != dx->c ||
      dx->offset != 0)
    return invalid("dx must be (n, h/2, w/2, c) with offset 0");
  return nn_status(nn_upsample2_bwd(dy, dx, stream), "gs_nn_upsample2_bwd");
}

int gs_nn_rgb_to_nhwc(const float* rgb, gs_act* x, gs_stream_t stream) {
  int st;
  if (!rgb) return invalid("rgb is NULL");
  if ((st = check_act(x, "x", false))) return st;
  if (x->offset != 0 || x->stride < 3) return invalid("x must have offset 0 and stride >= 3");
  return nn_status(nn_rgb_to_nhwc(rgb, x, stream), "gs_nn_rgb_to_nhwc");
}

int gs_nn_f32_to_bf16(const float* src, void* dst, int64_t n, gs_stream_t stream) {
  if (n < 0) return invalid("n < 0");
  if (n > 0 && (!src || !dst)) return invalid("a pointer is NULL");
  return nn_status(nn_f32_to_bf16(src, dst, n, stream), "gs_nn_f32_to_bf16");
}

int gs_nn_head(const gs_act* f, const float* w, const float* b, float* out, gs_stream_t stream) {
  int st;
  if ((st = check_act(f, "f", false))) return st;
  if (!w || !b || !out) return invalid("a head pointer is NULL");
  return nn_status(nn_head(f, w, b, out, stream), "gs_nn_head");
}

int gs_nn_head_bwd(const gs_act* f, const float* w, const float* dout, gs_act* df, float* dw,
                   float* db, gs_stream_t stream) {
  int st;
  if ((st = check_act(f, "f", false))) return st;
  if ((st = check_act(df, "df", false))) return st;
  if (!same_grid(f, df) || df->c != f->c) return invalid("df must match f");
  if (f->c > 64) return invalid("head supports at most 64 feature channels");
  if (!w || !dout || !dw || !db) return invalid("a head pointer is NULL");
  return nn_status(nn_head_bwd(f, w, dout, df, dw, db, stream), "gs_nn_head_bwd");
}

int gs_nn_depth_loss(const float* pred, const float* depth, int32_t n, int32_t h, int32_t w,
                     float fx, float* dpred, double* loss, void* ws, gs_stream_t stream) {
  if (!pred || !depth || !dpred || !ws) return invalid("a loss pointer is NULL");
  if (n < 1 || h < 1 || w < 1) return invalid("shape must be positive");
  if (!(fx > 0.f)) return invalid("fx must be > 0");
  return nn_status(nn_depth_loss(pred, depth, n, h, w, fx, dpred, loss, static_cast<int*>(ws),
                                 stream), "gs_nn_depth_loss");
}

size_t gs_bp_workspace_size(int32_t h, int32_t w) {
  if (h < 1 || w < 1) return 0;
  return bp_ws_bytes(h, w);
}

int gs_bp_labels(const float* cost, int32_t h, int32_t w, float lam, float trunc, int32_t iters,
                 float invalid_cost, int32_t* labels, float* depth, void* ws, size_t ws_bytes,
                 gs_stream_t stream) {
  if (!cost) return invalid("cost is NULL");
  if (h < 1 || w < 1) return invalid("h and w must be positive");
  if ((int64_t)h * w > (1ll << 26)) return invalid("too many pixels");
  if (!(std::isfinite(lam) && lam >= 0.f && std::isfinite(trunc) && trunc >= 0.f))
    return invalid("lam and trunc must be finite and >= 0");
  if (!std::isfinite(invalid_cost)) return invalid("invalid_cost must be finite");
  if (iters < 0) return invalid("iters < 0");
  const size_t need = bp_ws_bytes(h, w);
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    return GS_ERR_CAPACITY;
  }
  if (!ws) return invalid("workspace is NULL");
  return nn_status(launch_bp(cost, h, w, lam, trunc, iters, invalid_cost, labels, depth, ws, stream),
                   "gs_bp_labels");
}

size_t gs_cost_volume_workspace_size(int32_t k, int32_t h, int32_t w) {
  if (k < 2 || h < 4 || w < 4) return 0;
  return cost_volume_ws_bytes(k, h, w);
}

int gs_cost_volume_wta(const float* keyframes, const gs_views* cams, float* cost, float* depth,
                       void* ws, size_t ws_bytes, gs_stream_t stream) {
  if (!keyframes || !depth) return invalid("keyframes or depth is NULL");
  if (!cams || !cams->cams_host || !cams->cams_dev) return invalid("cameras are NULL");
  const int K = cams->n_views;
  if (K < 2 || K > GS_MAX_VIEWS) return invalid("need 2..%d keyframes", GS_MAX_VIEWS);
  const int W = cams->cams_host[0].width, H = cams->cams_host[0].height;
  for (int k = 0; k < K; ++k) {
    const gs_camera& c = cams->cams_host[k];
    if (c.width != W || c.height != H) return invalid("keyframes must share one image size");
    if (!(c.fx > 0.f && c.fy > 0.f)) return invalid("fx, fy must be > 0");
  }
  if (W % 4 || H % 4 || W < 4 || H < 4) return invalid("image size must be a multiple of 4");
  const size_t need = cost_volume_ws_bytes(K, H, W);
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    return GS_ERR_CAPACITY;
  }
  if (!ws) return invalid("workspace is NULL");
  return nn_status(launch_cost_volume(keyframes, K, H, W, cams->cams_dev, cost, depth, ws, stream),
                   "gs_cost_volume_wta");
}

}  // extern "C"
