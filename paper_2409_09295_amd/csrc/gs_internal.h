// Internal definitions shared by the libgsmi kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <utility>

#include "gs.h"
#include "gs_nn.h"

namespace gsmi {

// Renderer constants (see gs.h for the definition they belong to).
constexpr float kZNear = 0.2f;          // near-plane cull on camera-frame z
constexpr float kDilation = 0.3f;       // screen-space covariance dilation, px^2
constexpr float kAlphaMax = 0.99f;      // opacity clamp
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;          // early-termination transmittance
constexpr float kGuard = 1.3f;          // frustum guard on x/z, y/z inside J
constexpr float kLog2e = 1.4426950408889634f;

constexpr int kTile = 16;               // tile edge in pixels
constexpr int kBlock = 256;             // threads per tile block (one per pixel)

// Per-view layout derived on the host from gs_views::cams_host and passed to
// kernels by value (it lands in the kernel-argument segment, read with scalar
// loads, and is captured by value in a hipGraph).
struct ViewInfo {
  int32_t tile_base;   // first global tile id of the view
  int32_t tiles_x;
  int32_t tiles_y;
  int32_t width;
  int32_t height;
  int32_t pad;
  int64_t pix_base;    // first pixel of the view in packed [H][W] buffers
};

struct ViewTable {
  int32_t n_views;
  int32_t n_tiles;     // total over views
  int64_t n_pixels;    // total over views
  ViewInfo v[GS_MAX_VIEWS];
};

// Global tile id -> view (tiles of view v occupy [tile_base, tile_base + tiles_x*tiles_y)).
__device__ __forceinline__ int find_view(const ViewTable& vt, int tile) {
  int v = 0;
  for (int i = 1; i < vt.n_views; ++i) v = (tile >= vt.v[i].tile_base) ? i : v;
  return v;
}

// Half-open tile rectangle of a splat: tiles that hold a pixel centre
// i + 1/2 with |i + 1/2 - u| <= r (and likewise in y), clamped to the image.
// Evaluated in float64 from the float32 centre so that the integer result is
// exact for the stored inputs.  Returns false (and an empty rect) when no
// pixel centre is covered.
struct Rect {
  int32_t x0, x1, y0, y1;
};

__device__ __forceinline__ bool tile_rect(float uf, float vf, int32_t r, int32_t W, int32_t H,
                                          Rect& out) {
  out.x0 = out.x1 = out.y0 = out.y1 = 0;
  if (r <= 0) return false;
  const double u = (double)uf, v = (double)vf, rd = (double)r;
  if (!(isfinite(u) && isfinite(v))) return false;
  const double ilo = ceil(u - rd - 0.5), ihi = floor(u + rd - 0.5);
  const double jlo = ceil(v - rd - 0.5), jhi = floor(v + rd - 0.5);
  if (!(ilo <= ihi && jlo <= jhi && ihi >= 0.0 && ilo <= (double)(W - 1) && jhi >= 0.0 &&
        jlo <= (double)(H - 1)))
    return false;
  const int32_t i0 = (int32_t)fmax(ilo, 0.0), i1 = (int32_t)fmin(ihi, (double)(W - 1));
  const int32_t j0 = (int32_t)fmax(jlo, 0.0), j1 = (int32_t)fmin(jhi, (double)(H - 1));
  out.x0 = i0 / kTile;
  out.x1 = i1 / kTile + 1;
  out.y0 = j0 / kTile;
  out.y1 = j1 / kTile + 1;
  return true;
}

// Splat record staged in LDS by the compositing kernels.  The conic is
// pre-scaled so that log2 of the Gaussian falloff is
//   p2 = a dx^2 + b dx dy + c dy^2,
// a = -log2(e)/2 Q00, b = -log2(e) Q01, c = -log2(e)/2 Q11, i.e. p2 = log2(e) * power.
// The fields every walk step reads come first, so one LDS base address
// serves all reads of a record.
struct StagedSplat {
  float4 geo;   // u, v, a, b
  float4 app;   // c, opacity, red, green
  float4 ext;   // blue, quadrant mask bits, depth, accumulator index bits
};

// Minimum over the box [x0, x1] x [y0, y1] of f(x, y) = a x^2 + 2 b x y + c y^2
// (a, c > 0, ac > b^2): 0 if the box holds the origin, otherwise attained on
// an edge, where f is a convex parabola minimised at the clamped vertex.
__device__ __forceinline__ float quad_box_min(float a, float b, float c, float x0, float x1,
                                              float y0, float y1) {
  if (x0 <= 0.f && x1 >= 0.f && y0 <= 0.f && y1 >= 0.f) return 0.f;
  // approximate reciprocals only move the clamped vertex by a relative
  // 1e-7, which raises f there by a negligible second-order amount
  const float ia = __builtin_amdgcn_rcpf(a), ic = __builtin_amdgcn_rcpf(c);
  float best = INFINITY;
  const float ys[2] = {y0, y1}, xs[2] = {x0, x1};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float y = ys[k];
    const float x = fminf(fmaxf(-b * y * ia, x0), x1);
    best = fminf(best, a * x * x + 2.0f * b * x * y + c * y * y);
    const float xe = xs[k];
    const float ye = fminf(fmaxf(-b * xe * ic, y0), y1);
    best = fminf(best, a * xe * xe + 2.0f * b * xe * ye + c * ye * ye);
  }
  return best;
}

// Which 8x8 quadrants of the tile whose top-left pixel is (tx0, ty0) a splat
// can reach: bit q (quadrant x offset 8 (q & 1), y offset 8 (q >> 1)) is
// clear only if at every pixel centre of the quadrant the splat's alpha is
// below 1/255 with a margin that covers the float32 rounding of the
// per-pixel evaluation, so a pixel of a clear quadrant would skip the splat
// anyway and skipping it for the whole quadrant changes no result.
// alpha >= 1/255 needs o e^(-m/2) >= 1/255 with m = d^T Q d, i.e.
// m <= 2 ln(255 o); the box minimum of m decides.
__device__ __forceinline__ uint32_t quadrant_mask(float u, float v, float q00, float q01,
                                                  float q11, float o, int tx0, int ty0, int W,
                                                  int H) {
  if (!(o * 255.0f >= 1.0f - 1e-4f)) return 0u;
  const float lvl = 2.0f * __logf(fmaxf(o * 255.0f, 1.0f));
  uint32_t mask = 0u;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int px0 = tx0 + 8 * (q & 1), py0 = ty0 + 8 * (q >> 1);
    if (px0 >= W || py0 >= H) continue;
    const float x0 = (float)px0 + 0.5f - u, x1 = (float)min(px0 + 7, W - 1) + 0.5f - u;
    const float y0 = (float)py0 + 0.5f - v, y1 = (float)min(py0 + 7, H - 1) + 0.5f - v;
    const float m = quad_box_min(q00, q01, q11, x0, x1, y0, y1);
    const float dx = fmaxf(fabsf(x0), fabsf(x1)), dy = fmaxf(fabsf(y0), fabsf(y1));
    const float terms = q00 * dx * dx + 2.0f * fabsf(q01) * dx * dy + q11 * dy * dy;
    const float margin = 1e-4f * lvl + 1e-5f * terms + 1e-5f;
    if (!(m > lvl + margin)) mask |= 1u << q;
  }
  return mask;
}

// Wave-uniform 64-bit value (a mask read by every lane from the same LDS word).
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// x of another lane by DPP (0 where the source lane is out of its row).
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ float dpp_or_zero(float x) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, BANK_MASK, false));
}

// Sum over the 64 lanes of a wavefront; the total lands in lane 63.
__device__ __forceinline__ float wave_sum_to_lane63(float x) {
  x += dpp_or_zero<0xb1, 0xf, 0xf>(x);   // quad_perm [1,0,3,2]
  x += dpp_or_zero<0x4e, 0xf, 0xf>(x);   // quad_perm [2,3,0,1]
  x += dpp_or_zero<0x124, 0xf, 0xf>(x);  // row_ror:4
  x += dpp_or_zero<0x128, 0xf, 0xf>(x);  // row_ror:8 -> every lane holds its row sum
  x += dpp_or_zero<0x142, 0xa, 0xf>(x);  // row_bcast:15 into rows 1 and 3
  x += dpp_or_zero<0x143, 0xc, 0xf>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// Stages splat g (index view * n + Gaussian into the [V][n] splat arrays,
// also the index of its accumulator in the [V][n][9] gradient buffer) as
// the tile kernels' LDS record and returns the quadrants of the tile whose
// top-left pixel is (tx0, ty0) it can reach.
__device__ __forceinline__ uint32_t stage_splat(uint32_t g, const float2* __restrict__ xy,
                                                const float4* __restrict__ co,
                                                const float4* __restrict__ rd, int tx0, int ty0,
                                                int W, int H, StagedSplat& out) {
  const float2 m = xy[g];
  const float4 c = co[g];
  const float4 r = rd[g];
  const uint32_t reach = quadrant_mask(m.x, m.y, c.x, c.y, c.z, c.w, tx0, ty0, W, H);
  out.geo = make_float4(m.x, m.y, -0.5f * kLog2e * c.x, -kLog2e * c.y);
  out.app = make_float4(-0.5f * kLog2e * c.z, c.w, r.x, r.y);
  out.ext = make_float4(r.z, __uint_as_float(reach), r.w, __uint_as_float(g));
  return reach;
}

// Blending decision shared bit-for-bit by the forward and backward kernels.
// The exponent (log2 units) at pixel (px, py) is
//   power = a dx^2 + dy (c dy + b dx),   dx = px - u, dy = py - v,
// with (u, v, a, b) = geo and c = app.x.  The terms that depend only on dx
// are shared by every pixel of one column (a lane's pixels often share their
// x), so they are computed once per splat and column.
struct ColumnTerms {
  float dx, adx2, bdx;
};

__device__ __forceinline__ ColumnTerms column_terms(const float4& geo, float px) {
  ColumnTerms t;
  t.dx = px - geo.x;
  t.bdx = geo.w * t.dx;
  t.adx2 = (geo.z * t.dx) * t.dx;
  return t;
}

// Without a branch: the return value says whether the splat is kept
// (power <= 0 and alpha >= 1/255); alpha = min(0.99, o G), raw = o G,
// G = 2^power.  With CLAMP, G is clamped to [0, 1] (equal to 2^min(power, 0)),
// which changes nothing where the splat is kept and keeps every output finite
// for every pixel (for a caller that multiplies G into zeros); without it a
// pixel that skips the splat may see G > 1.
template <bool CLAMP>
__device__ __forceinline__ bool eval_alpha_at(const ColumnTerms& ct, const float4& geo,
                                              const float4& app, float py, float& alpha,
                                              float& raw, float& G, float& dy) {
  dy = py - geo.y;
  const float p2 = __builtin_fmaf(dy, __builtin_fmaf(app.x, dy, ct.bdx), ct.adx2);
  // the clamp is an output modifier of the exp (no extra instruction)
  G = CLAMP ? __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(p2), 0.0f, 1.0f)
            : __builtin_amdgcn_exp2f(p2);
  raw = app.y * G;
  alpha = fminf(kAlphaMax, raw);
  return p2 <= 0.0f && alpha >= kAlphaMin;
}

// Tile scheduling of the compositing kernels.  With one workgroup per tile
// the workgroup's slot is its block index; with persistent workgroups each
// draws slots from a counter until they run out.  Slot i names tile order[i]
// (longest lists first) or tile i when there is no order.
//
// next_slot: the whole workgroup's next slot (>= n_slots: none left).  The
// slots are dealt to kq = min(GS_QUEUE_COUNTERS, gridDim.x) queues, slot
// q + kq t to queue q, and workgroup b draws from queue b % kq (the
// dispatcher places consecutive workgroups on different XCDs, so each XCD
// drains one queue, and the draws of a launch spread over several counters,
// each in its own 128-byte line, instead of queueing on one address).  A
// queue's counter is its next t.  Every workgroup of a queue draws until it
// gets one past the queue's end, so queue q sees exactly (its slots + its
// workgroups) draws; the workgroup holding the last one sets the counter
// back to zero, ready for the next launch.  The draw reaches the other waves
// and lanes through LDS between two barriers, also with one wavefront per
// workgroup: a wave-level broadcast of lane 0's draw instead lets the
// compiler have lanes leave the slot loop separately, and the remaining
// lanes then broadcast a value they never drew.
__device__ __forceinline__ uint32_t next_slot(uint32_t* counters, uint32_t n_slots,
                                              uint32_t* s_slot) {
  const uint32_t kq = min((uint32_t)GS_QUEUE_COUNTERS, gridDim.x);
  const uint32_t q = blockIdx.x % kq;
  __syncthreads();   // every wave has read the previous slot
  if (threadIdx.x == 0) {
    const uint32_t n_q = (n_slots + kq - 1 - q) / kq;      // slots q, q + kq, ...
    const uint32_t g_q = (gridDim.x + kq - 1 - q) / kq;    // workgroups b = q mod kq
    uint32_t* c = counters + GS_QUEUE_STRIDE * q;
    const uint32_t t = atomicAdd(c, 1u);
    if (t == n_q + g_q - 1) atomicExch(c, 0u);
    *s_slot = t < n_q ? q + kq * t : n_slots;
  }
  __syncthreads();
  return *s_slot;
}

// Schedule of one compositing launch, from a GS_SCHEDULE_* tuning value:
// the tile order to follow (NULL: tile id order), the queue counter
// (non-NULL only for persistent workgroups) and the grid size.
struct TileSchedule {
  const uint32_t* order;
  uint32_t* counter;
  unsigned grid;
};
// resident: workgroups of the kernel that fit on the device at once
TileSchedule tile_schedule(int schedule, const gs_bins& bins, int call, int n_tiles,
                           int resident);
// Workgroups of `kernel` (block threads each, no dynamic LDS) that the
// current device holds at once; 0 on error.
int resident_workgroups(const void* kernel, int block);

// Process-wide tuning values (see gs_set_tuning); always a supported value.
int tuning(int key);

// Splats per thread and LDS batch from a GS_TUNE_*_STAGE value (0: the
// kernel's default).
inline int stage_per_thread(int value, int fallback) { return value == 0 ? fallback : value; }

// Optional per-kernel timing events (see gs_set_kernel_events).
void kernel_event_start(int kernel, hipStream_t s);
void kernel_event_stop(int kernel, hipStream_t s);

// Error reporting (thread-local buffer behind gs_last_error()).
void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// ---- kernel launchers (host functions, one per .hip translation unit) -----

hipError_t launch_preprocess(const gs_gaussians& g, const gs_camera* cams_dev, int n_views,
                             const gs_projected& out, hipStream_t s);

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);

struct BinSortPlan {
  int64_t n_entries;     // V * n
  int64_t capacity;
  int64_t chunks;        // binning workgroups per view
  int32_t n_tiles;
  int32_t lds_tiles;     // LDS histogram bins (largest view, at most the LDS limit)
  int32_t max_view_tiles;
  // workspace layout (byte offsets)
  size_t off_matrix, off_list, off_ids, off_list_count, off_counts, off_starts, off_long, off_flag, off_partial, off_order,
      off_staged, off_spare, total;
};
BinSortPlan make_bin_sort_plan(int64_t n, const ViewTable& vt, int64_t capacity);
int run_bin_sort(const gs_projected& p, int64_t n, const ViewTable& vt, const gs_bins& bins,
                 uint32_t* n_keys_host, char* ws, const BinSortPlan& plan, hipStream_t s);

// target == nullptr: plain compositing; otherwise also the L1 gradient into
// dL, per-tile loss shares into tile_loss and (loss != nullptr) their sum.
hipError_t launch_render_fwd(const gs_projected& p, const gs_bins& bins, const ViewTable& vt,
                             float3 bg, float* image, float* final_T, uint32_t* n_contrib,
                             float* depth, const float* target, float* dL, double* loss,
                             float* tile_loss, hipStream_t s);

// Device address of gs_render_fwd_l1_noalloc's static per-tile scratch on the
// current device (taken with hipGetSymbolAddress on first use per device).
hipError_t noalloc_scratch(float** out);

struct BwdPlan {
  size_t off_grad2d, off_pose, total;
};
BwdPlan make_bwd_plan(int64_t n, const ViewTable& vt);
hipError_t launch_render_bwd(const gs_gaussians& g, const gs_projected& p, const gs_bins& bins,
                             const gs_camera* cams_dev, const ViewTable& vt, float3 bg,
                             const float* dL_dimage, const float* final_T,
                             const uint32_t* n_contrib, const gs_grads& grads, uint32_t flags,
                             char* ws, const BwdPlan& plan, hipStream_t s);

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float beta1, float beta2, float eps, int32_t step, const uint8_t* mask,
                       hipStream_t s);

// gauss_mask (optional): per-Gaussian update mask over groups laid out
// [C][n_gauss] (element e belongs to Gaussian e % n_gauss).
hipError_t launch_adam_groups(const gs_adam_group* groups, int n_groups, float beta1,
                              float beta2, float eps, int32_t* step_dev,
                              const uint32_t* guard_n_keys, int64_t guard_capacity,
                              hipStream_t s, const uint8_t* gauss_mask = nullptr,
                              int64_t n_gauss = 0);
hipError_t launch_adam_dev(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                           float beta1, float beta2, float eps, int32_t* step_dev, int32_t commit,
                           const uint8_t* mask, const uint32_t* guard_n_keys,
                           int64_t guard_capacity, hipStream_t s);

hipError_t launch_render_error(const gs_projected& p, int64_t n, const gs_bins& bins,
                               const ViewTable& vt, const float* image, const float* target,
                               const uint32_t* n_contrib, float* err, hipStream_t s);
hipError_t launch_active_set(const float* err, int64_t n, int n_views, float eps,
                             const uint8_t* always, uint8_t* mask, float* err_max,
                             uint32_t* n_active, hipStream_t s);

hipError_t launch_concat(const gs_concat_array* arrays, int n_arrays, int64_t na, int64_t nb,
                         hipStream_t s);
hipError_t launch_prune_mask(const float* ologit, int64_t n, float min_logit, uint8_t* keep,
                             hipStream_t s);
size_t compact_ws_bytes(int64_t n);
hipError_t launch_compact(const gs_compact_array* arrays, int n_arrays, int64_t n,
                          const uint8_t* keep, uint32_t* n_kept, void* ws, hipStream_t s);
hipError_t launch_pose_adam(gs_camera* cams_dev, const float* grad_xi, float* m, float* v,
                            int n_views, const uint8_t* view_mask, float lr_trans, float lr_rot,
                            float beta1, float beta2, float eps, int32_t* step_dev,
                            hipStream_t s);
hipError_t launch_iso_loss_grad(const float* log_scales, int64_t n, float weight,
                                float* grad_log_scales, double* loss, hipStream_t s);

hipError_t launch_l1_loss_grad(const float* image, const float* target, const ViewTable& vt,
                               float* dL_dimage, double* loss, hipStream_t s);

// ---- learned / plain initialiser (nn.hip, costvol.hip) --------------------

hipError_t nn_conv3x3(const gs_act* x1, const gs_act* x2, const gs_act* mask, const void* w,
                      int cout, const float* bias, int relu, gs_act* y, float* yf, int yf_stride,
                      hipStream_t s);
hipError_t nn_conv3x3_wgrad(const gs_act* x1, const gs_act* x2, const gs_act* dz,
                            const gs_act* mask, float* dw, float* dbias, hipStream_t s);
hipError_t nn_flip_weights(const void* w, int cout, int cin, void* wt, hipStream_t s);
hipError_t nn_avgpool2(const gs_act* x, gs_act* y, hipStream_t s);
hipError_t nn_avgpool2_bwd(const gs_act* dy, const gs_act* add, gs_act* dx, int accumulate,
                           hipStream_t s);
hipError_t nn_upsample2(const gs_act* x, gs_act* y, hipStream_t s);
hipError_t nn_upsample2_bwd(const gs_act* dy, gs_act* dx, hipStream_t s);
hipError_t nn_rgb_to_nhwc(const float* rgb, gs_act* x, hipStream_t s);
hipError_t nn_f32_to_bf16(const float* src, void* dst, int64_t n, hipStream_t s);
hipError_t nn_head(const gs_act* f, const float* w, const float* b, float* out, hipStream_t s);
hipError_t nn_head_bwd(const gs_act* f, const float* w, const float* dout, gs_act* df, float* dw,
                       float* db, hipStream_t s);
hipError_t nn_depth_loss(const float* pred, const float* depth, int N, int H, int W, float fx,
                         float* dpred, double* loss, int* count_ws, hipStream_t s);
size_t cost_volume_ws_bytes(int K, int H, int W);
size_t bp_ws_bytes(int h, int w);
hipError_t launch_bp(const float* cost, int h, int w, float lam, float trunc, int iters,
                     float invalid, int32_t* labels, float* depth, void* ws, hipStream_t s);
hipError_t launch_cost_volume(const float* keyframes, int K, int H, int W,
                              const gs_camera* cams_dev, float* cost, float* depth, void* ws,
                              hipStream_t s);

}  // namespace gsmi
