// gs_render_error and gs_active_set: the per-Gaussian rendering error of the
// global stage's active-set selection (Sec. III-B2) and its thresholding.
//
// The error of splat g in view k sums, over the pixels g blends into, its
// blending weight w = alpha T times the pixel's L1 colour residual between
// the render and the view's reference image.  The walk is the forward's:
// one workgroup per 16x16 tile, the tile's sorted splats staged 64 at a time
// in LDS with their quadrant reach masks, every pixel walking its list front
// to back.  A pixel blends
// exactly the splats at list positions below its n_contrib that pass the
// alpha test (the forward stopped after its last blended splat), and its
// transmittance is updated with the forward's own float32 operations, so
// every weight equals the forward's bit for bit.  One wavefront covers the
// tile (four pixels per lane, one in each quadrant, as the forward at four
// pixels per lane); per splat, the lane's w * residual products are summed
// over the wavefront with DPP and added to the splat's error by one lane.
#include "gs_internal.h"

namespace gsmi {

namespace {

constexpr int kStage = 64;   // splats staged per batch: one per lane
constexpr int kPPL = 4;      // pixels per lane: one wavefront covers the tile

template <bool Q>
__global__ __launch_bounds__(64) void render_error_kernel(
    ViewTable vt, const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ values,
    const uint32_t* __restrict__ order, const float2* __restrict__ xy,
    const float4* __restrict__ co, const float4* __restrict__ rd, const float* __restrict__ image,
    const float* __restrict__ target, const uint32_t* __restrict__ n_contrib,
    float* __restrict__ err, uint32_t* __restrict__ counter) {
  __shared__ StagedSplat s_splat[kStage];
  __shared__ uint64_t s_reach[4];   // bit b of [q]: staged splat b reaches quadrant q
  __shared__ uint32_t s_slot;
  // slot i: tile order[i] (longest lists first) when the binning produced
  // an order; one slot per workgroup, or (Q) slots drawn from `counter`
  for (uint32_t slot = blockIdx.x;;) {
    if constexpr (Q) slot = next_slot(counter, (uint32_t)vt.n_tiles, &s_slot);
    if (slot >= (uint32_t)vt.n_tiles) break;
    const int tile = order ? (int)order[slot] : (int)slot;
    const int v = find_view(vt, tile);
    const ViewInfo& vi = vt.v[v];
    const int lt = tile - vi.tile_base;
    const int tx = lt % vi.tiles_x, ty = lt / vi.tiles_x;
    const int lane = threadIdx.x;
    // pixel k of the lane: quadrant k (8 x 8 pixels each), the forward's
    // assignment at four pixels per lane, so even and odd k share a column
    constexpr int NC = 2;
    float fpx[kPPL], fpy[kPPL], T[kPPL], resid[kPPL];
    uint32_t last[kPPL], wl = 0;
    const int64_t plane = (int64_t)vi.width * vi.height;
#pragma unroll
    for (int k = 0; k < kPPL; ++k) {
      const int i = k * 64 + lane;
      const int q = i >> 6, l = i & 63;
      const int px = tx * kTile + (q & 1) * 8 + (l & 7);
      const int py = ty * kTile + (q >> 1) * 8 + (l >> 3);
      fpx[k] = (float)px + 0.5f;
      fpy[k] = (float)py + 0.5f;
      T[k] = 1.0f;
      resid[k] = 0.0f;   // L1 colour residual of the pixel
      last[k] = 0;
      if (px < vi.width && py < vi.height) {
        const int64_t off = (int64_t)py * vi.width + px;
        const int64_t o = 3 * vi.pix_base + off;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
          resid[k] += fabsf(image[o + ch * plane] - target[o + ch * plane]);
        last[k] = n_contrib[vi.pix_base + off];
      }
      wl = max(wl, last[k]);
    }
    // positions the wave walks: below the largest n_contrib of its pixels
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) wl = max(wl, (uint32_t)__shfl_xor((int)wl, d, 64));
    const uint32_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
    // n_contrib never exceeds the list length for a matching forward; the
    // clamp keeps every list read inside [s, e) regardless
    const int64_t list_len = (int64_t)e - (int64_t)s;
    const int64_t wave_last = min((int64_t)__builtin_amdgcn_readfirstlane(wl), max(list_len, (int64_t)0));
    for (int64_t b = 0; b < wave_last; b += kStage) {
      __syncthreads();   // the previous batch's records have been read
      const int64_t k = b + lane;
      uint32_t reach = 0;
      if (k < wave_last)
        reach = stage_splat(values[s + (uint32_t)k], xy, co, rd, tx * kTile, ty * kTile, vi.width,
                            vi.height, s_splat[lane]);
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const uint64_t bq = __ballot((reach >> qq) & 1u);
        if (lane == 0) s_reach[qq] = bq;
      }
      __syncthreads();
      // splats that reach one of the quadrants, at positions below wave_last
      uint64_t m = uniform_u64(s_reach[0] | s_reach[1] | s_reach[2] | s_reach[3]);
      const int64_t lim = wave_last - b;
      if (lim < 64) m &= (uint64_t(1) << lim) - 1;
      while (m) {
        const int j = __builtin_ctzll(m);
        m &= m - 1;
        const uint32_t pos = (uint32_t)(b + j);
        const float4 geo = s_splat[j].geo;
        const float4 app = s_splat[j].app;
        const uint32_t sreach = __builtin_amdgcn_readfirstlane(__float_as_uint(s_splat[j].ext.y));
        ColumnTerms ct[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) ct[c] = column_terms(geo, fpx[c]);
        float part = 0.0f;
#pragma unroll
        for (int kk = 0; kk < kPPL; ++kk) {
          if (!(sreach & (1u << kk))) continue;   // quadrant kk: wave-uniform
          float alpha, raw, G, dy;
          const bool ok =
              eval_alpha_at<false>(ct[kk % NC], geo, app, fpy[kk], alpha, raw, G, dy) && pos < last[kk];
          if (ok) {
            part += (alpha * T[kk]) * resid[kk];
            T[kk] = __builtin_fmaf(-T[kk], alpha, T[kk]);   // as the forward computes it
          }
        }
        if (!__ballot(part != 0.0f)) continue;
        const float tot = wave_sum_to_lane63(part);
        if (lane == 63) {
          const uint32_t acc = __float_as_uint(s_splat[j].ext.w);
          unsafeAtomicAdd(err + acc, tot);
        }
      }
    }
    if constexpr (!Q) break;
  }
}

__global__ __launch_bounds__(256) void fill_f32_kernel(float* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// One lane per Gaussian: the largest error over the views, compared with eps.
__global__ __launch_bounds__(256) void active_set_kernel(
    const float* __restrict__ err, int64_t n, int n_views, float eps,
    const uint8_t* __restrict__ always, uint8_t* __restrict__ mask, float* __restrict__ err_max,
    uint32_t* __restrict__ n_active) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool on = false;
  if (i < n) {
    float mx = err[i];
    for (int v = 1; v < n_views; ++v) mx = fmaxf(mx, err[(int64_t)v * n + i]);
    on = mx > eps || (always && always[i] != 0);
    mask[i] = on ? 1 : 0;
    if (err_max) err_max[i] = mx;
  }
  if (n_active) {
    const uint64_t b = __ballot(on);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(n_active, (uint32_t)__popcll(b));
  }
}

__global__ void zero_u32_kernel(uint32_t* p) { *p = 0u; }

}  // namespace

hipError_t launch_render_error(const gs_projected& p, int64_t n, const gs_bins& bins,
                               const ViewTable& vt, const float* image, const float* target,
                               const uint32_t* n_contrib, float* err, hipStream_t s) {
  const int64_t entries = n * (int64_t)vt.n_views;
  if (entries > 0)
    hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, s,
                       err, entries);
  if (vt.n_tiles > 0 && n > 0) {
    // the backward's schedule: the same reverse walk over the same lists
    const int sched = tuning(GS_TUNE_BWD_SCHEDULE);
    const int resident = sched >= GS_SCHEDULE_PERSISTENT
                             ? resident_workgroups((const void*)render_error_kernel<true>, 64)
                             : 0;
    const TileSchedule sc = tile_schedule(sched, bins, GS_QUEUE_ERROR, vt.n_tiles, resident);
    const auto* xy = reinterpret_cast<const float2*>(p.xy);
    const auto* co = reinterpret_cast<const float4*>(p.conic_opacity);
    const auto* rd = reinterpret_cast<const float4*>(p.rgb_depth);
    if (sc.counter)
      hipLaunchKernelGGL(render_error_kernel<true>, dim3(sc.grid), dim3(64), 0, s, vt,
                         bins.ranges, bins.values, sc.order, xy, co, rd, image, target,
                         n_contrib, err, sc.counter);
    else
      hipLaunchKernelGGL(render_error_kernel<false>, dim3(sc.grid), dim3(64), 0, s, vt,
                         bins.ranges, bins.values, sc.order, xy, co, rd, image, target,
                         n_contrib, err, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_active_set(const float* err, int64_t n, int n_views, float eps,
                             const uint8_t* always, uint8_t* mask, float* err_max,
                             uint32_t* n_active, hipStream_t s) {
  if (n_active) hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, s, n_active);
  if (n > 0)
    hipLaunchKernelGGL(active_set_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, err,
                       n, n_views, eps, always, mask, err_max, n_active);
  return hipGetLastError();
}

}  // namespace gsmi
