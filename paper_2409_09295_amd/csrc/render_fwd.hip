// gs_render_fwd: front-to-back compositing, one 256-thread workgroup per
// 16x16 tile of any view in the batch (one grid over all views).
//
// Each wavefront owns an 8x8 quadrant of the tile (lane -> pixel).  The
// workgroup stages the tile's sorted splats in LDS 256 at a time (one
// gathered record per thread), then every lane walks the batch; records are
// read as LDS broadcasts.  A workgroup stops fetching batches once every
// pixel has terminated.
#include "gs_internal.h"

namespace gsmi {

namespace {

__device__ __forceinline__ void stage_splat(uint32_t g, const float2* __restrict__ xy,
                                            const float4* __restrict__ co,
                                            const float4* __restrict__ rd, StagedSplat& out) {
  const float2 m = xy[g];
  const float4 c = co[g];
  const float4 r = rd[g];
  out.geo = make_float4(m.x, m.y, -0.5f * kLog2e * c.x, -kLog2e * c.y);
  out.app = make_float4(-0.5f * kLog2e * c.z, c.w, r.w, 0.0f);
  out.col = make_float4(r.x, r.y, r.z, __uint_as_float(g));
}

__global__ __launch_bounds__(kBlock) void render_fwd_kernel(
    ViewTable vt, const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ values,
    const float2* __restrict__ xy, const float4* __restrict__ co, const float4* __restrict__ rd,
    float3 bg, float* __restrict__ image, float* __restrict__ final_T,
    uint32_t* __restrict__ n_contrib, float* __restrict__ depth_out) {
  __shared__ StagedSplat s_splat[kBlock];
  const int tile = blockIdx.x;
  const int v = find_view(vt, tile);
  const ViewInfo& vi = vt.v[v];
  const int lt = tile - vi.tile_base;
  const int tx = lt % vi.tiles_x, ty = lt / vi.tiles_x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int px = tx * kTile + (w & 1) * 8 + (lane & 7);
  const int py = ty * kTile + (w >> 1) * 8 + (lane >> 3);
  const bool inside = px < vi.width && py < vi.height;
  const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;

  const uint32_t s = ranges[2 * tile], e = ranges[2 * tile + 1];
  bool done = !inside;
  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f;
  uint32_t last = 0;
  for (int64_t b = s; b < (int64_t)e; b += kBlock) {
    if (__syncthreads_count(done ? 0 : 1) == 0) break;
    const int64_t idx = b + threadIdx.x;
    if (idx < (int64_t)e) stage_splat(values[idx], xy, co, rd, s_splat[threadIdx.x]);
    __syncthreads();
    const int cnt = (int)min((int64_t)kBlock, (int64_t)e - b);
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        const float4 geo = s_splat[j].geo;
        const float4 app = s_splat[j].app;
        float alpha, raw, G, dx, dy;
        if (!eval_alpha(geo, app, fpx, fpy, alpha, raw, G, dx, dy)) continue;
        const float Tn = T * (1.0f - alpha);
        if (Tn < kTMin) {
          done = true;
          break;
        }
        const float4 col = s_splat[j].col;
        const float wgt = alpha * T;
        C0 += col.x * wgt;
        C1 += col.y * wgt;
        C2 += col.z * wgt;
        D += app.z * wgt;
        T = Tn;
        last = (uint32_t)(b - (int64_t)s) + (uint32_t)j + 1;
      }
    }
  }
  if (inside) {
    const int64_t pix = vi.pix_base + (int64_t)py * vi.width + px;
    const int64_t plane = (int64_t)vi.width * vi.height;
    float* img = image + 3 * vi.pix_base;
    const int64_t off = (int64_t)py * vi.width + px;
    img[off] = C0 + T * bg.x;
    img[plane + off] = C1 + T * bg.y;
    img[2 * plane + off] = C2 + T * bg.z;
    final_T[pix] = T;
    n_contrib[pix] = last;
    if (depth_out) depth_out[pix] = D;
  }
}

}  // namespace

hipError_t launch_render_fwd(const gs_projected& p, const gs_bins& bins, const ViewTable& vt,
                             float3 bg, float* image, float* final_T, uint32_t* n_contrib,
                             float* depth, hipStream_t s) {
  if (vt.n_tiles == 0) return hipSuccess;
  kernel_event_start(GS_KERNEL_RENDER_FWD, s);
  hipLaunchKernelGGL(render_fwd_kernel, dim3((unsigned)vt.n_tiles), dim3(kBlock), 0, s, vt,
                     bins.ranges, bins.values, reinterpret_cast<const float2*>(p.xy),
                     reinterpret_cast<const float4*>(p.conic_opacity),
                     reinterpret_cast<const float4*>(p.rgb_depth), bg, image, final_T, n_contrib,
                     depth);
  kernel_event_stop(GS_KERNEL_RENDER_FWD, s);
  return hipGetLastError();
}

}  // namespace gsmi
